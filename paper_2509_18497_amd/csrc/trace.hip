// Ray casting through the surfel LBVH with alpha compositing.
//
// k_ff_trace      one workgroup per receiver surfel, one thread per ray:
//                 multi-round k-buffer traversal (the KB nearest hits beyond
//                 the last composited key per round, keys (t, j)), front-to-
//                 back compositing, every composited hit recorded per ray.
// k_ff_aggregate  one workgroup per receiver: replays the records, LDS hash
//                 table with 2^-40 fixed-point sums (integer adds are order
//                 independent, so F is bit-deterministic), radix select of
//                 the top-k entries, bitonic sort by column, one ELL row.
// k_direct        one thread per (surfel, light): shadow-ray transmittance.
// k_opacity_bwd   compositing backward, two recomputing passes.
#include <functional>

#include "gsrad_internal.h"
#include "sh_api.h"
#include "sh_basis.h"
#include "trace_api.h"

namespace gsrad {

namespace {

// Traversal stack entries per lane (LDS).  The form-factor trace first runs
// with the shallow stack (it keeps three workgroups per CU resident); a
// tree deep enough to overflow it is traced again with the deep one, which
// covers any LBVH of 30-bit Morton codes plus 32 index bits.
constexpr int kStackShallow = 32;
constexpr int kStackDeep = 64;
constexpr int kKB = 20;   // k-buffer entries per traversal round (measured best of 8-32)
constexpr uint32_t kEmpty = 0xffffffffu;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of receivers so its L2 sees one region of the scene.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t g) {
    const int64_t x = b & 7, q = b >> 3, per = g >> 3, rem = g & 7;
    return x * per + (x < rem ? x : rem) + q;
}

// Keys (t bits, j) of the k-buffer.  t > 0 is a finite FP32 value, so the
// 64-bit key has a clear sign bit and an exponent field below all ones: read
// as an FP64 number it is a positive finite double, and positive finite
// doubles order exactly as their bit patterns.  The sorted insertion then
// takes one FP64 min and one max per entry instead of a 64-bit compare and
// four selects.  The empty entry is the largest finite double.
constexpr uint64_t kKeyEmpty = 0x7fefffffffffffffull;

__device__ __forceinline__ uint64_t key_bits(double k) { return (uint64_t)__double_as_longlong(k); }

// One step of the insertion: (a, x) <- (min(a, x), max(a, x)).  Written as
// the two VALU instructions: keys are never NaN, so the input quieting the
// compiler would add before an IEEE min/max is not needed.
__device__ __forceinline__ void key_insert_step(double &a, double &x) {
    double hi;
    asm volatile("v_max_f64 %1, %0, %2\n\tv_min_f64 %0, %0, %2" : "+v"(a), "=&v"(hi) : "v"(x));
    x = hi;
}

// Leaf visit of the sorted traversal: FP32 hit decision, then insertion
// into the ascending k-buffer of keys (t bits, j).  The kernel value and
// the face of a hit are found only for the hits that end up buffered.
template <int KB>
__device__ __forceinline__ void visit_leaf(const SurfRec *__restrict__ rec, int s, uint32_t self, float ox, float oy,
                                           float oz, float dx, float dy, float dz, float t_eps, uint64_t last,
                                           double (&key)[KB], int &found, float &t1) {
    const SurfRec r = rec[s];
    // all four 16-byte parts of the record are requested together: left to
    // itself the compiler loads the part holding j first and the rest only
    // after the self test, a second memory latency per leaf
    asm volatile("" : : "v"(r.a.x), "v"(r.b.x), "v"(r.c.x), "v"(r.d.w));
    const uint32_t j = __float_as_uint(r.d.w);
    if (j == self) return;
    float t, r2;
    bool front;
    if (!hit_test(r, ox, oy, oz, dx, dy, dz, t_eps, 0.0f, false, t, r2, front)) return;
    const uint64_t kk = ((uint64_t)__float_as_uint(t) << 32) | (uint64_t)j;
    if (kk <= last) return;
    ++found;
    if (kk >= key_bits(key[KB - 1])) return;
    double x = __longlong_as_double((long long)kk);
#pragma unroll
    for (int k = 0; k < KB; ++k) key_insert_step(key[k], x);
    if (found >= KB) t1 = __uint_as_float((uint32_t)(key_bits(key[KB - 1]) >> 32)) * 1.00001f + 1e-30f;
}

// All hits of one ray in (t, j) order, composited front to back until the
// transmittance drops below t_min; on_hit(j, alpha, T_before, front, gamma)
// is called for every composited hit (plus its depth t).  Returns the final
// transmittance.
template <int KB, int STK = kStackDeep, typename OnHit>
__device__ __forceinline__ float trace_sorted(const BvhDev &bv, float ox, float oy, float oz, float dx, float dy,
                                              float dz, uint32_t self, float t_eps, float t_min,
                                              uint32_t *stack, int stride, int *err, OnHit &&on_hit) {
    const float ix = safe_inv(dx), iy = safe_inv(dy), iz = safe_inv(dz);
    uint64_t last = 0;
    float T = 1.0f;
    for (;;) {
        double key[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) key[k] = __longlong_as_double((long long)kKeyEmpty);
        int found = 0;
        const float tlo = last ? __uint_as_float((uint32_t)(last >> 32)) : t_eps;
        const float t0 = tlo * 0.99999f;
        float t1 = INFINITY;
        if (bv.n == 1) {
            visit_leaf<KB>(bv.rec, 0, self, ox, oy, oz, dx, dy, dz, t_eps, last, key, found, t1);
        } else {
            int sp = 0, node = 0;
            bool ovf = false;
            for (;;) {
                const Node nd = bv.nodes[node];
                float tn0, tn1;
                bool h0 = slab(nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y, ox, oy, oz, ix, iy, iz, t0, t1, tn0);
                bool h1 = slab(nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w, ox, oy, oz, ix, iy, iz, t0, t1, tn1);
                const int c0 = nd.ch.x, c1 = nd.ch.y;
                if (h0 && c0 < 0) {
                    visit_leaf<KB>(bv.rec, ~c0, self, ox, oy, oz, dx, dy, dz, t_eps, last, key, found, t1);
                    h0 = false;
                }
                if (h1 && c1 < 0) {
                    visit_leaf<KB>(bv.rec, ~c1, self, ox, oy, oz, dx, dy, dz, t_eps, last, key, found, t1);
                    h1 = false;
                }
                // descend into the nearer hit child and push the other; with
                // no child left, pop.  A push past the stack's end ends the
                // walk with an error (the caller traces again with the deep
                // stack).
                const bool both = h0 && h1;
                const bool n0 = !h1 || (h0 && tn0 <= tn1);
                ovf = both && sp >= STK;
                if (both) stack[min(sp, STK - 1) * stride] = (uint32_t)(n0 ? c1 : c0);
                sp += both ? 1 : 0;
                node = n0 ? c0 : c1;
                if (!h0 && !h1) {
                    if (sp == 0) break;
                    --sp;
                    node = (int)stack[sp * stride];
                }
                if (ovf) break;
            }
            if (ovf) {
                atomicOr(err, kErrStack);
                return T;
            }
        }
        const int m = found < KB ? found : KB;
        // kernel values (FP64 hit point) and faces of the buffered hits only
        float gam[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            gam[k] = 0.0f;
            if (k < m) {
                const SurfRec r = bv.rec[bv.inv[(uint32_t)key_bits(key[k])]];
                const float den = __builtin_fmaf(dz, r.b.z, __builtin_fmaf(dy, r.b.y, __fmul_rn(dx, r.b.x)));
                const float g = kernel_gamma(hit_r2_exact(r, ox, oy, oz, dx, dy, dz));
                gam[k] = den < 0.0f ? g : -g;
            }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if (k < m) {
                const uint32_t j = (uint32_t)key_bits(key[k]);
                const float g = fabsf(gam[k]);
                const bool front = gam[k] > 0.0f;
                const float x = __fmul_rn(bv.c[j], g);
                const float alpha = -expm1f(-x);
                on_hit(j, alpha, T, front, g, __uint_as_float((uint32_t)(key_bits(key[k]) >> 32)));
                T = __fmul_rn(T, exp_fx(-x));
                if (T < t_min) return T;
            }
        }
        // a full buffer pruned every box beyond its last entry, so more hits
        // may exist: only a buffer that did not fill ends the ray
        if (found < KB) return T;
        last = key_bits(key[KB - 1]);
    }
}

// Transmittance of the segment t in (t_lo, 1) of o + t d: product of
// (1 - alpha) over every surfel crossed (order-free).
__device__ __forceinline__ float trace_shadow(const BvhDev &bv, float ox, float oy, float oz, float dx, float dy,
                                              float dz, uint32_t self, float t_lo, uint32_t *stack, int stride,
                                              int *err) {
    const float ix = safe_inv(dx), iy = safe_inv(dy), iz = safe_inv(dz);
    const float t0 = t_lo * 0.99999f, t1 = 1.00001f;
    float T = 1.0f;
    auto leaf = [&](int s) {
        const SurfRec r = bv.rec[s];
        asm volatile("" : : "v"(r.a.x), "v"(r.b.x), "v"(r.c.x), "v"(r.d.w));   // whole record in one latency
        const uint32_t j = __float_as_uint(r.d.w);
        if (j == self) return;
        float t, r2;
        bool front;
        if (!hit_test(r, ox, oy, oz, dx, dy, dz, t_lo, 1.0f, true, t, r2, front)) return;
        // kernel value from the exact intersection (the FP32 hit point loses
        // the offset from the centre when the centre is many radii away)
        T = __fmul_rn(T, transmit(r.c.w, kernel_gamma(hit_r2_exact(r, ox, oy, oz, dx, dy, dz))));
    };
    if (bv.n == 1) {
        leaf(0);
        return T;
    }
    int sp = 0, node = 0;
    bool ovf = false;
    for (;;) {
        const Node nd = bv.nodes[node];
        float tn0, tn1;
        bool h0 = slab(nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y, ox, oy, oz, ix, iy, iz, t0, t1, tn0);
        bool h1 = slab(nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w, ox, oy, oz, ix, iy, iz, t0, t1, tn1);
        const int c0 = nd.ch.x, c1 = nd.ch.y;
        if (h0 && c0 < 0) {
            leaf(~c0);
            h0 = false;
        }
        if (h1 && c1 < 0) {
            leaf(~c1);
            h1 = false;
        }
        // descend (first child first), push the other; none left: pop.  A
        // push past the stack's end ends the walk with an error.
        const bool both = h0 && h1;
        ovf = both && sp >= kStackDeep;
        if (both) stack[min(sp, kStackDeep - 1) * stride] = (uint32_t)c1;
        sp += both ? 1 : 0;
        node = h0 ? c0 : c1;
        if (!h0 && !h1) {
            if (sp == 0) break;
            --sp;
            node = (int)stack[sp * stride];
        }
        if (ovf) break;
    }
    if (ovf) atomicOr(err, kErrStack);
    return T;
}

// ---------------------------------------------------------------------------
// form factors
// ---------------------------------------------------------------------------
// Octahedral 2 x 8-bit Morton key of a direction: rays with close keys
// leave in close directions.
__device__ __forceinline__ uint32_t dir_key(float dx, float dy, float dz) {
    const float l1 = fabsf(dx) + fabsf(dy) + fabsf(dz);
    float px = dx / l1, py = dy / l1;
    if (dz < 0.0f) {
        const float qx = (1.0f - fabsf(py)) * (px >= 0.0f ? 1.0f : -1.0f);
        const float qy = (1.0f - fabsf(px)) * (py >= 0.0f ? 1.0f : -1.0f);
        px = qx;
        py = qy;
    }
    const uint32_t ux = min(255u, (uint32_t)((px * 0.5f + 0.5f) * 256.0f));
    const uint32_t uy = min(255u, (uint32_t)((py * 0.5f + 0.5f) * 256.0f));
    uint32_t k = 0;
#pragma unroll
    for (int bt = 0; bt < 8; ++bt) k |= (((ux >> bt) & 1u) << (2 * bt)) | (((uy >> bt) & 1u) << (2 * bt + 1));
    return k;
}

constexpr int kPoolRays = 1024;   // rays sorted and pooled per batch

// Every composited hit of ray r of the receiver in slot `slot` is recorded
// as (j, +-gamma), the sign being the front face, at
// recs[(slot*rcap + q)*R + r] (hit-major inside a receiver, so a wave
// touches one record per lane with one coalesced access); rcnt[slot*R + r]
// is the number of composited hits (more than rcap: records incomplete).
// slot = original index i when the records of all receivers are kept,
// else the receiver's position in the current chunk.
//
// One workgroup traces the rays of `group` consecutive receivers (Morton
// order).  Per batch of up to 1024 rays the directions are generated, the
// rays sorted by direction key, and the lanes pull rays from the sorted
// pool through an LDS counter: neighbouring lanes trace rays that leave
// close origins in close directions, and a lane whose ray ends early takes
// the next one instead of idling until its wave's longest ray is done.
// Three waves per SIMD (at most 168 VGPRs), held by a launch bound; four
// (at most 128) were measured no faster.
template <int STK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) k_ff_trace(BvhDev bv, int R, uint64_t seed, float t_eps, float t_min,
                                                  int64_t s_begin, int64_t count, int group, int64_t nblocks,
                                                  int by_orig, uint2 *__restrict__ recs,
                                                  uint32_t *__restrict__ rcnt, int rcap, int *err) {
    extern __shared__ uint32_t stack_mem[];
    __shared__ uint32_t pool_key[kPoolRays];
    __shared__ float pool_d[kPoolRays][3];
    __shared__ uint32_t next;
    const int64_t gb = xcd_block(blockIdx.x, nblocks);
    const int tid = threadIdx.x;
    const int64_t r0 = gb * group;                                 // first receiver (chunk-relative)
    const int g = (int)min<int64_t>(group, count - r0);            // receivers in this group
    const int64_t total = (int64_t)g * R;
    for (int64_t base = 0; base < total; base += kPoolRays) {
        const int nb = (int)min<int64_t>(kPoolRays, total - base);
        int P = 1;
        while (P < nb) P <<= 1;
        for (int k = tid; k < P; k += blockDim.x) {
            uint32_t key = 0xffffffffu;
            if (k < nb) {
                const int64_t id = base + k;
                const SurfRec rr = bv.rec[s_begin + r0 + id / R];
                const int r = (int)(id % R);
                float dx, dy, dz;
                ray_direction(rr.c.x, rr.c.y, rr.c.z, rr.d.x, rr.d.y, rr.d.z, rr.b.x, rr.b.y, rr.b.z, (uint64_t)r,
                              (uint64_t)__float_as_uint(rr.d.w), seed, 0, dx, dy, dz);
                pool_d[k][0] = dx;
                pool_d[k][1] = dy;
                pool_d[k][2] = dz;
                key = (dir_key(dx, dy, dz) << 10) | (uint32_t)k;
            }
            pool_key[k] = key;
        }
        if (tid == 0) next = 0;
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = tid; t < P / 2; t += blockDim.x) {
                    const int idx = 2 * stride * (t / stride) + (t % stride);
                    const int par = idx + stride;
                    const bool asc = (idx & size) == 0;
                    const uint32_t x = pool_key[idx], y = pool_key[par];
                    if ((x > y) == asc) {
                        pool_key[idx] = y;
                        pool_key[par] = x;
                    }
                }
                __syncthreads();
            }
        }
        for (;;) {
            const uint32_t p = atomicAdd(&next, 1u);
            if (p >= (uint32_t)nb) break;
            const int k = (int)(pool_key[p] & 1023u);
            const int64_t id = base + k;
            const int64_t recv = r0 + id / R;                        // chunk-relative receiver
            const int r = (int)(id % R);
            const SurfRec rr = bv.rec[s_begin + recv];
            const uint32_t i = __float_as_uint(rr.d.w);
            const int64_t slot = by_orig ? (int64_t)i : recv;
            uint32_t q = 0;
            uint2 *rec_out = recs + slot * rcap * R + r;
            trace_sorted<kKB, STK>(bv, rr.a.x, rr.a.y, rr.a.z, pool_d[k][0], pool_d[k][1], pool_d[k][2], i, t_eps, t_min,
                              stack_mem + tid, blockDim.x, err, [&](uint32_t j, float, float, bool front, float gg, float) {
                                  if (q < (uint32_t)rcap)
                                      rec_out[(int64_t)q * R] = make_uint2(j, __float_as_uint(front ? gg : -gg));
                                  ++q;
                              });
            rcnt[slot * R + r] = q;
            if (q > (uint32_t)rcap) {
                atomicOr(err, kErrRecords);
                atomicMax(err + 3, (int)q);
            }
        }
        __syncthreads();
    }
}

// Slot of surfel j in an open-addressing table of 2^log2h entries.  A full
// avalanche mixer (the 32-bit finaliser of "lowbias32"), not a single
// golden-ratio multiply: surfels laid out on Fibonacci lattices have index
// differences that are Fibonacci numbers, which golden-ratio hashing sends
// to nearly the same slot.
__device__ __forceinline__ uint32_t hash_slot(uint32_t j, int log2h) {
    uint32_t h = j;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h >> (32 - log2h);
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ __forceinline__ uint64_t badness(uint32_t j, float v) {
    // ascending badness = value descending, then column ascending
    return ((uint64_t)(~__float_as_uint(v)) << 32) | (uint64_t)j;
}

// Block-wide exclusive scan of one count per thread (256 threads).
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan_u32(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

constexpr int kAggMaxPer = 32;   // table slots (or entries) per thread: H <= 8192

// One workgroup per receiver.  The rays' records are replayed with the same
// FP32 alpha/T sequence as the trace; front-hit weights are summed per
// sender in an LDS hash table in 2^-40 fixed point (integer adds commute, so
// the sums do not depend on the order of the atomics).  The distinct senders
// are compacted, the topk largest (value desc, column asc) kept by a radix
// select on the FP32 values, and the row sorted by column (bitonic).
//
// A row whose insertion probes max_probe slots (a table nearly full) is
// given up: with redo_list set its slot b is appended there (and counted in
// err[2]) for the REDO pass, which takes the listed rows one after the
// other (a ticket per row) with the largest table; without a list, or in
// the REDO pass, the row is an overflow.  Either table size gives the same
// row.
template <bool REDO>
__global__ void __launch_bounds__(256) k_ff_aggregate(BvhDev bv, const uint2 *__restrict__ recs,
                                                      const uint32_t *__restrict__ rcnt, int rcap, int64_t s_begin,
                                                      int by_orig, int R, int topk, int log2h, int max_probe,
                                                      int32_t *redo_list, uint32_t *redo_cnt, int64_t cap_row,
                                                      int32_t *__restrict__ ell_col, float *__restrict__ ell_val,
                                                      uint32_t *__restrict__ row_len, int *err) {
    extern __shared__ __align__(16) unsigned char sm[];
    const int H = 1 << log2h;
    unsigned long long *hval = reinterpret_cast<unsigned long long *>(sm);   // [H]
    uint32_t *hkey = reinterpret_cast<uint32_t *>(hval + H);                  // [H]
    // after compaction the same memory holds the entries: columns in the
    // key region, FP32 values in the first half of the value region
    uint32_t *cj = hkey;
    float *cv = reinterpret_cast<float *>(hval);
    __shared__ uint32_t hist[256], wsum[4], dsel, before_sh, habort, ticket;
    volatile uint32_t *abort_v = &habort;
    const int tid = threadIdx.x;
    for (;;) {
    int64_t b;
    if (REDO) {
        if (tid == 0) ticket = atomicAdd(redo_cnt + 1, 1u);
        __syncthreads();
        const uint32_t k = ticket;
        if (k >= redo_cnt[0]) break;
        b = redo_list[k];
    } else {
        b = blockIdx.x;
    }
    const uint32_t i = __float_as_uint(bv.rec[s_begin + b].d.w);
    const int64_t slot = by_orig ? (int64_t)i : b;
    for (int k = tid; k < H; k += 256) {
        hkey[k] = kEmpty;
        hval[k] = 0ull;
    }
    if (tid == 0) habort = 0;
    __syncthreads();
    for (int r = tid; r < R; r += 256) {
        const uint32_t m = min(rcnt[slot * R + r], (uint32_t)rcap);
        const uint2 *in = recs + slot * rcap * R + r;
        float T = 1.0f;
        // the record one step ahead and its sender's c, the record two
        // steps ahead: each load has a record's work to land
        uint2 h1 = m > 0 ? in[0] : make_uint2(0u, 0u);
        uint2 h2 = m > 1 ? in[(int64_t)R] : make_uint2(0u, 0u);
        float c1 = m > 0 ? bv.c[h1.x] : 0.0f;
        for (uint32_t q = 0; q < m; ++q) {
            if ((q & 7) == 0 && *abort_v) break;
            const uint2 h = h1;
            const float cq = c1;
            h1 = h2;
            if (q + 2 < m) h2 = in[(int64_t)(q + 2) * R];
            if (q + 1 < m) c1 = bv.c[h1.x];
            const float gs = __uint_as_float(h.y);
            const float x = cq * fabsf(gs);
            if (gs > 0.0f) {
                const float w = -expm1f(-x) * T;
                const unsigned long long fx = (unsigned long long)__float2ull_rn(w * kFixScaleF);
                uint32_t hs = hash_slot(h.x, log2h);
                int probe = 0;
                for (; probe < max_probe; ++probe) {
                    const uint32_t prev = atomicCAS(&hkey[hs], kEmpty, h.x);
                    if (prev == kEmpty || prev == h.x) {
                        atomicAdd(&hval[hs], fx);
                        break;
                    }
                    hs = (hs + 1) & (uint32_t)(H - 1);
                }
                if (probe == max_probe) *abort_v = 1;
            }
            T = __fmul_rn(T, exp_fx(-x));
        }
    }
    __syncthreads();
    if (habort) {
        if (tid == 0) {
            row_len[i] = 0;
            if (!REDO && redo_list) {
                redo_list[atomicAdd(redo_cnt, 1u)] = (int32_t)b;
                atomicAdd(err + 2, 1);
            } else {
                atomicOr(err, kErrTable);
            }
        }
        if (!REDO) return;
        __syncthreads();
        continue;
    }
    // compact the table in place: each thread stages its own slots
    const double scale = 1.0 / (kFixScale * (double)R);
    const int per = H >> 8;
    // staged by static index so the arrays stay in registers
    uint32_t sj[kAggMaxPer];
    float sv[kAggMaxPer];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kAggMaxPer; ++k) {
        sj[k] = kEmpty;
        sv[k] = 0.0f;
        if (k < per) {
            const int sl = tid * per + k;
            const uint32_t key = hkey[sl];
            if (key != kEmpty) {
                sj[k] = key;
                sv[k] = (float)((double)hval[sl] * scale);
                ++c;
            }
        }
    }
    uint32_t m;
    uint32_t pos = block_scan_u32(c, wsum, m);
#pragma unroll
    for (int k = 0; k < kAggMaxPer; ++k) {
        if (sj[k] != kEmpty) {
            cj[pos] = sj[k];
            cv[pos] = sv[k];
            ++pos;
        }
    }
    __syncthreads();
    if (topk > 0 && m > (uint32_t)topk) {
        // radix select of the topk-th smallest badness key, MSB first
        uint64_t prefix = 0, pmask = 0;
        uint32_t need = (uint32_t)topk;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            hist[tid] = 0;
            __syncthreads();
            for (uint32_t e = tid; e < m; e += 256) {
                const uint64_t key = badness(cj[e], cv[e]);
                if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid < 64) {
                uint32_t c4[4], s4 = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    c4[q] = hist[4 * tid + q];
                    s4 += c4[q];
                }
                uint32_t run = wave_incl_scan_u32(s4) - s4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (run < need && need <= run + c4[q]) {
                        dsel = (uint32_t)(4 * tid + q);
                        before_sh = run;
                    }
                    run += c4[q];
                }
            }
            __syncthreads();
            prefix |= (uint64_t)dsel << shift;
            pmask |= 255ull << shift;
            need -= before_sh;
            __syncthreads();
        }
        // keep badness <= prefix (exactly topk entries: keys are unique),
        // compacted in place through registers
        const uint32_t pe = (m + 255u) >> 8;
        uint32_t kc = 0;
#pragma unroll
        for (int k = 0; k < kAggMaxPer; ++k) {
            const uint32_t e = (uint32_t)tid * pe + (uint32_t)k;
            sj[k] = kEmpty;
            sv[k] = 0.0f;
            if ((uint32_t)k < pe && e < m) {
                const uint32_t jj = cj[e];
                const float vv = cv[e];
                if (badness(jj, vv) <= prefix) {
                    sj[k] = jj;
                    sv[k] = vv;
                    ++kc;
                }
            }
        }
        uint32_t kept;
        uint32_t kpos = block_scan_u32(kc, wsum, kept);
#pragma unroll
        for (int k = 0; k < kAggMaxPer; ++k) {
            if (sj[k] != kEmpty) {
                cj[kpos] = sj[k];
                cv[kpos] = sv[k];
                ++kpos;
            }
        }
        m = kept;
        __syncthreads();
    }
    // bitonic sort of the m entries by column
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t e = m + tid; e < P; e += 256) cj[e] = kEmpty;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = tid; t < P / 2; t += 256) {
                const uint32_t idx = 2 * stride * (t / stride) + (t % stride);
                const uint32_t par = idx + stride;
                const bool asc = (idx & size) == 0;
                const uint32_t a = cj[idx], cc = cj[par];
                if ((a > cc) == asc) {
                    cj[idx] = cc;
                    cj[par] = a;
                    const float va = cv[idx];
                    cv[idx] = cv[par];
                    cv[par] = va;
                }
            }
            __syncthreads();
        }
    }
    if (m > cap_row) {
        if (tid == 0) atomicOr(err, kErrRow);
        m = (uint32_t)cap_row;
    }
    for (uint32_t e = tid; e < m; e += 256) {
        ell_col[(int64_t)i * cap_row + e] = (int32_t)cj[e];
        ell_val[(int64_t)i * cap_row + e] = cv[e];
    }
    if (tid == 0) row_len[i] = m;
    if (!REDO) return;
    __syncthreads();   // the LDS is reused by the next listed row
    }
}

__global__ void __launch_bounds__(256) k_ell_to_csr(const int32_t *__restrict__ ell_col,
                                                    const float *__restrict__ ell_val, int64_t cap_row,
                                                    const int64_t *__restrict__ row_ptr, int64_t n,
                                                    int32_t *__restrict__ col, float *__restrict__ val) {
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (row >= n) return;
    const int64_t b = row_ptr[row], len = row_ptr[row + 1] - b;
    for (int64_t e = __lane_id(); e < len; e += 64) {
        col[b + e] = ell_col[row * cap_row + e];
        val[b + e] = ell_val[row * cap_row + e];
    }
}

// ---------------------------------------------------------------------------
// direct light
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128) k_direct(BvhDev bv, const float *__restrict__ albedo,
                                                const float *__restrict__ lpos, const float *__restrict__ lI, int Lt,
                                                int K, float *__restrict__ E, int *err) {
    extern __shared__ uint32_t stack_mem[];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= bv.n * Lt) return;
    const int64_t i = idx / Lt;
    const int l = (int)(idx - i * Lt);
    const SurfRec rr = bv.rec[bv.inv[i]];
    float *e = E + ((i * Lt + l) * K) * 3;
    const float dx = __fsub_rn(lpos[3 * l + 0], rr.a.x);
    const float dy = __fsub_rn(lpos[3 * l + 1], rr.a.y);
    const float dz = __fsub_rn(lpos[3 * l + 2], rr.a.z);
    const float dd = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __fmul_rn(dx, dx)));
    const float len = sqrt_rn(dd);
    const float ndot = rr.b.x * dx + rr.b.y * dy + rr.b.z * dz;
    float base = 0.0f;
    if (ndot > 0.0f && dd > 0.0f) {
        const float t_lo = __fdiv_rn(bv.bounds[6], len);
        const float T = trace_shadow(bv, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz, (uint32_t)i, t_lo,
                                     stack_mem + threadIdx.x, blockDim.x, err);
        base = bv.op[i] * 1.1283791670955126f * lI[l] * (ndot / len) / dd * T;
    }
    e[0] = base * albedo[3 * i + 0];
    e[1] = base * albedo[3 * i + 1];
    e[2] = base * albedo[3 * i + 2];
    for (int c = 3; c < 3 * K; ++c) e[c] = 0.0f;
}

// Direct light with the BRDF: E_i,l = (R_i / pi) (.) Y(w^(i)) I_l max(0, n_i . w) / r^2 T_il
// with w the unit direction to the light expressed in i's tangent frame.
template <int K>
__global__ void __launch_bounds__(128) k_direct_sh(BvhDev bv, const float *__restrict__ R,
                                                   const float *__restrict__ lpos, const float *__restrict__ lI, int Lt,
                                                   float *__restrict__ E, int *err) {
    extern __shared__ uint32_t stack_mem[];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= bv.n * Lt) return;
    const int64_t i = idx / Lt;
    const int l = (int)(idx - i * Lt);
    const SurfRec rr = bv.rec[bv.inv[i]];
    float *e = E + ((i * Lt + l) * K) * 3;
    const float dx = __fsub_rn(lpos[3 * l + 0], rr.a.x);
    const float dy = __fsub_rn(lpos[3 * l + 1], rr.a.y);
    const float dz = __fsub_rn(lpos[3 * l + 2], rr.a.z);
    const float dd = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __fmul_rn(dx, dx)));
    const float len = sqrt_rn(dd);
    const float ndot = rr.b.x * dx + rr.b.y * dy + rr.b.z * dz;
    float base = 0.0f;
    float Y[K];
    if (ndot > 0.0f && dd > 0.0f) {
        const float t_lo = __fdiv_rn(bv.bounds[6], len);
        const float T = trace_shadow(bv, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz, (uint32_t)i, t_lo,
                                     stack_mem + threadIdx.x, blockDim.x, err);
        base = lI[l] * (ndot / len) / dd * T * 0.318309886183791f;
        const float il = 1.0f / len;
        sh_eval<K>((dx * rr.c.x + dy * rr.c.y + dz * rr.c.z) * il, (dx * rr.d.x + dy * rr.d.y + dz * rr.d.z) * il,
                   ndot * il, Y);
    } else {
#pragma unroll
        for (int a = 0; a < K; ++a) Y[a] = 0.0f;
    }
    const float *Ri = R + i * K * 3;
#pragma unroll
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < 3; ++c) e[3 * a + c] = Ri[3 * a + c] * Y[a] * base;
}

// ---------------------------------------------------------------------------
// opacity backward (compositing backward, recomputing the hits)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float row_lookup(const uint32_t *lc, const float *lg, int len, uint32_t j) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lc[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < len && lc[lo] == j) ? lg[lo] : 0.0f;
}

// For one ray with composited hits q = 1..m (alpha_q, transmittance T_q in
// front of the hit, kernel value g_q) and G_q = dL/dF[i, j_q] / R on front
// hits kept in F (0 otherwise), the F-part of the loss is
// sum_q G_q alpha_q T_q, so
//   dL/dalpha_q = G_q T_q - S_q / (1 - alpha_q),  S_q = sum_{p>q} G_p alpha_p T_p
//   dalpha_q/do = g_q (1 - o)^(g_q - 1) = g_q e^(c (1 - g_q)).
// S_q = W - P_q (W the ray's total, P_q the running sum through q) is formed
// in double-float arithmetic (pairs of FP32 with error-free sums and
// products), so the difference keeps the digits that the division by
// 1 - alpha_q (down to 1e-4) magnifies; 1 - alpha_q is the transmit factor
// e^(-c g) the transmittance uses, not 1 minus the rounded alpha.
//
// The contributions are summed per sender in 64-bit fixed point: integer
// adds commute, so the gradient is bit-identical between runs whatever the
// order of the atomics.  The scale 2^e is a power of two chosen from
// max|dL/dF| so that no sum can leave the int64 range: a contribution is at
// most 2 max|G| max_g g e^(c(1-g)) <= 800 max|G| for c <= -ln(1e-4), and a
// sender is composited at most once per ray (k_fx_exp).  Each XCD adds into
// its own copy of the accumulators with atomics kept in its L2 (scope of
// the workgroup: every workgroup that touches copy x runs on XCD x), and
// k_opacity_finish adds the copies.
struct DF {
    float hi, lo;
};

__device__ __forceinline__ DF df_add(DF x, DF y) {
    const float s = x.hi + y.hi;
    const float bb = s - x.hi;
    const float e = ((x.hi - (s - bb)) + (y.hi - bb)) + (x.lo + y.lo);
    const float hi = s + e;
    return {hi, e - (hi - s)};
}

// G * alpha * T as an unevaluated pair (relative error about 2^-46)
__device__ __forceinline__ DF df_prod3(float G, float a, float T) {
    const float p = a * T;
    const float pe = __builtin_fmaf(a, T, -p);
    const float h = G * p;
    return {h, __builtin_fmaf(G, p, -h) + G * pe};
}

__device__ __forceinline__ int xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7;   // HW_REG_XCC_ID
}

__device__ __forceinline__ void fx_add(unsigned long long *acc, float v, float scale) {
    const long long q = __float2ll_rn(v * scale);
    if (q != 0)
        __hip_atomic_fetch_add(acc, (unsigned long long)q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One hit of the second walk: the sender's contribution to dL/do.
__device__ __forceinline__ void opacity_hit(const BvhDev &bv, uint32_t j, float G, float alpha, float f, float T,
                                            float g, DF W, DF &P, unsigned long long *acc, float scale) {
    if (G != 0.0f) P = df_add(P, df_prod3(G, alpha, T));
    const float oraw = bv.raw_op[j];
    if (!(oraw > 0.0f && oraw < kOpacityMax)) return;
    const DF Sd = df_add(W, DF{-P.hi, -P.lo});
    const float dLda = G * T - Sd.hi / f;
    const float dado = g * expf(bv.c[j] * (1.0f - g));
    fx_add(acc + j, dLda * dado, scale);
}

// max |dL/dF| as float bits (non-negative floats order like their bits)
__global__ void __launch_bounds__(256) k_absmax(const float *__restrict__ v, int64_t n, uint32_t *out) {
    uint32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = max(m, __float_as_uint(fabsf(v[i])));
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    if (__lane_id() == 0) atomicMax(out, m);
}

// exponent e of the fixed-point scale: 801 max|dL/dF| n < 2^(62 - e)
// (max|G| = max|dL/dF| / R, at most n R rays); kFxNonFinite marks a
// non-finite dL/dF (the gradient is then NaN)
constexpr int kFxNonFinite = 1 << 20;
__global__ void k_fx_exp(const uint32_t *maxbits, int64_t n, int *e_out) {
    const float m = __uint_as_float(*maxbits);
    int e = 0;
    if (!(m <= 3.0e38f)) {
        e = kFxNonFinite;
    } else if (m > 0.0f) {
        int ex;
        (void)frexpf(801.0f * m * (float)n, &ex);
        e = min(120, max(-120, 62 - ex));
    }
    *e_out = e;
}

__global__ void __launch_bounds__(256) k_opacity_bwd(BvhDev bv, int R, uint64_t seed, float t_eps, float t_min,
                                                     int64_t nblocks, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const float *__restrict__ gF,
                                                     int max_row, float2 *__restrict__ wbuf, const int *fx_exp,
                                                     unsigned long long *acc, int pass,
                                                     const uint32_t *__restrict__ rcnt, int rcap, int *err) {
    extern __shared__ uint32_t sm2[];
    uint32_t *lc = sm2;                                   // [max_row]
    float *lg = reinterpret_cast<float *>(lc + max_row);  // [max_row]
    uint32_t *stack_mem = reinterpret_cast<uint32_t *>(lg + max_row);
    const int64_t b = xcd_block(blockIdx.x, nblocks);
    const int tid = threadIdx.x;
    const SurfRec rr = bv.rec[b];
    const uint32_t i = __float_as_uint(rr.d.w);
    const int64_t e0 = row_ptr[i];
    const int len = (int)(row_ptr[i + 1] - e0);
    const float invR = 1.0f / (float)R;
    const float scale = __builtin_ldexpf(1.0f, *fx_exp);
    unsigned long long *my = acc + (int64_t)xcc_id() * bv.n;
    for (int k = tid; k < len; k += blockDim.x) {
        lc[k] = (uint32_t)col[e0 + k];
        lg[k] = gF[e0 + k] * invR;
    }
    __syncthreads();
    for (int r = tid; r < R; r += blockDim.x) {
        // with records, only rays whose records overflowed are recomputed here
        if (rcnt && rcnt[(int64_t)i * R + r] <= (uint32_t)rcap) continue;
        float dx, dy, dz;
        ray_direction(rr.c.x, rr.c.y, rr.c.z, rr.d.x, rr.d.y, rr.d.z, rr.b.x, rr.b.y, rr.b.z, (uint64_t)r,
                      (uint64_t)i, seed, 0, dx, dy, dz);
        if (pass == 0) {
            DF W{0.0f, 0.0f};
            trace_sorted<kKB>(bv, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz, i, t_eps, t_min, stack_mem + tid, blockDim.x,
                              err, [&](uint32_t j, float alpha, float T, bool front, float, float) {
                                  const float G = front ? row_lookup(lc, lg, len, j) : 0.0f;
                                  if (G != 0.0f) W = df_add(W, df_prod3(G, alpha, T));
                              });
            wbuf[(int64_t)i * R + r] = make_float2(W.hi, W.lo);
        } else {
            const float2 w2 = wbuf[(int64_t)i * R + r];
            const DF W{w2.x, w2.y};
            if (W.hi == 0.0f) continue;   // every G_q alpha_q T_q is 0: no contribution
            DF P{0.0f, 0.0f};
            trace_sorted<kKB>(bv, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz, i, t_eps, t_min, stack_mem + tid, blockDim.x,
                              err, [&](uint32_t j, float alpha, float T, bool front, float g, float) {
                                  const float G = front ? row_lookup(lc, lg, len, j) : 0.0f;
                                  const float f = exp_fx(-__fmul_rn(bv.c[j], g));
                                  opacity_hit(bv, j, G, alpha, f, T, g, W, P, my, scale);
                              });
        }
    }
}

// Compositing backward from the recorded hits: the same FP32 alpha and T
// sequence as the forward trace, G from an LDS hash of row i of dL/dF.
__device__ __forceinline__ float row_hash_lookup(const uint32_t *hk, const float *hv, int log2h, uint32_t j) {
    const uint32_t mask = (1u << log2h) - 1u;
    uint32_t h = hash_slot(j, log2h);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const uint32_t k = hk[h];
        if (k == j) return hv[h];
        if (k == kEmpty) return 0.0f;
        h = (h + 1) & mask;
    }
    return 0.0f;
}

__global__ void __launch_bounds__(256) k_opacity_rec(BvhDev bv, int R, const uint2 *__restrict__ recs,
                                                     const uint32_t *__restrict__ rcnt, int rcap, int64_t nblocks,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const float *__restrict__ gF,
                                                     int log2h, const int *fx_exp, unsigned long long *acc) {
    extern __shared__ uint32_t sm3[];
    const int H = 1 << log2h;
    uint32_t *hk = sm3;
    float *hv = reinterpret_cast<float *>(sm3 + H);
    const int64_t b = xcd_block(blockIdx.x, nblocks);
    const int tid = threadIdx.x;
    const uint32_t i = __float_as_uint(bv.rec[b].d.w);
    for (int k = tid; k < H; k += blockDim.x) hk[k] = kEmpty;
    __syncthreads();
    const int64_t e0 = row_ptr[i];
    const int len = (int)(row_ptr[i + 1] - e0);
    const float invR = 1.0f / (float)R;
    const float scale = __builtin_ldexpf(1.0f, *fx_exp);
    unsigned long long *my = acc + (int64_t)xcc_id() * bv.n;
    for (int k = tid; k < len; k += blockDim.x) {
        const uint32_t j = (uint32_t)col[e0 + k];
        uint32_t h = hash_slot(j, log2h);
        while (atomicCAS(&hk[h], kEmpty, j) != kEmpty) h = (h + 1) & (uint32_t)(H - 1);
        hv[h] = gF[e0 + k] * invR;
    }
    __syncthreads();
    for (int r = tid; r < R; r += blockDim.x) {
        const uint32_t m = rcnt[(int64_t)i * R + r];
        if (m > (uint32_t)rcap) continue;
        const uint2 *in = recs + (int64_t)i * rcap * R + r;
        DF W{0.0f, 0.0f};
        float T = 1.0f;
        for (uint32_t q = 0; q < m; ++q) {
            const uint2 h = in[(int64_t)q * R];
            const float gs = __uint_as_float(h.y);
            const float x = bv.c[h.x] * fabsf(gs);
            if (gs > 0.0f) {
                const float G = row_hash_lookup(hk, hv, log2h, h.x);
                if (G != 0.0f) W = df_add(W, df_prod3(G, -expm1f(-x), T));
            }
            T = __fmul_rn(T, exp_fx(-x));
        }
        if (W.hi == 0.0f) continue;   // every G_q alpha_q T_q is 0: no contribution
        DF P{0.0f, 0.0f};
        T = 1.0f;
        for (uint32_t q = 0; q < m; ++q) {
            const uint2 h = in[(int64_t)q * R];
            const float gs = __uint_as_float(h.y);
            const float g = fabsf(gs);
            const float x = bv.c[h.x] * g;
            const float f = exp_fx(-x);
            const float G = gs > 0.0f ? row_hash_lookup(hk, hv, log2h, h.x) : 0.0f;
            opacity_hit(bv, h.x, G, -expm1f(-x), f, T, g, W, P, my, scale);
            T = __fmul_rn(T, f);
        }
    }
}

__global__ void __launch_bounds__(256) k_opacity_finish(BvhDev bv, const unsigned long long *__restrict__ acc,
                                                        const int *fx_exp, const float *__restrict__ grad_rho,
                                                        const float *__restrict__ albedo, float *grad_o, float *grad_a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= bv.n) return;
    const float oraw = bv.raw_op[i];
    const bool inside = oraw > 0.0f && oraw < kOpacityMax;
    unsigned long long s = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) s += acc[(int64_t)x * bv.n + i];
    const int e = *fx_exp;
    float g = e == kFxNonFinite ? __builtin_nanf("") : __builtin_ldexpf(__ll2float_rn((long long)s), -e);
    if (grad_rho && albedo && inside)
        g += grad_rho[3 * i] * albedo[3 * i] + grad_rho[3 * i + 1] * albedo[3 * i + 1] +
             grad_rho[3 * i + 2] * albedo[3 * i + 2];
    if (grad_o) grad_o[i] = g;
    if (grad_a) {
        const float o = bv.op[i];
        for (int c = 0; c < 3; ++c) grad_a[3 * i + c] = grad_rho ? grad_rho[3 * i + c] * o : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// centre-to-centre form factors (Sec. 8) and their gradients
// ---------------------------------------------------------------------------
// Every surfel other than skip_a and skip_b whose support the segment
// o + t d, t in (t_lo, t_hi), crosses (D_hit, both faces occlude);
// on_hit(record) per crossing, in traversal order.
template <typename OnHit>
__device__ __forceinline__ void trace_segment(const BvhDev &bv, float ox, float oy, float oz, float dx, float dy,
                                              float dz, uint32_t skip_a, uint32_t skip_b, float t_lo, float t_hi,
                                              uint32_t *stack, int stride, int *err, OnHit &&on_hit) {
    const float ix = safe_inv(dx), iy = safe_inv(dy), iz = safe_inv(dz);
    const float t0 = t_lo * 0.99999f, t1 = t_hi * 1.00001f;
    auto leaf = [&](int s) {
        const SurfRec r = bv.rec[s];
        asm volatile("" : : "v"(r.a.x), "v"(r.b.x), "v"(r.c.x), "v"(r.d.w));   // whole record in one latency
        const uint32_t j = __float_as_uint(r.d.w);
        if (j == skip_a || j == skip_b) return;
        float t, r2;
        bool front;
        if (!hit_test(r, ox, oy, oz, dx, dy, dz, t_lo, t_hi, true, t, r2, front)) return;
        on_hit(r);
    };
    if (bv.n == 1) {
        leaf(0);
        return;
    }
    int sp = 0, node = 0;
    bool ovf = false;
    for (;;) {
        const Node nd = bv.nodes[node];
        float tn0, tn1;
        bool h0 = slab(nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y, ox, oy, oz, ix, iy, iz, t0, t1, tn0);
        bool h1 = slab(nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w, ox, oy, oz, ix, iy, iz, t0, t1, tn1);
        const int c0 = nd.ch.x, c1 = nd.ch.y;
        if (h0 && c0 < 0) {
            leaf(~c0);
            h0 = false;
        }
        if (h1 && c1 < 0) {
            leaf(~c1);
            h1 = false;
        }
        // descend (first child first), push the other; none left: pop.  A
        // push past the stack's end ends the walk with an error.
        const bool both = h0 && h1;
        ovf = both && sp >= kStackDeep;
        if (both) stack[min(sp, kStackDeep - 1) * stride] = (uint32_t)c1;
        sp += both ? 1 : 0;
        node = h0 ? c0 : c1;
        if (!h0 && !h1) {
            if (sp == 0) break;
            --sp;
            node = (int)stack[sp * stride];
        }
        if (ovf) break;
    }
    if (ovf) atomicOr(err, kErrStack);
}

constexpr int kCenterThreads = 128;   // two rows (waves) per workgroup
constexpr int kCenterFields = 16;     // p(3), t_u(3), t_v(3), n(3), s_u, s_v, o, lambda
constexpr float kInvPi = 0.318309886183790672f;

struct Segment {
    float ox, oy, oz, dx, dy, dz, t_lo, t_hi;
};

// The segment between the centres of ri and rj, its ends trimmed by t_eps
__device__ __forceinline__ Segment make_segment(const SurfRec &ri, const SurfRec &rj, float t_eps) {
    Segment g;
    g.ox = ri.a.x;
    g.oy = ri.a.y;
    g.oz = ri.a.z;
    g.dx = __fsub_rn(rj.a.x, ri.a.x);
    g.dy = __fsub_rn(rj.a.y, ri.a.y);
    g.dz = __fsub_rn(rj.a.z, ri.a.z);
    const float len = sqrt_rn(__builtin_fmaf(g.dz, g.dz, __builtin_fmaf(g.dy, g.dy, __fmul_rn(g.dx, g.dx))));
    g.t_lo = __fdiv_rn(t_eps, len);
    g.t_hi = __fsub_rn(1.0f, g.t_lo);
    return g;
}

// F_ij = lambda_j A_j T_ij |n_i . v| |n_j . v| / (pi |v|^4) per stored entry
// of the pattern (v = p_j - p_i); one wave per row, lanes over entries.
__global__ void __launch_bounds__(kCenterThreads) k_ff_center(BvhDev bv, const int64_t *__restrict__ row_ptr,
                                                              const int32_t *__restrict__ col, int64_t n,
                                                              const float *__restrict__ lambda,
                                                              float *__restrict__ val, int64_t nblocks,
                                                              const int32_t *__restrict__ order, int *err) {
    extern __shared__ uint32_t stack_mem[];
    const int64_t idx = xcd_block(blockIdx.x, nblocks) * (kCenterThreads / 64) + threadIdx.x / 64;
    if (idx >= n) return;
    const int64_t row = order ? (int64_t)order[idx] : idx;
    const int lane = __lane_id();
    const SurfRec ri = bv.rec[bv.inv[row]];
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    const float t_eps = bv.bounds[6];
    for (int64_t kk = b + lane; kk < e; kk += 64) {
        const int32_t j = col[kk];
        const SurfRec rj = bv.rec[bv.inv[j]];
        const Segment g = make_segment(ri, rj, t_eps);
        float T = 1.0f;
        trace_segment(bv, g.ox, g.oy, g.oz, g.dx, g.dy, g.dz, (uint32_t)row, (uint32_t)j, g.t_lo, g.t_hi,
                      stack_mem + threadIdx.x, kCenterThreads, err, [&](const SurfRec &r) {
                          T = __fmul_rn(T, transmit(r.c.w, kernel_gamma(hit_r2_exact(r, g.ox, g.oy, g.oz, g.dx,
                                                                                     g.dy, g.dz))));
                      });
        const float a = ri.b.x * g.dx + ri.b.y * g.dy + ri.b.z * g.dz;
        const float bb = rj.b.x * g.dx + rj.b.y * g.dy + rj.b.z * g.dz;
        const float r2 = g.dx * g.dx + g.dy * g.dy + g.dz * g.dz;
        const float phi = (fabsf(a) * fabsf(bb)) / (r2 * r2);
        val[kk] = lambda[j] * (float)bv.area[j] * T * phi * kInvPi;
    }
}

// Gradients of sum_e G_e F_e (same decomposition as the oracle's): pass 0
// finds max |contribution| per field, pass 1 adds the contributions in
// 64-bit fixed point with a per-field power-of-two scale (integer adds
// commute: bit-identical between runs) into one copy per XCD.
template <int PASS>
struct CenterSink {
    float m[kCenterFields];   // pass 0: largest |contribution| per field
    float qm;                 // pass 1: largest |scaled contribution| (INFINITY once one is not finite)
    unsigned long long *acc;
    const int *fx;
    int64_t n;
    __device__ __forceinline__ void track(float q) {
        const float a = fabsf(q);
        qm = a <= 3.0e38f ? fmaxf(qm, a) : INFINITY;
    }
    __device__ __forceinline__ void add(int f, uint32_t surfel, float v) {
        if (PASS == 0) {
            m[f] = fmaxf(m[f], fabsf(v));
        } else {
            const float q = v * __builtin_ldexpf(1.0f, fx[f]);
            track(q);
            const long long qq = __float2ll_rn(q);
            if (qq != 0)
                __hip_atomic_fetch_add(acc + (int64_t)f * n + surfel, (unsigned long long)qq, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __device__ __forceinline__ void add3(int f, uint32_t surfel, float x, float y, float z) {
        add(f, surfel, x);
        add(f + 1, surfel, y);
        add(f + 2, surfel, z);
    }
    // wave maxima to maxbits[0..15] (pass 0) or maxbits[32] (pass 1); every
    // lane of the wave calls this
    template <int P>
    __device__ __forceinline__ void report(uint32_t *maxbits) {
        if (P == 0) {
#pragma unroll
            for (int f = 0; f < kCenterFields; ++f) {
                float v = m[f];
                for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
                if (__lane_id() == 0 && v > 0.0f) atomicMax(maxbits + f, __float_as_uint(v));
            }
        } else {
            float v = qm;
            for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
            if (__lane_id() == 0 && v > 0.0f) atomicMax(maxbits + 2 * kCenterFields, __float_as_uint(v));
        }
    }
};

// Contributions of one thread to NF fields of one surfel that the whole
// wave shares (the row's receiver): summed per thread in the fields' 64-bit
// fixed point (exact), then over the wave, and added with one atomic per
// field instead of one per contribution to the same address.
template <int NF>
struct SharedSurfelAcc {
    long long q[NF];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int f = 0; f < NF; ++f) q[f] = 0;
    }
    template <int PASS, typename Sink>
    __device__ __forceinline__ void add(Sink &sink, int slot, int field, float v) {
        if (PASS == 0) {
            sink.m[field] = fmaxf(sink.m[field], fabsf(v));
        } else {
            const float qv = v * __builtin_ldexpf(1.0f, sink.fx[field]);
            sink.track(qv);
            q[slot] += __float2ll_rn(qv);
        }
    }
    // every lane of the wave must call this (shuffles); lanes whose surfel
    // differs from lane 0's are not allowed
    template <int PASS>
    __device__ __forceinline__ void flush(unsigned long long *acc, int64_t n, uint32_t surfel, const int *fields) {
        if (PASS == 0) return;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            long long v = q[f];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (__lane_id() == 0 && v != 0)
                __hip_atomic_fetch_add(acc + (int64_t)fields[f] * n + surfel, (unsigned long long)v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
};

template <int PASS>
__global__ void __launch_bounds__(kCenterThreads) k_center_bwd(BvhDev bv, const int64_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col,
                                                               const float *__restrict__ fval, int64_t n,
                                                               const float *__restrict__ lambda,
                                                               const float *__restrict__ gF, uint32_t *maxbits,
                                                               const int *fx, unsigned long long *acc,
                                                               int64_t nblocks, const int32_t *__restrict__ order,
                                                               int stride, int *err) {
    extern __shared__ uint32_t stack_mem[];
    const int64_t idx = (xcd_block(blockIdx.x, nblocks) * (kCenterThreads / 64) + threadIdx.x / 64) * stride;
    CenterSink<PASS> sink;
#pragma unroll
    for (int f = 0; f < kCenterFields; ++f) sink.m[f] = 0.0f;
    sink.qm = 0.0f;
    sink.acc = acc + (int64_t)xcc_id() * kCenterFields * n;
    sink.fx = fx;
    sink.n = n;
    const float t_eps = bv.bounds[6];
    SharedSurfelAcc<6> accI;   // the row's receiver: p (fields 0-2) and n (9-11)
    accI.zero();
    uint32_t i = 0;
    if (idx < n) {
        const int64_t row = order ? (int64_t)order[idx] : idx;
        i = (uint32_t)row;
        const SurfRec ri = bv.rec[bv.inv[row]];
        const int64_t b = row_ptr[row], e = row_ptr[row + 1];
        for (int64_t kk = b + __lane_id(); kk < e; kk += 64) {
            const float G = gF[kk];
            if (G == 0.0f) continue;
            const uint32_t j = (uint32_t)col[kk];
            const SurfRec rj = bv.rec[bv.inv[j]];
            const Segment g = make_segment(ri, rj, t_eps);
            const float W = G * fval[kk];
            float T = 1.0f;
            float gpi[3] = {0.0f, 0.0f, 0.0f}, gpj[3] = {0.0f, 0.0f, 0.0f};
            trace_segment(bv, g.ox, g.oy, g.oz, g.dx, g.dy, g.dz, i, j, g.t_lo, g.t_hi, stack_mem + threadIdx.x,
                          kCenterThreads, err, [&](const SurfRec &r) {
                              // exact kernel value for T, FP32 geometry for the derivatives
                              const float gam = kernel_gamma(hit_r2_exact(r, g.ox, g.oy, g.oz, g.dx, g.dy, g.dz));
                              T = __fmul_rn(T, transmit(r.c.w, gam));
                              const uint32_t k = __float_as_uint(r.d.w);
                              const float qx = r.a.x - g.ox, qy = r.a.y - g.oy, qz = r.a.z - g.oz;
                              const float den = g.dx * r.b.x + g.dy * r.b.y + g.dz * r.b.z;
                              const float tk = (qx * r.b.x + qy * r.b.y + qz * r.b.z) / den;
                              const float hx = tk * g.dx - qx, hy = tk * g.dy - qy, hz = tk * g.dz - qz;
                              const float u = (hx * r.c.x + hy * r.c.y + hz * r.c.z) * r.a.w;
                              const float w = (hx * r.d.x + hy * r.d.y + hz * r.d.z) * r.b.w;
                              const float f = W * 3.4f * r.c.w * gam;
                              const float fu = f * u * r.a.w, fw = f * w * r.b.w;
                              const float ghx = fu * r.c.x + fw * r.d.x, ghy = fu * r.c.y + fw * r.d.y,
                                          ghz = fu * r.c.z + fw * r.d.z;
                              const float beta = (ghx * g.dx + ghy * g.dy + ghz * g.dz) / den;
                              const float gqx = beta * r.b.x - ghx, gqy = beta * r.b.y - ghy,
                                          gqz = beta * r.b.z - ghz;
                              sink.add3(0, k, gqx, gqy, gqz);
                              sink.add3(3, k, fu * hx, fu * hy, fu * hz);
                              sink.add3(6, k, fw * hx, fw * hy, fw * hz);
                              sink.add3(9, k, -beta * hx, -beta * hy, -beta * hz);
                              sink.add(12, k, -fu * u);
                              sink.add(13, k, -fw * w);
                              const float ok = bv.raw_op[k];
                              if (ok > 0.0f && ok < kOpacityMax) sink.add(14, k, -W * gam / (1.0f - ok));
                              gpi[0] -= (1.0f - tk) * gqx;
                              gpi[1] -= (1.0f - tk) * gqy;
                              gpi[2] -= (1.0f - tk) * gqz;
                              gpj[0] -= tk * gqx;
                              gpj[1] -= tk * gqy;
                              gpj[2] -= tk * gqz;
                          });
            // the pair's own terms: Phi = |a| |b| / r^4, kappa = lambda_j A_j / pi
            const float a = ri.b.x * g.dx + ri.b.y * g.dy + ri.b.z * g.dz;
            const float bb = rj.b.x * g.dx + rj.b.y * g.dy + rj.b.z * g.dz;
            const float r2 = g.dx * g.dx + g.dy * g.dy + g.dz * g.dz;
            const float r4 = r2 * r2;
            const float aa = fabsf(a), ab = fabsf(bb);
            const float sa = a > 0.0f ? 1.0f : (a < 0.0f ? -1.0f : 0.0f);
            const float sb = bb > 0.0f ? 1.0f : (bb < 0.0f ? -1.0f : 0.0f);
            const float A = (float)bv.area[j];
            const float kT = G * lambda[j] * A * T * kInvPi;
            const float c1 = kT * sa * ab / r4, c2 = kT * aa * sb / r4, c3 = 4.0f * kT * aa * ab / (r4 * r2);
            const float dpx = c1 * ri.b.x + c2 * rj.b.x - c3 * g.dx;
            const float dpy = c1 * ri.b.y + c2 * rj.b.y - c3 * g.dy;
            const float dpz = c1 * ri.b.z + c2 * rj.b.z - c3 * g.dz;
            sink.add3(0, j, dpx + gpj[0], dpy + gpj[1], dpz + gpj[2]);
            accI.add<PASS>(sink, 0, 0, gpi[0] - dpx);
            accI.add<PASS>(sink, 1, 1, gpi[1] - dpy);
            accI.add<PASS>(sink, 2, 2, gpi[2] - dpz);
            accI.add<PASS>(sink, 3, 9, c1 * g.dx);
            accI.add<PASS>(sink, 4, 10, c1 * g.dy);
            accI.add<PASS>(sink, 5, 11, c1 * g.dz);
            sink.add3(9, j, c2 * g.dx, c2 * g.dy, c2 * g.dz);
            const float phi = aa * ab / r4;
            sink.add(15, j, G * A * T * phi * kInvPi);
            const float gA = G * lambda[j] * T * phi * kInvPi;
            sink.add(12, j, gA * A * rj.a.w);
            sink.add(13, j, gA * A * rj.b.w);
            sink.add(14, j, gA * bv.dado[j]);
        }
    }
    // one row per wave: every lane's receiver is the row's
    if (idx < n) {
        const int fI[6] = {0, 1, 2, 9, 10, 11};
        accI.flush<PASS>(sink.acc, n, i, fI);
    }
    sink.template report<PASS>(maxbits);
}

// per-field exponent: (max contribution) * count * 2^margin < 2^62 (count
// bounds the contributions a surfel's field can receive; margin: headroom
// over a maximum estimated on sampled rows)
__global__ void k_center_exp_count(const uint32_t *maxbits, int64_t count, int margin, int *fx) {
    const int f = threadIdx.x;
    if (f >= kCenterFields) return;
    const float m = __uint_as_float(maxbits[f]);
    int e = 0;
    if (!(m <= 3.0e38f)) {
        e = kFxNonFinite;
    } else if (m > 0.0f) {
        int ex;
        (void)frexpf(m * (float)count, &ex);
        e = min(120, max(-120, 62 - ex - margin));
    }
    fx[f] = e;
}


__global__ void __launch_bounds__(256) k_center_finish(const unsigned long long *__restrict__ acc, const int *fx,
                                                       int64_t n, CenterOutputs out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * kCenterFields) return;
    const int f = (int)(t / n);
    const int64_t i = t - (int64_t)f * n;
    float *o = out.p[f];
    if (!o) return;
    unsigned long long s = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) s += acc[((int64_t)x * kCenterFields + f) * n + i];
    const int e = fx[f];
    o[i] = e == kFxNonFinite ? __builtin_nanf("") : __builtin_ldexpf(__ll2float_rn((long long)s), -e);
}

// ---------------------------------------------------------------------------
// geometry gradients through the ray-cast form factors (recorded hits)
// ---------------------------------------------------------------------------
// The compositing backward's dL/dalpha per recorded hit (as k_opacity_rec)
// chained to the hit surfel's centre, frame, scales and opacity and to the
// receiver's centre and frame (ray origin p_i, direction
// d = x t_u + y t_v + z n): alpha = 1 - e^(-c gamma), gamma = e^(-1.7 (u^2+w^2)),
// u = h . t_u / s_u, w = h . t_v / s_v, h = t d - q, q = p_k - p_i,
// t = (q . n_k)/(d . n_k).  The hit point is the FP64 intersection.  Sums in
// 64-bit fixed point with per-field scales from a first pass (bit-identical
// between runs), one copy per XCD; fields px..o as in CenterOutputs.
template <int PASS>
__global__ void __launch_bounds__(256) k_geometry_rec(BvhDev bv, int R, uint64_t seed, const uint2 *__restrict__ recs,
                                                      const uint32_t *__restrict__ rcnt, int rcap, int64_t nblocks,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col, const float *__restrict__ gF,
                                                      int log2h, uint32_t *maxbits, const int *fx,
                                                      unsigned long long *acc, int stride) {
    extern __shared__ uint32_t sm4[];
    const int H = 1 << log2h;
    uint32_t *hk = sm4;
    float *hv = reinterpret_cast<float *>(sm4 + H);
    const int64_t b = xcd_block(blockIdx.x, nblocks) * stride;
    const int tid = threadIdx.x;
    const SurfRec ri = bv.rec[b];
    const uint32_t i = __float_as_uint(ri.d.w);
    for (int k = tid; k < H; k += blockDim.x) hk[k] = kEmpty;
    __syncthreads();
    const int64_t e0 = row_ptr[i];
    const int len = (int)(row_ptr[i + 1] - e0);
    const float invR = 1.0f / (float)R;
    for (int k = tid; k < len; k += blockDim.x) {
        const uint32_t j = (uint32_t)col[e0 + k];
        uint32_t h = hash_slot(j, log2h);
        while (atomicCAS(&hk[h], kEmpty, j) != kEmpty) h = (h + 1) & (uint32_t)(H - 1);
        hv[h] = gF[e0 + k] * invR;
    }
    __syncthreads();
    CenterSink<PASS> sink;
#pragma unroll
    for (int f = 0; f < kCenterFields; ++f) sink.m[f] = 0.0f;
    sink.qm = 0.0f;
    sink.acc = acc + (int64_t)xcc_id() * kCenterFields * bv.n;
    sink.fx = fx;
    sink.n = bv.n;
    SharedSurfelAcc<12> accI;   // the receiver: p, t_u, t_v, n (fields 0-11)
    accI.zero();
    for (int r = tid; r < R; r += blockDim.x) {
        const uint32_t m = rcnt[(int64_t)i * R + r];
        if (m > (uint32_t)rcap) continue;
        const uint2 *in = recs + (int64_t)i * rcap * R + r;
        DF W{0.0f, 0.0f};
        float T = 1.0f;
        for (uint32_t q = 0; q < m; ++q) {
            const uint2 h = in[(int64_t)q * R];
            const float gs = __uint_as_float(h.y);
            const float x = bv.c[h.x] * fabsf(gs);
            if (gs > 0.0f) {
                const float G = row_hash_lookup(hk, hv, log2h, h.x);
                if (G != 0.0f) W = df_add(W, df_prod3(G, -expm1f(-x), T));
            }
            T = __fmul_rn(T, exp_fx(-x));
        }
        if (W.hi == 0.0f) continue;
        float dx, dy, dz, sx, sy, sz;
        ray_direction(ri.c.x, ri.c.y, ri.c.z, ri.d.x, ri.d.y, ri.d.z, ri.b.x, ri.b.y, ri.b.z, (uint64_t)r,
                      (uint64_t)i, seed, 0, dx, dy, dz);
        ray_sample((uint64_t)r, (uint64_t)i, seed, 0, sx, sy, sz);
        float gd[3] = {0.0f, 0.0f, 0.0f}, gpi[3] = {0.0f, 0.0f, 0.0f};
        DF P{0.0f, 0.0f};
        T = 1.0f;
        for (uint32_t q = 0; q < m; ++q) {
            const uint2 h = in[(int64_t)q * R];
            const float gs = __uint_as_float(h.y);
            const float g = fabsf(gs);
            const uint32_t k = h.x;
            const float c = bv.c[k];
            const float x = c * g;
            const float f = exp_fx(-x);
            const float alpha = -expm1f(-x);
            const float G = gs > 0.0f ? row_hash_lookup(hk, hv, log2h, k) : 0.0f;
            if (G != 0.0f) P = df_add(P, df_prod3(G, alpha, T));
            const DF Sd = df_add(W, DF{-P.hi, -P.lo});
            const float dLda = G * T - Sd.hi / f;
            T = __fmul_rn(T, f);
            if (dLda == 0.0f) continue;
            const float ok = bv.raw_op[k];
            if (ok > 0.0f && ok < kOpacityMax) sink.add(14, k, dLda * g * f / (1.0f - ok));
            // the FP64 hit point of the FP32 ray on k's plane
            const SurfRec rk = bv.rec[bv.inv[k]];
            const double nx = rk.b.x, ny = rk.b.y, nz = rk.b.z;
            const double qx = (double)rk.a.x - ri.a.x, qy = (double)rk.a.y - ri.a.y, qz = (double)rk.a.z - ri.a.z;
            const double den = (double)dx * nx + (double)dy * ny + (double)dz * nz;
            const double tk = (qx * nx + qy * ny + qz * nz) / den;
            const float hx = (float)(tk * dx - qx), hy = (float)(tk * dy - qy), hz = (float)(tk * dz - qz);
            const float u = (hx * rk.c.x + hy * rk.c.y + hz * rk.c.z) * rk.a.w;
            const float w = (hx * rk.d.x + hy * rk.d.y + hz * rk.d.z) * rk.b.w;
            const float dLdg = dLda * c * f;
            const float du = dLdg * (-3.4f) * g * u * rk.a.w, dw = dLdg * (-3.4f) * g * w * rk.b.w;
            const float ghx = du * rk.c.x + dw * rk.d.x, ghy = du * rk.c.y + dw * rk.d.y, ghz = du * rk.c.z + dw * rk.d.z;
            const float beta = (ghx * dx + ghy * dy + ghz * dz) / (float)den;
            const float gqx = beta * rk.b.x - ghx, gqy = beta * rk.b.y - ghy, gqz = beta * rk.b.z - ghz;
            sink.add3(0, k, gqx, gqy, gqz);
            sink.add3(3, k, du * hx, du * hy, du * hz);
            sink.add3(6, k, dw * hx, dw * hy, dw * hz);
            sink.add3(9, k, -beta * hx, -beta * hy, -beta * hz);
            sink.add(12, k, -du * u);
            sink.add(13, k, -dw * w);
            const float tf = (float)tk;
            gpi[0] -= gqx;
            gpi[1] -= gqy;
            gpi[2] -= gqz;
            gd[0] -= tf * gqx;
            gd[1] -= tf * gqy;
            gd[2] -= tf * gqz;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            accI.add<PASS>(sink, c, c, gpi[c]);
            accI.add<PASS>(sink, 3 + c, 3 + c, sx * gd[c]);
            accI.add<PASS>(sink, 6 + c, 6 + c, sy * gd[c]);
            accI.add<PASS>(sink, 9 + c, 9 + c, sz * gd[c]);
        }
    }
    {
        const int fI[12] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
        accI.flush<PASS>(sink.acc, bv.n, i, fI);
    }
    sink.template report<PASS>(maxbits);
}


// ---------------------------------------------------------------------------
// direct-light gradients: light positions and intensities, albedo, surfel
// fields of the receivers and of the occluders on the shadow segments
// ---------------------------------------------------------------------------
// One thread per receiver, lights in turn.  With v = x_l - p_i, r = |v|,
// ndot = n_i . v > 0, E_c = o a_c kappa I ndot T / r^3 (kappa = 2/sqrt(pi)),
// S = sum_c dL/dE_c a_c, Q = S o kappa I T:
//   dL/dI += S o kappa ndot T / r^3, dL/da_c += dL/dE_c o kappa I ndot T / r^3,
//   dL/do_i += S kappa I ndot T / r^3, g_v = Q (n/r^3 - 3 ndot v/r^5):
//   x_l += g_v, p_i -= g_v, n_i += Q v / r^3,
// and the shadow segment's occluders as for a centre-to-centre segment with
// W = S o kappa I ndot T / r^3.  Fields 0..14 surfel (px..o), 15..18 the
// light (x, y, z, I) in their own accumulators; fixed point as above.
constexpr int kLightFields = 19;

template <int PASS>
struct LightSink {
    float m[kLightFields];
    unsigned long long *acc;     // surfel fields [16][n] of this XCD
    unsigned long long *lacc;    // light fields [4][Lt] of this XCD
    const int *fx;
    int64_t n;
    int Lt;
    __device__ __forceinline__ void add(int f, uint32_t surfel, float v) {
        if (PASS == 0) m[f] = fmaxf(m[f], fabsf(v));
        else fx_add(acc + (int64_t)f * n + surfel, v, __builtin_ldexpf(1.0f, fx[f]));
    }
    __device__ __forceinline__ void add3(int f, uint32_t surfel, float x, float y, float z) {
        add(f, surfel, x);
        add(f + 1, surfel, y);
        add(f + 2, surfel, z);
    }
};

template <int PASS>
__global__ void __launch_bounds__(128) k_direct_bwd(BvhDev bv, const float *__restrict__ albedo,
                                                    const float *__restrict__ lpos, const float *__restrict__ lI,
                                                    int Lt, int K, const float *__restrict__ gE, uint32_t *maxbits,
                                                    const int *fx, unsigned long long *acc, unsigned long long *lacc,
                                                    float *__restrict__ g_alb, int *err) {
    extern __shared__ uint32_t stack_mem[];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    LightSink<PASS> sink;
#pragma unroll
    for (int f = 0; f < kLightFields; ++f) sink.m[f] = 0.0f;
    const int xcc = xcc_id();
    sink.acc = acc + (int64_t)xcc * kCenterFields * bv.n;
    sink.lacc = lacc + (int64_t)xcc * 4 * Lt;
    sink.fx = fx;
    sink.n = bv.n;
    sink.Lt = Lt;
    const bool live = i < bv.n;
    const SurfRec rr = live ? bv.rec[bv.inv[i]] : bv.rec[0];
    const float oc = live ? bv.op[i] : 0.0f;
    const float oraw = live ? bv.raw_op[i] : 0.0f;
    const bool inside = oraw > 0.0f && oraw < kOpacityMax;
    float ga[3] = {0.0f, 0.0f, 0.0f};
    const float a0 = live ? albedo[3 * i] : 0.0f, a1 = live ? albedo[3 * i + 1] : 0.0f,
                a2 = live ? albedo[3 * i + 2] : 0.0f;
    for (int l = 0; l < Lt; ++l) {
        float gl[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        const float *ge = gE + ((i * Lt + l) * K) * 3;
        const float S = live ? ge[0] * a0 + ge[1] * a1 + ge[2] * a2 : 0.0f;
        const float dx = __fsub_rn(lpos[3 * l + 0], rr.a.x);
        const float dy = __fsub_rn(lpos[3 * l + 1], rr.a.y);
        const float dz = __fsub_rn(lpos[3 * l + 2], rr.a.z);
        const float dd = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __fmul_rn(dx, dx)));
        const float ndot = rr.b.x * dx + rr.b.y * dy + rr.b.z * dz;
        if (live && ndot > 0.0f && dd > 0.0f && S != 0.0f) {
            const float len = sqrt_rn(dd);
            const float t_lo = __fdiv_rn(bv.bounds[6], len);
            const float r3 = dd * len, r5 = r3 * dd;
            // the transmittance first (the occluders' weight W needs it)
            float T = 1.0f;
            trace_segment(bv, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz, (uint32_t)i, (uint32_t)i, t_lo, 1.0f,
                          stack_mem + threadIdx.x, blockDim.x, err, [&](const SurfRec &r) {
                              T = __fmul_rn(T, transmit(r.c.w, kernel_gamma(hit_r2_exact(r, rr.a.x, rr.a.y, rr.a.z,
                                                                                         dx, dy, dz))));
                          });
            const float kI = 1.1283791670955126f * lI[l];
            const float base = kI * ndot * T / r3;
            gl[3] = S * oc * 1.1283791670955126f * ndot * T / r3;
            ga[0] += ge[0] * oc * base;
            ga[1] += ge[1] * oc * base;
            ga[2] += ge[2] * oc * base;
            if (inside) sink.add(14, (uint32_t)i, S * base);
            const float Q = S * oc * kI * T;
            const float gvx = Q * (rr.b.x / r3 - 3.0f * ndot * dx / r5);
            const float gvy = Q * (rr.b.y / r3 - 3.0f * ndot * dy / r5);
            const float gvz = Q * (rr.b.z / r3 - 3.0f * ndot * dz / r5);
            float gpi[3] = {-gvx, -gvy, -gvz};
            gl[0] = gvx;
            gl[1] = gvy;
            gl[2] = gvz;
            sink.add3(9, (uint32_t)i, Q * dx / r3, Q * dy / r3, Q * dz / r3);
            const float W = S * oc * base;
            trace_segment(bv, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz, (uint32_t)i, (uint32_t)i, t_lo, 1.0f,
                          stack_mem + threadIdx.x, blockDim.x, err, [&](const SurfRec &r) {
                              const float gam = kernel_gamma(hit_r2_exact(r, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz));
                              const uint32_t k = __float_as_uint(r.d.w);
                              const float qx = r.a.x - rr.a.x, qy = r.a.y - rr.a.y, qz = r.a.z - rr.a.z;
                              const float den = dx * r.b.x + dy * r.b.y + dz * r.b.z;
                              const float tk = (qx * r.b.x + qy * r.b.y + qz * r.b.z) / den;
                              const float hx = tk * dx - qx, hy = tk * dy - qy, hz = tk * dz - qz;
                              const float u = (hx * r.c.x + hy * r.c.y + hz * r.c.z) * r.a.w;
                              const float w = (hx * r.d.x + hy * r.d.y + hz * r.d.z) * r.b.w;
                              const float f = W * 3.4f * r.c.w * gam;
                              const float fu = f * u * r.a.w, fw = f * w * r.b.w;
                              const float ghx = fu * r.c.x + fw * r.d.x, ghy = fu * r.c.y + fw * r.d.y,
                                          ghz = fu * r.c.z + fw * r.d.z;
                              const float beta = (ghx * dx + ghy * dy + ghz * dz) / den;
                              const float gqx = beta * r.b.x - ghx, gqy = beta * r.b.y - ghy,
                                          gqz = beta * r.b.z - ghz;
                              sink.add3(0, k, gqx, gqy, gqz);
                              sink.add3(3, k, fu * hx, fu * hy, fu * hz);
                              sink.add3(6, k, fw * hx, fw * hy, fw * hz);
                              sink.add3(9, k, -beta * hx, -beta * hy, -beta * hz);
                              sink.add(12, k, -fu * u);
                              sink.add(13, k, -fw * w);
                              const float ok = bv.raw_op[k];
                              if (ok > 0.0f && ok < kOpacityMax) sink.add(14, k, -W * gam / (1.0f - ok));
                              gpi[0] -= (1.0f - tk) * gqx;
                              gpi[1] -= (1.0f - tk) * gqy;
                              gpi[2] -= (1.0f - tk) * gqz;
                              gl[0] -= tk * gqx;
                              gl[1] -= tk * gqy;
                              gl[2] -= tk * gqz;
                          });
            sink.add3(0, (uint32_t)i, gpi[0], gpi[1], gpi[2]);
        }
        // the light's fields: one wave sum, then one fixed-point add per wave
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (PASS == 0) {
                sink.m[15 + q] = fmaxf(sink.m[15 + q], fabsf(gl[q]));
            } else {
                const long long fxv = __float2ll_rn(gl[q] * __builtin_ldexpf(1.0f, fx[15 + q]));
                unsigned long long tot = (unsigned long long)fxv;
                for (int off = 32; off > 0; off >>= 1) tot += (unsigned long long)__shfl_xor((long long)tot, off, 64);
                if (__lane_id() == 0 && tot != 0)
                    __hip_atomic_fetch_add(sink.lacc + (int64_t)q * Lt + l, tot, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    if (PASS == 1 && live && g_alb) {
        g_alb[3 * i + 0] = ga[0];
        g_alb[3 * i + 1] = ga[1];
        g_alb[3 * i + 2] = ga[2];
    }
    if (PASS == 0) {
#pragma unroll
        for (int f = 0; f < kLightFields; ++f) {
            float v = sink.m[f];
            for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
            if (__lane_id() == 0 && v > 0.0f) atomicMax(maxbits + f, __float_as_uint(v));
        }
    }
}

__global__ void k_light_exp(const uint32_t *maxbits, int64_t count_surfel, int64_t count_light, int *fx) {
    const int f = threadIdx.x;
    if (f >= kLightFields) return;
    const float m = __uint_as_float(maxbits[f]);
    int e = 0;
    if (!(m <= 3.0e38f)) {
        e = kFxNonFinite;
    } else if (m > 0.0f) {
        int ex;
        (void)frexpf(m * (float)(f < 15 ? count_surfel : count_light), &ex);
        e = min(120, max(-120, 62 - ex));
    }
    fx[f] = e;
}

__global__ void k_light_finish(const unsigned long long *__restrict__ lacc, const int *fx, int Lt, float *g_lpos,
                               float *g_lI) {
    const int t = threadIdx.x + blockIdx.x * blockDim.x;
    if (t >= 4 * Lt) return;
    const int q = t / Lt, l = t % Lt;
    unsigned long long s = 0;
    for (int x = 0; x < 8; ++x) s += lacc[((int64_t)x * 4 + q) * Lt + l];
    const int e = fx[15 + q];
    const float v = e == kFxNonFinite ? __builtin_nanf("") : __builtin_ldexpf(__ll2float_rn((long long)s), -e);
    if (q < 3) {
        if (g_lpos) g_lpos[3 * l + q] = v;
    } else if (g_lI) {
        g_lI[l] = v;
    }
}

// ---------------------------------------------------------------------------
// Monte-Carlo TD(0) solver (Sec. 7, Alg. Monte-Carlo Solver, App. D)
// ---------------------------------------------------------------------------
// K-Means groups of the surfels (positions; the group keeps its mean
// centre, mean normal and the summed luminance of its members' current
// radiance as the proxy), then per step one next event per selected
// receiver a: a group g drawn with probability proportional to
//   w_g = L_g (|n_a . w_g| + beta)(|nbar_g . w_g| + beta) / max(r_g^2, r_min^2)
// and a member j != a of g proportional to the importance of Eq.
// importance-sampling, w_j = lum(B_j) |n_a . v||n_j . v| / |v|^4 (v = p_j - p_a);
// the one-point estimate (Eq. one-point-estimator) with the centre-to-centre
// decay of Sec. 8,
//   delta_a = E_a + rho_a F_aj B_j / Pr[j],  F_aj = lambda_j A_j T_aj |a||b| / (pi |v|^4),
// then the TD(0) averages (Eq. update): S += delta, S2 += delta^2, D += 1.
// Draws: Philox4x64-10 with counter (slot, step, 0, 2) (next event) and
// (slot, step, 1, 1) (receiver selection), key (seed, 0).
constexpr float kMcBeta = 0.05f;

__device__ __forceinline__ float lum3(const float *b) {
    return fmaxf(0.0f, 0.2126f * b[0] + 0.7152f * b[1] + 0.0722f * b[2]);
}

__device__ __forceinline__ float u01(uint64_t w) { return (float)(uint32_t)(w >> 40) * 0x1p-24f; }

__global__ void __launch_bounds__(256) k_km_init(BvhDev bv, int G, float *__restrict__ cent) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= G) return;
    const int64_t sidx = (int64_t)(((double)g + 0.5) * (double)bv.n / (double)G);
    const SurfRec r = bv.rec[min<int64_t>(sidx, bv.n - 1)];
    cent[3 * g + 0] = r.a.x;
    cent[3 * g + 1] = r.a.y;
    cent[3 * g + 2] = r.a.z;
}

__global__ void __launch_bounds__(256) k_km_assign(BvhDev bv, int G, const float *__restrict__ cent,
                                                   uint32_t *__restrict__ key, uint32_t *__restrict__ ids,
                                                   uint32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= bv.n) return;
    const SurfRec r = bv.rec[bv.inv[i]];
    float best = INFINITY;
    int bg = 0;
    for (int g = 0; g < G; ++g) {
        const float dx = r.a.x - cent[3 * g], dy = r.a.y - cent[3 * g + 1], dz = r.a.z - cent[3 * g + 2];
        const float d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < best) {
            best = d2;
            bg = g;
        }
    }
    key[i] = (uint32_t)bg;
    ids[i] = (uint32_t)i;
    atomicAdd(count + bg, 1u);
}

// wave per group: mean centre and mean normal of its members (fixed order);
// an empty group keeps its centre
__global__ void __launch_bounds__(256) k_km_update(BvhDev bv, int G, const int64_t *__restrict__ goff,
                                                   const uint32_t *__restrict__ members, float *__restrict__ cent,
                                                   float *__restrict__ gnrm) {
    const int g = blockIdx.x * 4 + threadIdx.x / 64;
    if (g >= G) return;
    const int lane = __lane_id();
    const int64_t b = goff[g], e = goff[g + 1];
    float s[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = b + lane; k < e; k += 64) {
        const SurfRec r = bv.rec[bv.inv[members[k]]];
        s[0] += r.a.x;
        s[1] += r.a.y;
        s[2] += r.a.z;
        s[3] += r.b.x;
        s[4] += r.b.y;
        s[5] += r.b.z;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
        for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off, 64);
    if (lane == 0 && e > b) {
        const float inv = 1.0f / (float)(e - b);
        cent[3 * g + 0] = s[0] * inv;
        cent[3 * g + 1] = s[1] * inv;
        cent[3 * g + 2] = s[2] * inv;
        gnrm[3 * g + 0] = s[3] * inv;
        gnrm[3 * g + 1] = s[4] * inv;
        gnrm[3 * g + 2] = s[5] * inv;
    }
}

// wave per group: summed luminance of the members' current radiance (the
// DC coefficient of every light)
__global__ void __launch_bounds__(256) k_mc_lum(int G, const int64_t *__restrict__ goff,
                                                const uint32_t *__restrict__ members, const float *__restrict__ B,
                                                int Lt, int K, float *__restrict__ L) {
    const int g = blockIdx.x * 4 + threadIdx.x / 64;
    if (g >= G) return;
    const int lane = __lane_id();
    const int C = Lt * K * 3;
    float s = 0.0f;
    for (int64_t k = goff[g] + lane; k < goff[g + 1]; k += 64) {
        const float *bj = B + (int64_t)members[k] * C;
        for (int l = 0; l < Lt; ++l) s += lum3(bj + l * K * 3);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) L[g] = s;
}

__device__ __forceinline__ float member_weight(const SurfRec &ra, const SurfRec &rj, float lumj) {
    const float vx = rj.a.x - ra.a.x, vy = rj.a.y - ra.a.y, vz = rj.a.z - ra.a.z;
    const float r2 = vx * vx + vy * vy + vz * vz;
    if (!(r2 > 0.0f)) return 0.0f;
    const float ca = fabsf(ra.b.x * vx + ra.b.y * vy + ra.b.z * vz);
    const float cj = fabsf(rj.b.x * vx + rj.b.y * vy + rj.b.z * vz);
    return lumj * (ca * cj) / (r2 * r2);
}

__device__ __forceinline__ float group_weight(const SurfRec &ra, const float *cent, const float *gnrm, float Lg,
                                              float rmin2) {
    const float vx = cent[0] - ra.a.x, vy = cent[1] - ra.a.y, vz = cent[2] - ra.a.z;
    const float r2 = fmaxf(vx * vx + vy * vy + vz * vz, rmin2);
    const float il = 1.0f / sqrtf(r2);
    const float ca = fabsf(ra.b.x * vx + ra.b.y * vy + ra.b.z * vz) * il;
    const float cg = fabsf(gnrm[0] * vx + gnrm[1] * vy + gnrm[2] * vz) * il;
    return Lg * (ca + kMcBeta) * (cg + kMcBeta) / r2;
}

// One next event per slot: receiver recv[slot] (slot itself when recv is
// NULL), current radiance B, writes delta [slots][C].
__global__ void __launch_bounds__(kCenterThreads) k_mc_ne(BvhDev bv, int G, const int64_t *__restrict__ goff,
                                                          const uint32_t *__restrict__ members,
                                                          const float *__restrict__ cent,
                                                          const float *__restrict__ gnrm, const float *__restrict__ Lg,
                                                          float rmin2, const int32_t *__restrict__ recv,
                                                          int64_t slots, const float *__restrict__ lambda,
                                                          const float *__restrict__ rho, const float *__restrict__ E,
                                                          const float *__restrict__ B, int Lt, int K, uint64_t seed,
                                                          int step, float *__restrict__ delta, int *err) {
    extern __shared__ uint32_t stack_mem[];
    const int64_t s = (int64_t)blockIdx.x * kCenterThreads + threadIdx.x;
    if (s >= slots) return;
    const int64_t a = recv ? (int64_t)recv[s] : s;
    const int C = Lt * K * 3;
    const SurfRec ra = bv.rec[bv.inv[a]];
    const float *Ea = E + a * C;
    float *out = delta + s * C;
    uint64_t w[4];
    philox4x64_10((uint64_t)s, (uint64_t)step, 0ull, 2ull, seed, 0ull, w);
    // group: two passes (total, then the inverse CDF)
    float WG = 0.0f;
    for (int g = 0; g < G; ++g) WG += group_weight(ra, cent + 3 * g, gnrm + 3 * g, Lg[g], rmin2);
    int gsel = -1;
    float wg = 0.0f;
    if (WG > 0.0f) {
        const float target = u01(w[0]) * WG;
        float acc = 0.0f;
        for (int g = 0; g < G; ++g) {
            const float x = group_weight(ra, cent + 3 * g, gnrm + 3 * g, Lg[g], rmin2);
            if (x <= 0.0f) continue;
            acc += x;
            gsel = g;
            wg = x;
            if (acc > target) break;
        }
    }
    int64_t jsel = -1;
    float pj = 0.0f;
    if (gsel >= 0) {
        const int64_t b = goff[gsel], e = goff[gsel + 1];
        float Wg = 0.0f;
        for (int64_t k = b; k < e; ++k) {
            const uint32_t j = members[k];
            if ((int64_t)j == a) continue;
            const SurfRec rj = bv.rec[bv.inv[j]];
            float lj = 0.0f;
            for (int l = 0; l < Lt; ++l) lj += lum3(B + (int64_t)j * C + l * K * 3);
            Wg += member_weight(ra, rj, lj);
        }
        if (Wg > 0.0f) {
            const float target = u01(w[1]) * Wg;
            float acc = 0.0f, wj = 0.0f;
            for (int64_t k = b; k < e; ++k) {
                const uint32_t j = members[k];
                if ((int64_t)j == a) continue;
                const SurfRec rj = bv.rec[bv.inv[j]];
                float lj = 0.0f;
                for (int l = 0; l < Lt; ++l) lj += lum3(B + (int64_t)j * C + l * K * 3);
                const float x = member_weight(ra, rj, lj);
                if (x <= 0.0f) continue;
                acc += x;
                jsel = j;
                wj = x;
                if (acc > target) break;
            }
            pj = (wg / WG) * (wj / Wg);
        }
    }
    float scale = 0.0f;
    if (jsel >= 0 && pj > 0.0f) {
        const SurfRec rj = bv.rec[bv.inv[jsel]];
        const Segment g = make_segment(ra, rj, bv.bounds[6]);
        float T = 1.0f;
        trace_segment(bv, g.ox, g.oy, g.oz, g.dx, g.dy, g.dz, (uint32_t)a, (uint32_t)jsel, g.t_lo, g.t_hi,
                      stack_mem + threadIdx.x, kCenterThreads, err, [&](const SurfRec &r) {
                          T = __fmul_rn(T, transmit(r.c.w, kernel_gamma(hit_r2_exact(r, g.ox, g.oy, g.oz, g.dx,
                                                                                     g.dy, g.dz))));
                      });
        const float aa = fabsf(ra.b.x * g.dx + ra.b.y * g.dy + ra.b.z * g.dz);
        const float bb = fabsf(rj.b.x * g.dx + rj.b.y * g.dy + rj.b.z * g.dz);
        const float r2 = g.dx * g.dx + g.dy * g.dy + g.dz * g.dz;
        const float F = lambda[jsel] * (float)bv.area[jsel] * T * (aa * bb) / (r2 * r2) * kInvPi;
        scale = F / pj;
    }
    const float *Bj = jsel >= 0 ? B + jsel * C : nullptr;
    for (int c = 0; c < C; ++c) {
        const float add = Bj ? rho[3 * a + c % 3] * scale * Bj[c] : 0.0f;
        out[c] = Ea[c] + add;
    }
}

// B = S / D per receiver (0 where never visited)
__global__ void __launch_bounds__(256) k_mc_mean(const float *__restrict__ S, const uint32_t *__restrict__ D,
                                                 int64_t n, int C, float *__restrict__ B) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * C) return;
    const uint32_t d = D[t / C];
    B[t] = d ? S[t] / (float)d : 0.0f;
}

// receiver a adds its slots' estimates (slots sorted by receiver; NULL recv:
// slot a is receiver a) in slot order
__global__ void __launch_bounds__(256) k_mc_accum(const int32_t *__restrict__ recv, int64_t slots,
                                                  const float *__restrict__ delta, int64_t n, int C,
                                                  float *__restrict__ S, float *__restrict__ S2,
                                                  uint32_t *__restrict__ D) {
    const int64_t a = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (a >= n) return;
    const int lane = __lane_id();
    int64_t lo = a, hi = a + 1;
    if (recv) {
        int64_t l = 0, h = slots;
        while (l < h) {
            const int64_t m = (l + h) >> 1;
            if (recv[m] < a) l = m + 1;
            else h = m;
        }
        lo = l;
        h = slots;
        while (l < h) {
            const int64_t m = (l + h) >> 1;
            if (recv[m] <= a) l = m + 1;
            else h = m;
        }
        hi = l;
    }
    if (hi <= lo) return;
    for (int c = lane; c < C; c += 64) {
        float s = S[a * C + c], s2 = S2[a * C + c];
        for (int64_t k = lo; k < hi; ++k) {
            const float d = delta[k * C + c];
            s += d;
            s2 = __builtin_fmaf(d, d, s2);
        }
        S[a * C + c] = s;
        S2[a * C + c] = s2;
    }
    if (lane == 0) D[a] += (uint32_t)(hi - lo);
}

// per-receiver variance of the estimates, summed over the columns, and its
// maximum (float bits)
__global__ void __launch_bounds__(256) k_mc_var(const float *__restrict__ S, const float *__restrict__ S2,
                                                const uint32_t *__restrict__ D, int64_t n, int C,
                                                float *__restrict__ var, uint32_t *maxbits) {
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float v = 0.0f;
    if (a < n && D[a] > 0) {
        const float id = 1.0f / (float)D[a];
        for (int c = 0; c < C; ++c) {
            const float m = S[a * C + c] * id;
            v += fmaxf(0.0f, S2[a * C + c] * id - m * m);
        }
        var[a] = v;
    } else if (a < n) {
        var[a] = 0.0f;
    }
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if (__lane_id() == 0 && v > 0.0f) atomicMax(maxbits, __float_as_uint(v));
}

// integer selection weights (variance relative to the maximum, 2^24 levels)
__global__ void __launch_bounds__(256) k_mc_quant(const float *__restrict__ var, const uint32_t *maxbits, int64_t n,
                                                  uint32_t *__restrict__ q) {
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (a >= n) return;
    const float m = __uint_as_float(*maxbits);
    q[a] = m > 0.0f ? (uint32_t)__float2uint_rn(var[a] / m * 16777216.0f) : 1u;
}

// slot s draws its receiver by the stratified inverse of the integer CDF:
// target = floor((s + xi_s) / N * total), receiver = first a with cdf[a+1] > target
__global__ void __launch_bounds__(256) k_mc_draw(const int64_t *__restrict__ cdf, int64_t n, uint64_t seed, int step,
                                                 int32_t *__restrict__ recv) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint64_t total = (uint64_t)cdf[n];
    uint64_t w[4];
    philox4x64_10((uint64_t)s, (uint64_t)step, 1ull, 1ull, seed, 0ull, w);
    // floor((s + w / 2^64) total / n) in integers
    int64_t target = (int64_t)(((uint64_t)s * total + __umul64hi(w[0], total)) / (uint64_t)n);
    if (target >= (int64_t)total) target = (int64_t)total - 1;
    int64_t l = 0, h = n;
    while (l < h) {
        const int64_t m = (l + h) >> 1;
        if (cdf[m + 1] <= target) l = m + 1;
        else h = m;
    }
    recv[s] = (int32_t)min<int64_t>(l, n - 1);
}

// Composited hit list of every ray of the listed receivers (diagnostics and
// parity tests): direction, count, and per hit (j, t, front).
__global__ void __launch_bounds__(256) k_ray_hits(BvhDev bv, int R, uint64_t seed, float t_eps, float t_min,
                                                  const int64_t *__restrict__ recv, int max_hits, float *dirs,
                                                  int32_t *cnt, int32_t *hj, float *ht, int8_t *hf, float *hT, int *err) {
    extern __shared__ uint32_t stack_mem[];
    const int64_t k = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t i = recv[k];
    const SurfRec rr = bv.rec[bv.inv[i]];
    for (int r = tid; r < R; r += blockDim.x) {
        float dx, dy, dz;
        ray_direction(rr.c.x, rr.c.y, rr.c.z, rr.d.x, rr.d.y, rr.d.z, rr.b.x, rr.b.y, rr.b.z, (uint64_t)r,
                      (uint64_t)i, seed, 0, dx, dy, dz);
        const int64_t ray = k * R + r;
        dirs[ray * 3 + 0] = dx;
        dirs[ray * 3 + 1] = dy;
        dirs[ray * 3 + 2] = dz;
        int q = 0;
        const float te = t_eps > 0.0f ? t_eps : bv.bounds[6];
        trace_sorted<kKB>(bv, rr.a.x, rr.a.y, rr.a.z, dx, dy, dz, (uint32_t)i, te, t_min, stack_mem + tid,
                          blockDim.x, err, [&](uint32_t j, float, float T, bool front, float, float t) {
                              if (q < max_hits) {
                                  hj[ray * max_hits + q] = (int32_t)j;
                                  ht[ray * max_hits + q] = t;
                                  hf[ray * max_hits + q] = front ? 1 : 0;
                                  hT[ray * max_hits + q] = T;
                              }
                              ++q;
                          });
        cnt[ray] = q;
    }
}

__global__ void __launch_bounds__(256) k_reflectance(BvhDev bv, const float *__restrict__ albedo, float *rho) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= bv.n) return;
    const float o = bv.op[i];
    rho[3 * i + 0] = o * albedo[3 * i + 0];
    rho[3 * i + 1] = o * albedo[3 * i + 1];
    rho[3 * i + 2] = o * albedo[3 * i + 2];
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
size_t ff_stack_bytes(int threads) { return (size_t)kStackDeep * threads * sizeof(uint32_t); }

gsrad_status launch_ff_trace(const BvhDev &bv, int R, uint64_t seed, float t_eps, float t_min, int64_t s_begin,
                             int64_t count, int by_orig, uint2 *recs, uint32_t *rcnt, int rcap, int deep, int *err,
                             hipStream_t st) {
    const int group = R >= kPoolRays ? 1 : kPoolRays / R;
    const int64_t nblocks = (count + group - 1) / group;
    if (deep) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ff_trace<kStackDeep>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kStackDeep * 256 * 4);
        hipLaunchKernelGGL(k_ff_trace<kStackDeep>, dim3((unsigned)nblocks), dim3(256),
                           (size_t)kStackDeep * 256 * sizeof(uint32_t), st, bv, R, seed, t_eps, t_min, s_begin, count,
                           group, nblocks, by_orig, recs, rcnt, rcap, err);
    } else {
        hipLaunchKernelGGL(k_ff_trace<kStackShallow>, dim3((unsigned)nblocks), dim3(256),
                           (size_t)kStackShallow * 256 * sizeof(uint32_t), st, bv, R, seed, t_eps, t_min, s_begin,
                           count, group, nblocks, by_orig, recs, rcnt, rcap, err);
    }
    return check_hip(hipGetLastError(), "ff trace launch");
}

size_t ff_aggregate_smem(int log2h) { return (size_t)(1 << log2h) * 12; }

gsrad_status launch_ff_aggregate(const BvhDev &bv, const uint2 *recs, const uint32_t *rcnt, int rcap, int64_t s_begin,
                                 int64_t count, int by_orig, int R, int topk, int log2h, int log2h_max,
                                 int32_t *redo_list, uint32_t *redo_cnt, int64_t cap_row, int32_t *ell_col,
                                 float *ell_val, uint32_t *row_len, int *err, hipStream_t st) {
    if (log2h < 8 || log2h > log2h_max || log2h_max > 13) {
        set_error("aggregation table size out of range");
        return GSRAD_EINVAL;
    }
    const bool redo = log2h < log2h_max;
    // a probe chain of 256 slots means a table nearly full (at 7/8 load the
    // mean chain is about 32): such rows are redone with the largest table
    const int max_probe = redo ? 256 : 1 << log2h;
    const size_t smem = ff_aggregate_smem(log2h);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ff_aggregate<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    gsrad_status e;
    if (redo && (e = check_hip(hipMemsetAsync(redo_cnt, 0, 8, st), "aggregate redo counter")) != GSRAD_OK) return e;
    hipLaunchKernelGGL(k_ff_aggregate<false>, dim3((unsigned)count), dim3(256), smem, st, bv, recs, rcnt, rcap,
                       s_begin, by_orig, R, topk, log2h, max_probe, redo ? redo_list : nullptr, redo_cnt, cap_row,
                       ell_col, ell_val, row_len, err);
    if ((e = check_hip(hipGetLastError(), "ff aggregate launch")) != GSRAD_OK || !redo) return e;
    const size_t smem_max = ff_aggregate_smem(log2h_max);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ff_aggregate<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_max);
    // one workgroup per CU holds the largest table; each takes listed rows
    // until the list is drained (none listed: every workgroup exits at once)
    const unsigned grid = (unsigned)std::min<int64_t>(count, 256);
    hipLaunchKernelGGL(k_ff_aggregate<true>, dim3(grid), dim3(256), smem_max, st, bv, recs, rcnt, rcap, s_begin,
                       by_orig, R, topk, log2h_max, 1 << log2h_max, redo_list, redo_cnt, cap_row, ell_col, ell_val,
                       row_len, err);
    return check_hip(hipGetLastError(), "ff aggregate redo launch");
}

gsrad_status launch_ell_to_csr(const int32_t *ell_col, const float *ell_val, int64_t cap_row, const int64_t *row_ptr,
                               int64_t n, int32_t *col, float *val, hipStream_t st) {
    hipLaunchKernelGGL(k_ell_to_csr, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, ell_col, ell_val, cap_row,
                       row_ptr, n, col, val);
    return check_hip(hipGetLastError(), "ell to csr launch");
}

gsrad_status launch_direct(const BvhDev &bv, const float *albedo, const float *lpos, const float *lI, int Lt, int K,
                           float *E, int *err, hipStream_t st) {
    const int64_t total = bv.n * Lt;
    hipLaunchKernelGGL(k_direct, dim3((unsigned)((total + 127) / 128)), dim3(128), ff_stack_bytes(128), st, bv, albedo,
                       lpos, lI, Lt, K, E, err);
    return check_hip(hipGetLastError(), "direct light launch");
}

size_t opacity_acc_bytes(int64_t n) { return (size_t)8 * n * sizeof(unsigned long long) + 256; }

gsrad_status launch_opacity_scale(const float *gF, int64_t nnz, int64_t n, void *acc, hipStream_t st) {
    uint32_t *maxbits = reinterpret_cast<uint32_t *>(static_cast<char *>(acc) + (size_t)8 * n * 8);
    int *e = reinterpret_cast<int *>(maxbits + 1);
    if (gF && nnz > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>((nnz + 255) / 256, 1024);
        hipLaunchKernelGGL(k_absmax, dim3(grid), dim3(256), 0, st, gF, nnz, maxbits);
    }
    hipLaunchKernelGGL(k_fx_exp, dim3(1), dim3(1), 0, st, maxbits, n, e);
    return check_hip(hipGetLastError(), "opacity scale launch");
}

static const int *fx_exp_ptr(const BvhDev &bv, const void *acc) {
    return reinterpret_cast<const int *>(static_cast<const char *>(acc) + (size_t)8 * bv.n * 8 + 4);
}

gsrad_status launch_ff_center(const BvhDev &bv, const Csr &P, const float *lambda, float *val, int *err,
                              hipStream_t st) {
    if (P.n == 0) return GSRAD_OK;
    const int64_t nb = (P.n + 1) / 2;
    hipLaunchKernelGGL(k_ff_center, dim3((unsigned)nb), dim3(kCenterThreads),
                       (size_t)kStackDeep * kCenterThreads * sizeof(uint32_t), st, bv, P.row_ptr, P.col, P.n, lambda,
                       val, nb, P.order, err);
    return check_hip(hipGetLastError(), "centre-to-centre form factor launch");
}


// The fixed-point exponents come from the largest contributions on every
// kScaleStride-th row, with 2^kScaleMargin headroom; the accumulating pass
// records the true maxima, and where one could overflow its field's sums the
// pass runs again with the exact exponents (the host reads one flag).
constexpr int kScaleStride = 64;
constexpr int kScaleMargin = 12;

size_t center_acc_bytes(int64_t n) { return (size_t)8 * kCenterFields * n * 8 + 512; }

// accumulator layout: [8 XCD copies][16 fields][n] u64, then maxbits[16],
// fx[16], the largest scaled contribution of the accumulating pass (as
// float bits) at maxbits[32]
static gsrad_status center_scaled_passes(int64_t n, int64_t count, void *acc, hipStream_t st,
                                         const std::function<void(int pass, int stride)> &run) {
    unsigned long long *a = static_cast<unsigned long long *>(acc);
    uint32_t *maxbits = reinterpret_cast<uint32_t *>(a + (size_t)8 * kCenterFields * n);
    int *fx = reinterpret_cast<int *>(maxbits + kCenterFields);
    run(0, kScaleStride);
    hipLaunchKernelGGL(k_center_exp_count, dim3(1), dim3(64), 0, st, maxbits, count, kScaleMargin, fx);
    run(1, 1);
    uint32_t qbits = 0;
    gsrad_status e = check_hip(hipMemcpyAsync(&qbits, maxbits + 2 * kCenterFields, 4, hipMemcpyDeviceToHost, st),
                               "scale check copy");
    if (e != GSRAD_OK) return e;
    if ((e = check_hip(hipStreamSynchronize(st), "scale check sync")) != GSRAD_OK) return e;
    // every |scaled contribution| times the count below 2^62: no sum overflows
    const double qmax = (double)reinterpret_cast<const float &>(qbits);
    if (!(qmax * (double)count < 4.6e18)) {
        // the sampled rows missed the largest contributions: exact maxima from
        // every row, then the sums again
        const size_t bytes = (size_t)8 * kCenterFields * n * 8;
        if ((e = check_hip(hipMemsetAsync(a, 0, bytes + 3 * kCenterFields * 4, st), "accumulators zero")) !=
            GSRAD_OK)
            return e;
        run(0, 1);
        hipLaunchKernelGGL(k_center_exp_count, dim3(1), dim3(64), 0, st, maxbits, count, 0, fx);
        run(1, 1);
    }
    return check_hip(hipGetLastError(), "scaled passes");
}

gsrad_status launch_center_backward(const BvhDev &bv, const Csr &F, const float *lambda, const float *gF, void *acc,
                                    const CenterOutputs &out, int *err, hipStream_t st) {
    if (F.n == 0) return GSRAD_OK;
    unsigned long long *a = static_cast<unsigned long long *>(acc);
    uint32_t *maxbits = reinterpret_cast<uint32_t *>(a + (size_t)8 * kCenterFields * F.n);
    int *fx = reinterpret_cast<int *>(maxbits + kCenterFields);
    const size_t smem = (size_t)kStackDeep * kCenterThreads * sizeof(uint32_t);
    auto run = [&](int pass, int stride) {
        const int64_t rows = (F.n + stride - 1) / stride;
        const int64_t nb = (rows + 1) / 2;
        if (pass == 0)
            hipLaunchKernelGGL(k_center_bwd<0>, dim3((unsigned)nb), dim3(kCenterThreads), smem, st, bv, F.row_ptr,
                               F.col, F.val, F.n, lambda, gF, maxbits, fx, a, nb, F.order, stride, err);
        else
            hipLaunchKernelGGL(k_center_bwd<1>, dim3((unsigned)nb), dim3(kCenterThreads), smem, st, bv, F.row_ptr,
                               F.col, F.val, F.n, lambda, gF, maxbits, fx, a, nb, F.order, stride, err);
    };
    gsrad_status e = center_scaled_passes(F.n, 2 * F.nnz + 2, acc, st, run);
    if (e != GSRAD_OK) return e;
    const int64_t tot = F.n * kCenterFields;
    hipLaunchKernelGGL(k_center_finish, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a, fx, F.n, out);
    return check_hip(hipGetLastError(), "centre-to-centre backward launch");
}

gsrad_status launch_geometry_rec(const BvhDev &bv, int R, uint64_t seed, const uint2 *recs, const uint32_t *rcnt,
                                 int rcap, const int64_t *row_ptr, const int32_t *col, const float *gF, int max_row,
                                 void *acc, const CenterOutputs &out, hipStream_t st) {
    const int threads = R >= 256 ? 256 : ((R + 63) / 64) * 64;
    int log2h = 4;
    while ((1 << log2h) < 2 * max_row) ++log2h;
    const size_t smem = (size_t)(1 << log2h) * 8;
    if (smem > 150 * 1024) {
        set_error("geometry backward: row of %d entries is too long for the LDS row table", max_row);
        return GSRAD_EINVAL;
    }
    static bool attr_set = false;
    if (!attr_set) {
        for (const void *fn : {reinterpret_cast<const void *>(&k_geometry_rec<0>),
                               reinterpret_cast<const void *>(&k_geometry_rec<1>)})
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
        attr_set = true;
    }
    unsigned long long *a = static_cast<unsigned long long *>(acc);
    uint32_t *maxbits = reinterpret_cast<uint32_t *>(a + (size_t)8 * kCenterFields * bv.n);
    int *fx = reinterpret_cast<int *>(maxbits + kCenterFields);
    auto run = [&](int pass, int stride) {
        const int64_t nb = (bv.n + stride - 1) / stride;
        if (pass == 0)
            hipLaunchKernelGGL(k_geometry_rec<0>, dim3((unsigned)nb), dim3(threads), smem, st, bv, R, seed, recs, rcnt,
                               rcap, nb, row_ptr, col, gF, log2h, maxbits, fx, a, stride);
        else
            hipLaunchKernelGGL(k_geometry_rec<1>, dim3((unsigned)nb), dim3(threads), smem, st, bv, R, seed, recs, rcnt,
                               rcap, nb, row_ptr, col, gF, log2h, maxbits, fx, a, stride);
    };
    gsrad_status e = center_scaled_passes(bv.n, bv.n * (int64_t)R + bv.n, acc, st, run);
    if (e != GSRAD_OK) return e;
    CenterOutputs o15 = out;
    o15.p[15] = nullptr;
    const int64_t tot = bv.n * kCenterFields;
    hipLaunchKernelGGL(k_center_finish, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a, fx, bv.n, o15);
    return check_hip(hipGetLastError(), "geometry backward launch");
}

size_t light_acc_bytes(int64_t n, int Lt) {
    return (size_t)8 * kCenterFields * n * 8 + (size_t)8 * 4 * Lt * 8 + 256;
}

gsrad_status launch_direct_backward(const BvhDev &bv, const float *albedo, const float *lpos, const float *lI, int Lt,
                                    int K, const float *gE, void *acc, float *g_lpos, float *g_lI, float *g_alb,
                                    const CenterOutputs &out, int *err, hipStream_t st) {
    unsigned long long *a = static_cast<unsigned long long *>(acc);
    unsigned long long *la = a + (size_t)8 * kCenterFields * bv.n;
    uint32_t *maxbits = reinterpret_cast<uint32_t *>(la + (size_t)8 * 4 * Lt);
    int *fx = reinterpret_cast<int *>(maxbits + 32);
    const dim3 grid((unsigned)((bv.n + 127) / 128));
    const size_t smem = ff_stack_bytes(128);
    hipLaunchKernelGGL(k_direct_bwd<0>, grid, dim3(128), smem, st, bv, albedo, lpos, lI, Lt, K, gE, maxbits, fx, a, la,
                       g_alb, err);
    hipLaunchKernelGGL(k_light_exp, dim3(1), dim3(64), 0, st, maxbits, bv.n * (int64_t)Lt + bv.n, bv.n, fx);
    hipLaunchKernelGGL(k_direct_bwd<1>, grid, dim3(128), smem, st, bv, albedo, lpos, lI, Lt, K, gE, maxbits, fx, a, la,
                       g_alb, err);
    CenterOutputs o15 = out;
    o15.p[15] = nullptr;
    const int64_t tot = bv.n * kCenterFields;
    hipLaunchKernelGGL(k_center_finish, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a, fx, bv.n, o15);
    hipLaunchKernelGGL(k_light_finish, dim3((unsigned)((4 * Lt + 63) / 64)), dim3(64), 0, st, la, fx, Lt, g_lpos, g_lI);
    return check_hip(hipGetLastError(), "direct light backward launch");
}

// --- Monte-Carlo solver host side ---------------------------------------
gsrad_status mc_kmeans(const BvhDev &bv, int G, int iters, McBuffers &mb, hipStream_t st) {
    const int64_t n = bv.n;
    const unsigned gn = (unsigned)((n + 255) / 256);
    int bits = 1;
    while ((1 << bits) < G) ++bits;
    hipLaunchKernelGGL(k_km_init, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, st, bv, G, mb.cent);
    for (int it = 0; it < iters; ++it) {
        gsrad_status e = check_hip(hipMemsetAsync(mb.count, 0, (size_t)G * 4, st), "k-means counts");
        if (e != GSRAD_OK) return e;
        hipLaunchKernelGGL(k_km_assign, dim3(gn), dim3(256), 0, st, bv, G, mb.cent, mb.key, mb.ids, mb.count);
        if ((e = radix_sort_pairs(mb.key, mb.ids, mb.skey, mb.members, n, bits, mb.rtemp, mb.rtemp_bytes, st)) !=
            GSRAD_OK)
            return e;
        if ((e = exclusive_scan_u32_i64(mb.count, mb.goff, G, mb.stemp, mb.stemp_bytes, st)) != GSRAD_OK) return e;
        hipLaunchKernelGGL(k_km_update, dim3((unsigned)((G + 3) / 4)), dim3(256), 0, st, bv, G, mb.goff, mb.members,
                           mb.cent, mb.gnrm);
    }
    return check_hip(hipGetLastError(), "k-means launch");
}

gsrad_status mc_step(const BvhDev &bv, const McBuffers &mb, int G, float rmin2, const float *lambda, const float *rho,
                     const float *E, const float *B, int Lt, int K, uint64_t seed, int step, const int32_t *recv,
                     float *delta, int *err, hipStream_t st) {
    const int64_t n = bv.n;
    hipLaunchKernelGGL(k_mc_lum, dim3((unsigned)((G + 3) / 4)), dim3(256), 0, st, G, mb.goff, mb.members, B, Lt, K,
                       mb.L);
    hipLaunchKernelGGL(k_mc_ne, dim3((unsigned)((n + kCenterThreads - 1) / kCenterThreads)), dim3(kCenterThreads),
                       (size_t)kStackDeep * kCenterThreads * sizeof(uint32_t), st, bv, G, mb.goff, mb.members, mb.cent,
                       mb.gnrm, mb.L, rmin2, recv, n, lambda, rho, E, B, Lt, K, seed, step, delta, err);
    return check_hip(hipGetLastError(), "next event launch");
}

gsrad_status mc_solve(const BvhDev &bv, const McBuffers &mb, int G, float rmin2, const float *lambda,
                      const float *rho, const float *E, int Lt, int K, int T, uint64_t seed, float *B_out,
                      int *err, hipStream_t st) {
    const int64_t n = bv.n;
    const int C = Lt * K * 3;
    const size_t bytes = (size_t)n * C * 4;
    gsrad_status e;
    if ((e = check_hip(hipMemsetAsync(mb.S, 0, bytes, st), "mc zero")) != GSRAD_OK) return e;
    if ((e = check_hip(hipMemsetAsync(mb.S2, 0, bytes, st), "mc zero")) != GSRAD_OK) return e;
    if ((e = check_hip(hipMemsetAsync(mb.D, 0, (size_t)n * 4, st), "mc zero")) != GSRAD_OK) return e;
    const unsigned gv = (unsigned)((n * C + 255) / 256), gn = (unsigned)((n + 255) / 256);
    for (int t = 0; t < T; ++t) {
        hipLaunchKernelGGL(k_mc_mean, dim3(gv), dim3(256), 0, st, mb.S, mb.D, n, C, mb.B);
        const int32_t *recv = nullptr;
        if (t >= 8) {
            if ((e = check_hip(hipMemsetAsync(mb.maxbits, 0, 4, st), "mc max")) != GSRAD_OK) return e;
            hipLaunchKernelGGL(k_mc_var, dim3(gn), dim3(256), 0, st, mb.S, mb.S2, mb.D, n, C, mb.var, mb.maxbits);
            hipLaunchKernelGGL(k_mc_quant, dim3(gn), dim3(256), 0, st, mb.var, mb.maxbits, n, mb.q);
            if ((e = exclusive_scan_u32_i64(mb.q, mb.cdf, n, mb.stemp, mb.stemp_bytes, st)) != GSRAD_OK) return e;
            hipLaunchKernelGGL(k_mc_draw, dim3(gn), dim3(256), 0, st, mb.cdf, n, seed, t, mb.recv);
            recv = mb.recv;
        }
        if ((e = mc_step(bv, mb, G, rmin2, lambda, rho, E, mb.B, Lt, K, seed, t, recv, mb.delta, err, st)) != GSRAD_OK)
            return e;
        hipLaunchKernelGGL(k_mc_accum, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, recv, n, mb.delta, n, C,
                           mb.S, mb.S2, mb.D);
    }
    hipLaunchKernelGGL(k_mc_mean, dim3(gv), dim3(256), 0, st, mb.S, mb.D, n, C, B_out);
    return check_hip(hipGetLastError(), "mc solve launch");
}

gsrad_status launch_direct_sh(const BvhDev &bv, const float *R, const float *lpos, const float *lI, int Lt, int K,
                              float *E, int *err, hipStream_t st) {
    const int64_t total = bv.n * Lt;
    const dim3 grid((unsigned)((total + 127) / 128));
    const size_t smem = ff_stack_bytes(128);
    switch (K) {
        case 1: hipLaunchKernelGGL(k_direct_sh<1>, grid, dim3(128), smem, st, bv, R, lpos, lI, Lt, E, err); break;
        case 4: hipLaunchKernelGGL(k_direct_sh<4>, grid, dim3(128), smem, st, bv, R, lpos, lI, Lt, E, err); break;
        case 9: hipLaunchKernelGGL(k_direct_sh<9>, grid, dim3(128), smem, st, bv, R, lpos, lI, Lt, E, err); break;
        case 16: hipLaunchKernelGGL(k_direct_sh<16>, grid, dim3(128), smem, st, bv, R, lpos, lI, Lt, E, err); break;
        default: set_error("direct light: K must be 1, 4, 9 or 16"); return GSRAD_EINVAL;
    }
    return check_hip(hipGetLastError(), "SH direct light launch");
}

gsrad_status launch_opacity_bwd(const BvhDev &bv, int R, uint64_t seed, float t_eps, float t_min,
                                const int64_t *row_ptr, const int32_t *col, const float *gF, int max_row, float2 *wbuf,
                                void *acc, int pass, const uint32_t *rcnt, int rcap, int *err, hipStream_t st) {
    const int threads = R >= 256 ? 256 : ((R + 63) / 64) * 64;
    const size_t smem = (size_t)max_row * 8 + ff_stack_bytes(threads);
    static bool attr_set = false;
    if (!attr_set) {
        hipFuncSetAttribute(reinterpret_cast<const void *>(&k_opacity_bwd), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024 - 4096);
        attr_set = true;
    }
    hipLaunchKernelGGL(k_opacity_bwd, dim3((unsigned)bv.n), dim3(threads), smem, st, bv, R, seed, t_eps, t_min, bv.n,
                       row_ptr, col, gF, max_row, wbuf, fx_exp_ptr(bv, acc),
                       static_cast<unsigned long long *>(acc), pass, rcnt, rcap, err);
    return check_hip(hipGetLastError(), "opacity backward launch");
}

gsrad_status launch_opacity_rec(const BvhDev &bv, int R, const uint2 *recs, const uint32_t *rcnt, int rcap,
                                const int64_t *row_ptr, const int32_t *col, const float *gF, int max_row,
                                void *acc, hipStream_t st) {
    const int threads = R >= 256 ? 256 : ((R + 63) / 64) * 64;
    int log2h = 4;
    while ((1 << log2h) < 2 * max_row) ++log2h;
    const size_t smem = (size_t)(1 << log2h) * 8;
    static bool attr_set = false;
    if (!attr_set) {
        hipFuncSetAttribute(reinterpret_cast<const void *>(&k_opacity_rec), hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024 - 4096);
        attr_set = true;
    }
    if (smem > 150 * 1024) {
        set_error("opacity backward: row of %d entries is too long for the LDS row table", max_row);
        return GSRAD_EINVAL;
    }
    hipLaunchKernelGGL(k_opacity_rec, dim3((unsigned)bv.n), dim3(threads), smem, st, bv, R, recs, rcnt, rcap, bv.n,
                       row_ptr, col, gF, log2h, fx_exp_ptr(bv, acc), static_cast<unsigned long long *>(acc));
    return check_hip(hipGetLastError(), "opacity records launch");
}

gsrad_status launch_opacity_finish(const BvhDev &bv, const void *acc, const float *grad_rho, const float *albedo,
                                   float *grad_o, float *grad_a, hipStream_t st) {
    hipLaunchKernelGGL(k_opacity_finish, dim3((unsigned)((bv.n + 255) / 256)), dim3(256), 0, st, bv,
                       static_cast<const unsigned long long *>(acc), fx_exp_ptr(bv, acc), grad_rho, albedo, grad_o,
                       grad_a);
    return check_hip(hipGetLastError(), "opacity finish launch");
}

gsrad_status launch_ray_hits(const BvhDev &bv, int R, uint64_t seed, float t_eps, float t_min, const int64_t *recv,
                             int64_t n_recv, int max_hits, float *dirs, int32_t *cnt, int32_t *hj, float *ht,
                             int8_t *hf, float *hT, int *err, hipStream_t st) {
    const int threads = R >= 256 ? 256 : ((R + 63) / 64) * 64;
    hipLaunchKernelGGL(k_ray_hits, dim3((unsigned)n_recv), dim3(threads), ff_stack_bytes(threads), st, bv, R, seed,
                       t_eps, t_min, recv, max_hits, dirs, cnt, hj, ht, hf, hT, err);
    return check_hip(hipGetLastError(), "ray hits launch");
}

gsrad_status launch_reflectance(const BvhDev &bv, const float *albedo, float *rho, hipStream_t st) {
    hipLaunchKernelGGL(k_reflectance, dim3((unsigned)((bv.n + 255) / 256)), dim3(256), 0, st, bv, albedo, rho);
    return check_hip(hipGetLastError(), "reflectance launch");
}

}  // namespace gsrad
