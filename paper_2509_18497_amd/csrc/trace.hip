// Ray casting through the surfel LBVH with alpha compositing.
//
// k_ff_trace      one workgroup per group of receivers, lanes taking rays
//                 from a direction-sorted pool: multi-round k-buffer
//                 traversal (the KB nearest hits beyond the last composited
//                 key per round, keys (t, j)), front-to-back compositing,
//                 every composited hit recorded per ray.
// k_ff_aggregate  one workgroup per receiver: replays the records (two
//                 threads per ray when they fit), LDS hash
//                 table with 2^-40 fixed-point sums (integer adds are order
//                 independent, so F is bit-deterministic), radix select of
//                 the top-k entries, bitonic sort by column, one ELL row.
// k_direct        one thread per (surfel, light): shadow-ray transmittance.
// k_opacity_bwd   compositing backward, two recomputing passes.
#include "gsrad_internal.h"
#include "sh_api.h"
#include "sh_basis.h"
#include "trace_api.h"
#include "traverse.h"

namespace gsrad {

namespace {

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

// pools of 256 rays (two receivers at R = 128): on the 100k fruit bowl the
// trace took 53.7 ms, against 54.3 (512), 55.4 (1024), 58.0 (2048)
constexpr int kPoolBits = 8;
constexpr int kPoolRays = 1 << kPoolBits;   // rays sorted and pooled per batch
constexpr int kCompChunk = 5;     // buffered hits whose kernel values are found together
// a wave composites once kFlushNum / kFlushDen of its lanes holding rays wait
constexpr int kFlushNum = 3, kFlushDen = 8;
// leaf children found by a node step wait in a per-lane queue of kLeafQ;
// a wave tests one queued leaf per lane once kLeafNum / kLeafDen of its
// lanes holding rays have one (or a queue is full, or no lane can step), so
// the costly leaf test and k-buffer insertion run with more lanes at once.
// Measured on the 100k fruit bowl: queues of 8 and a composite at 3/8 best
// (queue 6: +0.6 ms; composite at 1/2: +1.4 ms, at 1/4: +3.7 ms; leaf
// steps at 3/4 as good as at 1/2, at 1/4 +6 ms).
constexpr int kLeafQ = 8;
constexpr int kLeafNum = 1, kLeafDen = 2;

// Lane index within the wave, recomputed at each use (volatile: not hoisted
// out of the traversal loop into a register of its own).
__device__ __forceinline__ int lane_index() {
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// Every composited hit of ray r of the receiver in slot `slot` is recorded
// as (j, +-gamma), the sign being the front face, at
// recs[(slot*rcap + q)*R + r] (hit-major inside a receiver, so a wave
// touches one record per lane with one coalesced access); rcnt[slot*R + r]
// is the number of composited hits (more than rcap: records incomplete).
// slot = original index i when the records of all receivers are kept,
// else the receiver's position in the current chunk.
//
// The next pool for a workgroup on XCD xcd: each XCD has its own share of
// the pools, [npools * x / 8, npools * (x + 1) / 8) for XCD x, taken in
// order through the counter queue[64 * x] (one per 256-byte line); once its
// own share is taken it takes from the other XCDs' shares, so every pool is
// traced whatever XCDs the workgroups run on.  kNoPool once all are taken.
constexpr uint32_t kNoPool = 0xffffffffu;

__device__ __forceinline__ uint32_t next_pool(uint32_t *queue, int64_t npools, int xcd) {
    for (int t = 0; t < 8; ++t) {
        const int x = (xcd + t) & 7;
        const uint32_t lo = (uint32_t)((npools * x) / 8), hi = (uint32_t)((npools * (x + 1)) / 8);
        if (lo >= hi) continue;
        const uint32_t v = lo + atomicAdd(queue + 64 * x, 1u);
        if (v < hi) return v;
    }
    return kNoPool;
}

// Rays come in pools of pool_rays <= kPoolRays (ray id = receiver * R + r
// over the chunk's receivers in Morton order: the rays of kPoolRays / R
// consecutive receivers, or kPoolRays rays of one receiver when R is
// larger), sorted by direction key by k_ray_pools into
// list[pool * kPoolRays + p] = (ray index in the pool, direction).
//
// The trace workgroups are persistent and take pools through next_pool.  A
// workgroup's lanes pull rays from its current pool through one 64-bit LDS
// word, (pool, rays handed out), with one atomic add per wave, so
// neighbouring lanes trace rays that leave close origins in close
// directions.  The single pull whose range covers the pool's end installs
// the next pool (an exchange of the word); pulls between the two find no
// ray and are repeated, so the lanes that are done take rays of the next
// pool while the last rays of the current one are traced.  Every ray of a
// pool is handed out once before its successor is installed, every pool is
// installed once, and a wave ends when all of its lanes have found kNoPool
// and hold no ray.
//
// Each lane walks its ray one node per iteration, queueing the leaves it
// reaches; the wave tests queued leaves once half of its lanes hold one; a
// lane whose k-buffer round ends waits until enough lanes of its wave
// wait, the wave then composites them together, and a lane whose ray ends
// takes the next ray at once (the same hits, composited in the same order,
// as the plain per-ray walk).  Three waves per SIMD (at most 168 VGPRs),
// held by a launch bound; four (at most 128) were measured no faster.
template <int STK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) k_ff_trace(BvhDev bv, int R, float t_eps, float t_min,
                                                  int64_t s_begin, int64_t count, int pool_rays, int64_t npools,
                                                  const uint4 *__restrict__ list, uint32_t *queue,
                                                  int by_orig, uint2 *__restrict__ recs,
                                                  uint32_t *__restrict__ rcnt, int rcap, int *err) {
    extern __shared__ uint32_t stack_mem[];
    // the workgroup's current pool (high word; kNoPool: none left) and the
    // rays taken from it (low word)
    __shared__ unsigned long long pq;
    const int tid = threadIdx.x;
    const int xcd = xcc_id();
    if (tid == 0) pq = (unsigned long long)next_pool(queue, npools, xcd) << 32;
    __syncthreads();
    {
        // Lanes hold rays in one of two states: traversing (one node or one
        // queued leaf per iteration of the inner loop) or waiting, their
        // k-buffer round done, to composite.  Compositing is costly per hit (the FP64 hit point,
        // two exponentials), so the wave composites its waiting lanes
        // together, once they are kFlushNum / kFlushDen of the lanes holding
        // rays or no lane traverses.  The node steps have a loop of their
        // own: the k-buffer then stays in the same registers from step to
        // step (merged with the refill and compositing paths, the compiler
        // copied it at every step).
        const int lane = (int)__lane_id();
        const int wave_base = __builtin_amdgcn_readfirstlane(tid & ~63);
        bool have = false, trav = false, drained = false;
        uint32_t i = 0, q = 0;
        uint2 *rec_out = nullptr;
        uint32_t *cnt_out = nullptr;
        float ox = 0.0f, oy = 0.0f, oz = 0.0f, dx = 0.0f, dy = 0.0f, dz = 0.0f, ix = 0.0f, iy = 0.0f, iz = 0.0f;
        float T = 1.0f, t0 = 0.0f, t1 = INFINITY;
        uint64_t last = 0;
        double key[kKB];
#pragma unroll
        for (int k = 0; k < kKB; ++k) key[k] = __longlong_as_double((long long)kKeyEmpty);
        int found = 0, sp = 0, node = 0;
        // queued leaves (LIFO; the order of the leaf tests does not change
        // the round's buffer: it keeps the KB smallest keys whatever the
        // order), and whether the round's walk of the tree is done
        int lq[kLeafQ];
#pragma unroll
        for (int k = 0; k < kLeafQ; ++k) lq[k] = 0;
        int qn = 0;
        bool walked = false;
        // a new k-buffer round from the root, beyond the last composited key
        auto start_round = [&]() {
#pragma unroll
            for (int k = 0; k < kKB; ++k) key[k] = __longlong_as_double((long long)kKeyEmpty);
            found = 0;
            t0 = (last ? __uint_as_float((uint32_t)(last >> 32)) : t_eps) * 0.99999f;
            t1 = INFINITY;
            sp = 0;
            node = 0;
            qn = 0;
            walked = false;
            trav = true;
        };
        auto end_ray = [&]() {
            *cnt_out = q;
            if (q > (uint32_t)rcap) {
                atomicOr(err, kErrRecords);
                atomicMax(err + 3, (int)q);
            }
            have = false;
            trav = false;
        };
        for (;;) {
            // lanes without a ray take the next ones of the pool (one LDS
            // atomic per wave)
            const bool need = !have && !drained;
            const uint64_t needm = __ballot(need);
            if (needm) {
                const int leader = __ffsll((unsigned long long)needm) - 1;
                const uint32_t cnt = (uint32_t)__popcll(needm);
                unsigned long long old = 0;
                if (lane == leader) old = atomicAdd(&pq, (unsigned long long)cnt);
                const uint32_t pool = (uint32_t)__shfl((int)(uint32_t)(old >> 32), leader, 64);
                const uint32_t b0 = (uint32_t)__shfl((int)(uint32_t)old, leader, 64);
                if (pool == kNoPool) {
                    drained = need || drained;   // every pool is taken
                } else {
                    const int64_t id0 = (int64_t)pool * pool_rays;   // the pool's first ray
                    const uint32_t pnb = (uint32_t)min<int64_t>(pool_rays, count * R - id0);
                    // the one pull that covers the pool's end installs the
                    // next pool (pulls after it, until then, find none)
                    if (lane == leader && b0 <= pnb && pnb < b0 + cnt)
                        atomicExch(&pq, (unsigned long long)next_pool(queue, npools, xcd) << 32);
                    const uint32_t p = b0 + (uint32_t)__popcll(needm & ((1ull << lane) - 1ull));
                    if (need && p < pnb) {
                        const uint4 ent = list[(int64_t)pool * kPoolRays + p];
                        const int64_t id = id0 + (int64_t)ent.x;
                        const int64_t recv = id / R;   // chunk-relative receiver
                        const int r = (int)(id % R);
                        const SurfRec rr = bv.rec[s_begin + recv];
                        i = __float_as_uint(rr.d.w);
                        const int64_t slot = by_orig ? (int64_t)i : recv;
                        rec_out = recs + slot * rcap * R + r;
                        cnt_out = rcnt + slot * R + r;
                        ox = rr.a.x;
                        oy = rr.a.y;
                        oz = rr.a.z;
                        dx = __uint_as_float(ent.y);
                        dy = __uint_as_float(ent.z);
                        dz = __uint_as_float(ent.w);
                        ix = safe_inv(dx);
                        iy = safe_inv(dy);
                        iz = safe_inv(dz);
                        q = 0;
                        T = 1.0f;
                        last = 0;
                        have = true;
                        start_round();
                    }
                }
            }
            const int nact = __popcll(__ballot(have));
            if (nact == 0 && !__ballot(!drained)) break;
            if (nact == 0) continue;   // the next pool is being installed
            const int nwait = __popcll(__ballot(have && !trav));
            if (nwait > 0 && (kFlushDen * nwait >= kFlushNum * nact || nwait == nact)) {
                if (have && !trav) {
                    // kernel values (FP64 hit point) and faces of the buffered
                    // hits, kCompChunk at a time (a scheduling barrier between
                    // chunks keeps the loads of later chunks from being
                    // issued early, which would need more registers than
                    // the lane's traversal state leaves), front-to-back
                    // compositing and the records
                    const int m = found < kKB ? found : kKB;
                    bool done = false;
#pragma unroll
                    for (int c0 = 0; c0 < kKB; c0 += kCompChunk) {
                        if (!__any(c0 < m && !done)) break;
                        float gam[kCompChunk];
#pragma unroll
                        for (int k = 0; k < kCompChunk; ++k) {
                            gam[k] = 0.0f;
                            if (c0 + k < m && !done) {
                                const SurfRec h = bv.rec[bv.inv[(uint32_t)key_bits(key[c0 + k])]];
                                const float den = __builtin_fmaf(dz, h.b.z, __builtin_fmaf(dy, h.b.y, __fmul_rn(dx, h.b.x)));
                                const float g = kernel_gamma(hit_r2_exact(h, ox, oy, oz, dx, dy, dz));
                                gam[k] = den < 0.0f ? g : -g;
                            }
                        }
#pragma unroll
                        for (int k = 0; k < kCompChunk; ++k) {
                            if (c0 + k < m && !done) {
                                const uint32_t j = (uint32_t)key_bits(key[c0 + k]);
                                const float g = fabsf(gam[k]);
                                const float x = __fmul_rn(bv.c[j], g);
                                if (q < (uint32_t)rcap)
                                    rec_out[(int64_t)q * R] = make_uint2(j, __float_as_uint(gam[k] > 0.0f ? g : -g));
                                ++q;
                                T = __fmul_rn(T, exp_fx(-x));
                                done = T < t_min;
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    // a full buffer pruned every box beyond its last entry,
                    // so more hits may exist: only a buffer that did not fill
                    // ends the ray
                    if (done || found < kKB) {
                        end_ray();
                    } else {
                        last = key_bits(key[kKB - 1]);
                        start_round();
                    }
                }
                continue;
            }
            // node and leaf steps until a flush is due or a lane needs a ray
            for (;;) {
                const bool can = trav && !walked && qn <= kLeafQ - 2;
                const int nq = __popcll(__ballot(qn > 0));
                const bool leaf_step =
                    nq > 0 && (kLeafDen * nq >= kLeafNum * nact || !__ballot(can) || __ballot(qn > kLeafQ - 2));
                // per-lane conditions (a uniform if / else here made the
                // compiler copy the k-buffer between register sets)
                const bool do_leaf = leaf_step && qn > 0, do_node = !leaf_step && can;
                if (do_leaf) {
                    --qn;
                    int s = lq[0];
#pragma unroll
                    for (int k = 1; k < kLeafQ; ++k) s = qn == k ? lq[k] : s;
                    visit_leaf<kKB>(bv.rec, s, i, ox, oy, oz, dx, dy, dz, t_eps, last, key, found, t1);
                }
                if (do_node) {
                    const Node nd = bv.nodes[node];
                    float tn0, tn1;
                    bool h0 = slab(nd.b0.x, nd.b0.y, nd.b0.z, nd.b0.w, nd.b1.x, nd.b1.y, ox, oy, oz, ix, iy, iz, t0, t1, tn0);
                    bool h1 = slab(nd.b1.z, nd.b1.w, nd.b2.x, nd.b2.y, nd.b2.z, nd.b2.w, ox, oy, oz, ix, iy, iz, t0, t1, tn1);
                    const int c0 = nd.ch.x, c1 = nd.ch.y;
                    auto queue_leaf = [&](int leaf) {
#pragma unroll
                        for (int k = 0; k < kLeafQ; ++k) lq[k] = qn == k ? leaf : lq[k];
                        ++qn;
                    };
                    if (h0 && c0 < 0) {
                        queue_leaf(~c0);
                        h0 = false;
                    }
                    if (h1 && c1 < 0) {
                        queue_leaf(~c1);
                        h1 = false;
                    }
                    // descend into the nearer hit child and push the other;
                    // with no child left, pop; an empty stack ends the walk
                    // (the round ends once the queued leaves are tested too).
                    // A push past the stack's end ends the ray with an error
                    // (the launch is repeated with the deep stack).
                    const bool both = h0 && h1;
                    const bool n0 = !h1 || (h0 && tn0 <= tn1);
                    const bool ovf = both && sp >= STK;
                    // the lane's stack column: the wave's base (uniform) plus
                    // the lane index, read again here rather than held in a
                    // register across the loop
                    uint32_t *stack = stack_mem + wave_base + lane_index();
                    if (both) stack[min(sp, STK - 1) * 256] = (uint32_t)(n0 ? c1 : c0);
                    sp += both ? 1 : 0;
                    node = n0 ? c0 : c1;
                    if (!h0 && !h1) {
                        if (sp == 0) walked = true;
                        else {
                            --sp;
                            node = (int)stack[sp * 256];
                        }
                    }
                    if (ovf) {
                        atomicOr(err, kErrStack);
                        end_ray();
                        qn = 0;
                    }
                }
                if (trav && walked && qn == 0) trav = false;   // the round's hits are all tested
                const int nw = __popcll(__ballot(have && !trav));
                if ((nw > 0 && (kFlushDen * nw >= kFlushNum * nact || nw == nact)) || __ballot(!have && !drained)) break;
            }
        }
    }
}

// The ray pools of the trace: pool b holds the rays [b * pool_rays,
// (b + 1) * pool_rays) of the chunk (ray id = receiver * R + r), their
// directions generated and sorted by direction key (ties by ray index),
// written as
// list[b * kPoolRays + p] = (ray index in the pool, direction).  Block 0 also
// resets the trace's per-XCD pool counters.  A scene of one surfel has no
// node to walk and every ray starts in its own receiver, which the walk
// skips: its rays record no hit here and the trace is not run.
__global__ void __launch_bounds__(256) k_ray_pools(BvhDev bv, int R, uint64_t seed, int64_t s_begin, int64_t count,
                                                   int pool_rays, int by_orig, uint4 *__restrict__ list,
                                                   uint32_t *__restrict__ queue, uint32_t *__restrict__ rcnt) {
    __shared__ uint32_t pool_key[kPoolRays];
    __shared__ float pool_d[kPoolRays][3];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    if (b == 0 && tid < 8) queue[64 * tid] = 0;
    const int64_t id0 = b * pool_rays;
    const int nb = (int)min<int64_t>(pool_rays, count * R - id0);
    if (bv.n == 1) {
        for (int k = tid; k < nb; k += 256) {
            const int64_t recv = (id0 + k) / R;
            const int64_t slot = by_orig ? (int64_t)__float_as_uint(bv.rec[s_begin + recv].d.w) : recv;
            rcnt[slot * R + (id0 + k) % R] = 0;
        }
        return;
    }
    int P = 1;
    while (P < nb) P <<= 1;
    for (int k = tid; k < P; k += 256) {
        uint32_t key = 0xffffffffu;
        if (k < nb) {
            const int64_t id = id0 + k;
            const SurfRec rr = bv.rec[s_begin + id / R];
            float dx, dy, dz;
            ray_direction(rr.c.x, rr.c.y, rr.c.z, rr.d.x, rr.d.y, rr.d.z, rr.b.x, rr.b.y, rr.b.z, (uint64_t)(id % R),
                          (uint64_t)__float_as_uint(rr.d.w), seed, 0, dx, dy, dz);
            pool_d[k][0] = dx;
            pool_d[k][1] = dy;
            pool_d[k][2] = dz;
            key = (dir_key(dx, dy, dz) << kPoolBits) | (uint32_t)k;
        }
        pool_key[k] = key;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += 256) {
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
    for (int p = tid; p < nb; p += 256) {
        const int k = (int)(pool_key[p] & (uint32_t)(kPoolRays - 1));
        list[b * kPoolRays + p] = make_uint4((uint32_t)k, __float_as_uint(pool_d[k][0]), __float_as_uint(pool_d[k][1]),
                                             __float_as_uint(pool_d[k][2]));
    }
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
    __shared__ uint32_t hist[256], wsum[4], dsel, before_sh, dcnt, habort, ticket;
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
    // Two threads per ray when 2R <= 256: the first inserts the ray's first
    // half of the hits, the second its second half, starting from the
    // transmittance it finds by multiplying through the first half in the
    // same order (so T is bit-identical to one thread's walk).
    const int split = 2 * R <= 256 ? 2 : 1;
    for (int t = tid; t < split * R; t += 256) {
        const int r = t % R, h = t / R;
        const uint32_t m = min(rcnt[slot * R + r], (uint32_t)rcap);
        const uint2 *in = recs + slot * rcap * R + r;
        const uint32_t qmid = split == 2 ? (m + 1) / 2 : 0;
        const uint32_t qa = h == 0 ? 0 : qmid, qb = (split == 2 && h == 0) ? qmid : m;
        float T = 1.0f;
        for (uint32_t q = 0; q < qa; ++q) {
            const uint2 hq = in[(int64_t)q * R];
            T = __fmul_rn(T, exp_fx(-(bv.c[hq.x] * fabsf(__uint_as_float(hq.y)))));
        }
        // the record one step ahead and its sender's c, the record two
        // steps ahead: each load has a record's work to land
        uint2 h1 = qa < qb ? in[(int64_t)qa * R] : make_uint2(0u, 0u);
        uint2 h2 = qa + 1 < qb ? in[(int64_t)(qa + 1) * R] : make_uint2(0u, 0u);
        float c1 = qa < qb ? bv.c[h1.x] : 0.0f;
        for (uint32_t q = qa; q < qb; ++q) {
            if ((q & 7) == 0 && *abort_v) break;
            const uint2 hr = h1;
            const float cq = c1;
            h1 = h2;
            if (q + 2 < qb) h2 = in[(int64_t)(q + 2) * R];
            if (q + 1 < qb) c1 = bv.c[h1.x];
            const float gs = __uint_as_float(hr.y);
            const float x = cq * fabsf(gs);
            if (gs > 0.0f) {
                const float w = -expm1f(-x) * T;
                const unsigned long long fx = (unsigned long long)__float2ull_rn(w * kFixScaleF);
                uint32_t hs = hash_slot(hr.x, log2h);
                int probe = 0;
                for (; probe < max_probe; ++probe) {
                    const uint32_t prev = atomicCAS(&hkey[hs], kEmpty, hr.x);
                    if (prev == kEmpty || prev == hr.x) {
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
                        dcnt = c4[q];
                    }
                    run += c4[q];
                }
            }
            __syncthreads();
            prefix |= (uint64_t)dsel << shift;
            pmask |= 255ull << shift;
            need -= before_sh;
            const uint32_t in_bucket = dcnt;
            __syncthreads();
            // the topk-th key is the largest of the selected digit's keys:
            // all of them are kept, the lower digits need no pass
            if (need == in_bucket) {
                prefix |= ~pmask;
                break;
            }
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
    // A stage of stride below 64 pairs entries within the 128-entry span
    // t / 64 of each of its pair indices t, which only one wave takes: such
    // a stage needs a workgroup barrier only next to a stage of a wider
    // stride, a wave's own order otherwise.
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            const uint32_t next = stride > 1 ? stride >> 1 : (2 * size <= P ? size : 0);
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
            if (stride >= 64 || next >= 64) {
                __syncthreads();
            } else {
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __syncthreads();
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
// One hit of the second walk: the sender's contribution to dL/do.
// The same with the sender's c_j and raw opacity already loaded.
__device__ __forceinline__ void opacity_hit_c(uint32_t j, float G, float alpha, float f, float T, float g, float cj,
                                              float oraw, DF W, DF &P, unsigned long long *acc, float scale) {
    if (G != 0.0f) P = df_add(P, df_prod3(G, alpha, T));
    if (!(oraw > 0.0f && oraw < kOpacityMax)) return;
    const DF Sd = df_add(W, DF{-P.hi, -P.lo});
    const float dLda = G * T - Sd.hi / f;
    const float dado = g * expf(cj * (1.0f - g));
    fx_add(acc + j, dLda * dado, scale);
}

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
    // With one ray per thread, the threads take the rays in ascending order
    // of their record counts (a counting sort on min(count, 63); rays past
    // the cap count as 0), so that each wave's rays are alike in length.
    // Which thread takes a ray changes no sum: the per-ray arithmetic is
    // the ray's own and the fixed-point adds commute.
    __shared__ uint32_t bucket[64], ray_of[256];
    const bool by_len = R == (int)blockDim.x;
    if (by_len && tid < 64) bucket[tid] = 0;
    for (int k = tid; k < H; k += blockDim.x) hk[k] = kEmpty;
    __syncthreads();
    uint32_t bk = 0;
    if (by_len) {
        const uint32_t m0 = rcnt[(int64_t)i * R + tid];
        bk = m0 > (uint32_t)rcap ? 0u : min(m0, 63u);
        atomicAdd(&bucket[bk], 1u);
    }
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
    if (by_len) {
        if (tid < 64) {
            const uint32_t v = bucket[tid];
            bucket[tid] = wave_incl_scan_u32(v) - v;
        }
        __syncthreads();
        ray_of[atomicAdd(&bucket[bk], 1u)] = (uint32_t)tid;
        __syncthreads();
    }
    for (int t = tid; t < R; t += blockDim.x) {
        const int r = by_len ? (int)ray_of[t] : t;
        const uint32_t m = rcnt[(int64_t)i * R + r];
        if (m > (uint32_t)rcap) continue;
        const uint2 *in = recs + (int64_t)i * rcap * R + r;
        // Records are loaded two hits ahead and the sender's constants one
        // ahead.  In the second pass those loads are issued before the
        // current hit's atomic add: the memory counter the waits use is in
        // order, so a load issued after an atomic could only be waited for
        // together with the atomic.
        DF W{0.0f, 0.0f};
        float T = 1.0f;
        {
            uint2 h1 = m > 0 ? in[0] : make_uint2(0u, 0u);
            uint2 h2 = m > 1 ? in[(int64_t)R] : make_uint2(0u, 0u);
            float c1 = m > 0 ? bv.c[h1.x] : 0.0f;
            for (uint32_t q = 0; q < m; ++q) {
                const uint2 h = h1;
                const float cq = c1;
                h1 = h2;
                if (q + 2 < m) h2 = in[(int64_t)(q + 2) * R];
                if (q + 1 < m) c1 = bv.c[h1.x];
                const float gs = __uint_as_float(h.y);
                const float x = cq * fabsf(gs);
                if (gs > 0.0f) {
                    const float G = row_hash_lookup(hk, hv, log2h, h.x);
                    if (G != 0.0f) W = df_add(W, df_prod3(G, -expm1f(-x), T));
                }
                T = __fmul_rn(T, exp_fx(-x));
            }
        }
        if (W.hi == 0.0f) continue;   // every G_q alpha_q T_q is 0: no contribution
        DF P{0.0f, 0.0f};
        T = 1.0f;
        uint2 h1 = in[0];
        uint2 h2 = m > 1 ? in[(int64_t)R] : make_uint2(0u, 0u);
        float c1 = bv.c[h1.x], o1 = bv.raw_op[h1.x];
        for (uint32_t q = 0; q < m; ++q) {
            const uint2 h = h1;
            const float cq = c1, oq = o1;
            h1 = h2;
            if (q + 2 < m) h2 = in[(int64_t)(q + 2) * R];
            if (q + 1 < m) {
                c1 = bv.c[h1.x];
                o1 = bv.raw_op[h1.x];
            }
            const float gs = __uint_as_float(h.y);
            const float g = fabsf(gs);
            const float x = cq * g;
            const float f = exp_fx(-x);
            const float G = gs > 0.0f ? row_hash_lookup(hk, hv, log2h, h.x) : 0.0f;
            opacity_hit_c(h.x, G, -expm1f(-x), f, T, g, cq, oq, W, P, my, scale);
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

size_t ff_pool_list_bytes(int64_t count, int R) {
    const int pool_rays = R >= kPoolRays ? kPoolRays : (kPoolRays / R) * R;
    const int64_t npools = (count * R + pool_rays - 1) / pool_rays;
    return (size_t)npools * kPoolRays * sizeof(uint4) + 8 * 256;
}

gsrad_status launch_ray_pools(const BvhDev &bv, int R, uint64_t seed, int64_t s_begin, int64_t count, int by_orig,
                              uint32_t *rcnt, void *pools, hipStream_t st) {
    if (count <= 0) return GSRAD_OK;
    const int pool_rays = R >= kPoolRays ? kPoolRays : (kPoolRays / R) * R;
    const int64_t npools = (count * R + pool_rays - 1) / pool_rays;
    uint32_t *queue = static_cast<uint32_t *>(pools);                       // 8 counters, 256 B apart
    uint4 *list = reinterpret_cast<uint4 *>(static_cast<char *>(pools) + 8 * 256);
    hipLaunchKernelGGL(k_ray_pools, dim3((unsigned)npools), dim3(256), 0, st, bv, R, seed, s_begin, count, pool_rays,
                       by_orig, list, queue, rcnt);
    return check_hip(hipGetLastError(), "ray pools launch");
}

gsrad_status launch_ff_trace(const BvhDev &bv, int R, float t_eps, float t_min, int64_t s_begin, int64_t count,
                             int by_orig, uint2 *recs, uint32_t *rcnt, int rcap, int deep, void *pools, int *err,
                             hipStream_t st) {
    if (count <= 0 || bv.n == 1) return GSRAD_OK;
    const int pool_rays = R >= kPoolRays ? kPoolRays : (kPoolRays / R) * R;
    const int64_t npools = (count * R + pool_rays - 1) / pool_rays;
    uint32_t *queue = static_cast<uint32_t *>(pools);
    const uint4 *list = reinterpret_cast<const uint4 *>(static_cast<char *>(pools) + 8 * 256);
    gsrad_status s;
    // persistent workgroups: three per CU (twelve waves), at most one per pool
    int dev = 0, cus = 0;
    if ((s = check_hip(hipGetDevice(&dev), "ff trace device")) != GSRAD_OK) return s;
    if ((s = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "ff trace CUs")) !=
        GSRAD_OK)
        return s;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(npools, 3 * (int64_t)cus));
    if (deep) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ff_trace<kStackDeep>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kStackDeep * 256 * 4);
        hipLaunchKernelGGL(k_ff_trace<kStackDeep>, dim3((unsigned)grid), dim3(256),
                           (size_t)kStackDeep * 256 * sizeof(uint32_t), st, bv, R, t_eps, t_min, s_begin, count,
                           pool_rays, npools, list, queue, by_orig, recs, rcnt, rcap, err);
    } else {
        hipLaunchKernelGGL(k_ff_trace<kStackShallow>, dim3((unsigned)grid), dim3(256),
                           (size_t)kStackShallow * 256 * sizeof(uint32_t), st, bv, R, t_eps, t_min, s_begin, count,
                           pool_rays, npools, list, queue, by_orig, recs, rcnt, rcap, err);
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
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_opacity_bwd), hipFuncAttributeMaxDynamicSharedMemorySize,
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
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_opacity_rec), hipFuncAttributeMaxDynamicSharedMemorySize,
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
