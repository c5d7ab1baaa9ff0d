// Device-side traversal helpers shared by the ray-cast, gradient and
// Monte-Carlo kernels: the k-buffer all-hit walk (trace_sorted), the shadow
// walk (trace_shadow), the segment walk between two surfel centres
// (trace_segment), the open-addressing slot hash of surfel indices, and the
// double-float and fixed-point helpers of the deterministic gradient sums.
// Everything sits in an unnamed namespace: each kernel source gets its own
// inlined copy.
#pragma once

#include "gsrad_internal.h"

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

// Double-float pairs (error-free FP32 sums and products) and 64-bit
// fixed-point accumulation with atomics of workgroup scope (each XCD adds
// into its own copy of the accumulators, held in its L2).
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

// Exponent marker of a non-finite upstream gradient: the fixed-point sums
// then yield NaN.
constexpr int kFxNonFinite = 1 << 20;

// Value of surfel j in an LDS open-addressing table (keys hk, values hv),
// 0 when absent.
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

}  // namespace

}  // namespace gsrad
