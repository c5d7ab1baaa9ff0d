// Gradient kernels through the centre-to-centre form factors (Sec. 8), the
// ray-cast form factors' geometry (recorded hits) and the direct light.
//
// k_ff_center       one wave per row of a pattern: the centre-to-centre F
//                   with the learnable decay scale lambda.
// k_center_bwd      its gradient with respect to lambda and every surfel
//                   field on each segment (endpoints and occluders).
// k_geometry_rec    dL/dF through the recorded hits to centres, frames,
//                   scales and opacities.
// k_direct_bwd      the direct light's gradient: lights, albedo, receivers
//                   and shadow-segment occluders.
// All sums are 64-bit fixed point with per-field scales (bit-identical
// between runs), one copy per XCD.
#include <functional>

#include "gsrad_internal.h"
#include "sh_api.h"
#include "trace_api.h"
#include "traverse.h"

namespace gsrad {

namespace {

// ---------------------------------------------------------------------------
// centre-to-centre form factors (Sec. 8) and their gradients
// ---------------------------------------------------------------------------
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

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
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
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
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

}  // namespace gsrad
