// Monte-Carlo TD(0) radiosity solver (Sec. 7, App. D): K-Means groups of
// the surfels, next-event sampling of a group and a member, the one-point
// estimate with the centre-to-centre decay and the running averages.
#include "gsrad_internal.h"
#include "sh_api.h"
#include "trace_api.h"
#include "traverse.h"

namespace gsrad {

namespace {

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

}  // namespace

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

}  // namespace gsrad
