// Directional transfer of spherical-harmonic radiance through the diffuse +
// Phong BRDF (Eq. final-radiosity with f_i = f^c_i x Ybar, Sec. 3.2,
// Eq. brdf, App. A), its adjoint and the BRDF coefficients.
//
// The coefficient vectors of surfel i live in its tangent frame
// (t_u, t_v, n).  Per stored entry (i, j) of F the directional factors use
// the unit direction d from p_i to p_j:
//   (T X)_i[l][a][c] = sum_j F_ij Y_a(d in i's frame) sum_b Y_b(-d in j's frame) X_j[l][b][c]
//   B^(k+1) = E + R (.) (T B^(k)),  R_i = pi o_i f^c_i  (per coefficient, colour)
// The adjoint T^T has the same form on F^T with the roles of the row and the
// column swapped, so one kernel serves both (the backward propagates with
// the decay term reversed).
//
// One wave owns one output row: its lanes take the row's entries (one each,
// 64 at a time), evaluate both SH bases of the pair, gather the sender's
// row and accumulate all K x 3 outputs of the light; a butterfly over the
// wave then sums the lanes in a fixed order (deterministic results).
#include "gsrad_internal.h"
#include "sh_api.h"
#include "sh_basis.h"
#include "trace_api.h"

namespace gsrad {

namespace {

constexpr int kWavesPerBlock = 4;
constexpr float kPi = 3.14159265358979324f;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t g) {
    const int64_t x = b & 7, q = b >> 3, per = g >> 3, rem = g & 7;
    return x * per + (x < rem ? x : rem) + q;
}

// Unit direction from the centre of `ri` to the centre of `rj` in ri's
// frame (di) and its opposite in rj's frame (ej).  Coincident centres take
// the receiver's normal as the direction.
__device__ __forceinline__ void pair_dirs(const SurfRec &ri, const SurfRec &rj, float (&di)[3], float (&ej)[3]) {
    float dx = rj.a.x - ri.a.x, dy = rj.a.y - ri.a.y, dz = rj.a.z - ri.a.z;
    const float len2 = dx * dx + dy * dy + dz * dz;
    if (len2 > 0.0f) {
        const float inv = 1.0f / sqrtf(len2);
        dx *= inv;
        dy *= inv;
        dz *= inv;
    } else {
        dx = ri.b.x;
        dy = ri.b.y;
        dz = ri.b.z;
    }
    di[0] = dx * ri.c.x + dy * ri.c.y + dz * ri.c.z;
    di[1] = dx * ri.d.x + dy * ri.d.y + dz * ri.d.z;
    di[2] = dx * ri.b.x + dy * ri.b.y + dz * ri.b.z;
    ej[0] = -(dx * rj.c.x + dy * rj.c.y + dz * rj.c.z);
    ej[1] = -(dx * rj.d.x + dy * rj.d.y + dz * rj.d.z);
    ej[2] = -(dx * rj.b.x + dy * rj.b.y + dz * rj.b.z);
}

template <int N>
__device__ __forceinline__ void wave_sum(float (&v)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    }
}

template <int N>
__device__ __forceinline__ float pick(const float (&v)[N], int lane) {
    float r = 0.0f;
#pragma unroll
    for (int q = 0; q < N; ++q) r = lane == q ? v[q] : r;
    return r;
}

// mode 0 (bounce):  acc = (T X)_row;  out_a = acc (if set);  out_b = E + R (.) acc
// mode 1 (adjoint): acc = (T^T X)_row on F^T;  out_a = acc;  out_b += acc
template <int K>
__global__ void __launch_bounds__(256) k_transfer_sh(BvhDev bv, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const float *__restrict__ val,
                                                     int64_t n, int Lt, const float *__restrict__ X,
                                                     const float *__restrict__ E, const float *__restrict__ R,
                                                     float *__restrict__ out_a, float *__restrict__ out_b, int mode,
                                                     int64_t nblocks, const int32_t *__restrict__ order) {
    constexpr int W = 3 * K;
    const int64_t idx = xcd_block(blockIdx.x, nblocks) * kWavesPerBlock + threadIdx.x / 64;
    if (idx >= n) return;
    const int64_t row = order ? (int64_t)order[idx] : idx;
    const int lane = __lane_id();
    const SurfRec ri = bv.rec[bv.inv[row]];
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    for (int l = 0; l < Lt; ++l) {
        float acc[W];
#pragma unroll
        for (int q = 0; q < W; ++q) acc[q] = 0.0f;
        for (int64_t kk = b + lane; kk < e; kk += 64) {
            const int32_t j = col[kk];
            const float w = val[kk];
            const SurfRec rj = bv.rec[bv.inv[j]];
            float di[3], ej[3];
            pair_dirs(ri, rj, di, ej);
            float Yd[K], Ye[K];
            sh_eval<K>(di[0], di[1], di[2], Yd);
            sh_eval<K>(ej[0], ej[1], ej[2], Ye);
            const float *xj = X + ((int64_t)j * Lt + l) * W;
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                s0 = __builtin_fmaf(Ye[q], xj[3 * q + 0], s0);
                s1 = __builtin_fmaf(Ye[q], xj[3 * q + 1], s1);
                s2 = __builtin_fmaf(Ye[q], xj[3 * q + 2], s2);
            }
            s0 *= w;
            s1 *= w;
            s2 *= w;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                acc[3 * a + 0] = __builtin_fmaf(Yd[a], s0, acc[3 * a + 0]);
                acc[3 * a + 1] = __builtin_fmaf(Yd[a], s1, acc[3 * a + 1]);
                acc[3 * a + 2] = __builtin_fmaf(Yd[a], s2, acc[3 * a + 2]);
            }
        }
        wave_sum<W>(acc);
        const float v = pick<W>(acc, lane);
        if (lane < W) {
            const int64_t o = (row * Lt + l) * W + lane;
            if (mode == 0) {
                if (out_a) out_a[o] = v;
                out_b[o] = __builtin_fmaf(R[row * W + lane], v, E[o]);
            } else {
                out_a[o] = v;
                out_b[o] += v;
            }
        }
    }
}

// u = R (.) lambda, per light
__global__ void __launch_bounds__(256) k_scale_rows(const float *__restrict__ lam, const float *__restrict__ R,
                                                    int64_t n, int Lt, int W, float *__restrict__ u) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * Lt * W) return;
    const int64_t q = t % W, i = t / ((int64_t)Lt * W);
    u[t] = R[i * W + q] * lam[t];
}

// grad_F[e] = sum_k sum_l sum_c (Yd . (R (.) lambda^(k+1))_i[l][:, c]) (Ye . B^(k)_j[l][:, c])
template <int K>
__global__ void __launch_bounds__(256) k_sddmm_sh(BvhDev bv, const int64_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col, int64_t n, int Lt, int nb,
                                                  const float *__restrict__ Btape, const float *__restrict__ Ltape,
                                                  const float *__restrict__ R, float *__restrict__ grad_F,
                                                  int64_t nblocks, const int32_t *__restrict__ order) {
    constexpr int W = 3 * K;
    const int64_t idx = xcd_block(blockIdx.x, nblocks) * kWavesPerBlock + threadIdx.x / 64;
    if (idx >= n) return;
    const int64_t row = order ? (int64_t)order[idx] : idx;
    const int lane = __lane_id();
    const SurfRec ri = bv.rec[bv.inv[row]];
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    const float *Ri = R + row * W;
    const size_t plane = (size_t)n * Lt * W;
    for (int64_t kk = b + lane; kk < e; kk += 64) {
        const int32_t j = col[kk];
        const SurfRec rj = bv.rec[bv.inv[j]];
        float di[3], ej[3];
        pair_dirs(ri, rj, di, ej);
        float Yd[K], Ye[K];
        sh_eval<K>(di[0], di[1], di[2], Yd);
        sh_eval<K>(ej[0], ej[1], ej[2], Ye);
        float g = 0.0f;
        for (int k = 0; k < nb; ++k) {
            for (int l = 0; l < Lt; ++l) {
                const float *lam = Ltape + k * plane + (row * Lt + l) * W;
                const float *bj = Btape + k * plane + ((int64_t)j * Lt + l) * W;
                float p0 = 0.0f, p1 = 0.0f, p2 = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    p0 = __builtin_fmaf(Yd[q], Ri[3 * q + 0] * lam[3 * q + 0], p0);
                    p1 = __builtin_fmaf(Yd[q], Ri[3 * q + 1] * lam[3 * q + 1], p1);
                    p2 = __builtin_fmaf(Yd[q], Ri[3 * q + 2] * lam[3 * q + 2], p2);
                    s0 = __builtin_fmaf(Ye[q], bj[3 * q + 0], s0);
                    s1 = __builtin_fmaf(Ye[q], bj[3 * q + 1], s1);
                    s2 = __builtin_fmaf(Ye[q], bj[3 * q + 2], s2);
                }
                g = __builtin_fmaf(p0, s0, g);
                g = __builtin_fmaf(p1, s1, g);
                g = __builtin_fmaf(p2, s2, g);
            }
        }
        grad_F[kk] = g;
    }
}

// grad_R[i][q] = sum_k sum_l lambda^(k+1)_i[l][q] Q^(k)_i[l][q]
__global__ void __launch_bounds__(256) k_grad_R(const float *__restrict__ Ltape, const float *__restrict__ Qtape,
                                                int64_t n, int Lt, int W, int nb, float *__restrict__ grad_R) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * W) return;
    const int64_t i = t / W, q = t % W;
    const size_t plane = (size_t)n * Lt * W;
    float g = 0.0f;
    for (int k = 0; k < nb; ++k)
        for (int l = 0; l < Lt; ++l) {
            const size_t o = k * plane + (i * Lt + l) * W + q;
            g = __builtin_fmaf(Ltape[o], Qtape[o], g);
        }
    grad_R[t] = g;
}

// App. A: g_l(s) for the Phong lobe and its derivative, l = 1..3
__device__ __forceinline__ float lobe(int l, float s) {
    if (l == 1) return (s + 1.0f) / (s + 2.0f);
    if (l == 2) return s / (s + 3.0f);
    return ((s + 1.0f) * (s - 1.0f)) / ((s + 2.0f) * (s + 4.0f));
}

__device__ __forceinline__ float lobe_ds(int l, float s) {
    if (l == 1) return 1.0f / ((s + 2.0f) * (s + 2.0f));
    if (l == 2) return 3.0f / ((s + 3.0f) * (s + 3.0f));
    const float D = (s + 2.0f) * (s + 4.0f);
    return (2.0f * s * D - (s * s - 1.0f) * (2.0f * s + 6.0f)) / (D * D);
}

__device__ __forceinline__ float brdf_coef(int a, int c, float k, const float *ad, const float *as, float s) {
    if (a == 0) return 4.0f * k * ad[c] + (1.0f - k) * as[c];
    const float sgn = (sh_m(a) & 1) ? -1.0f : 1.0f;
    return sgn * (1.0f - k) * lobe(sh_l(a), s) * as[c];
}

__global__ void __launch_bounds__(256) k_brdf_reflectance(BvhDev bv, const float *__restrict__ kd,
                                                          const float *__restrict__ ad, const float *__restrict__ as,
                                                          const float *__restrict__ shin, int K, float *__restrict__ R) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= bv.n) return;
    const float o = bv.op[i];
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < 3; ++c)
            R[(i * K + a) * 3 + c] = kPi * o * brdf_coef(a, c, kd[i], ad + 3 * i, as + 3 * i, shin[i]);
}

__global__ void __launch_bounds__(256) k_brdf_backward(BvhDev bv, const float *__restrict__ kd,
                                                       const float *__restrict__ ad, const float *__restrict__ as,
                                                       const float *__restrict__ shin, int K,
                                                       const float *__restrict__ G, float *g_o, float *g_k,
                                                       float *g_ad, float *g_as, float *g_s) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= bv.n) return;
    const float o = bv.op[i], oraw = bv.raw_op[i];
    const bool inside = oraw > 0.0f && oraw < kOpacityMax;
    const float k = kd[i], s = shin[i];
    const float *adi = ad + 3 * i, *asi = as + 3 * i, *Gi = G + i * K * 3;
    float go = 0.0f, gk = 0.0f, gs = 0.0f, gad[3], gas[3];
    for (int c = 0; c < 3; ++c) {
        const float gp = kPi * o * Gi[c];
        gad[c] = gp * 4.0f * k;
        gas[c] = gp * (1.0f - k);
        gk += gp * (4.0f * adi[c] - asi[c]);
    }
    for (int a = 0; a < K; ++a) {
        const float sgn = (sh_m(a) & 1) ? -1.0f : 1.0f;
        const int l = sh_l(a);
        for (int c = 0; c < 3; ++c) {
            go += Gi[3 * a + c] * brdf_coef(a, c, k, adi, asi, s);
            if (a == 0) continue;
            const float gp = kPi * o * Gi[3 * a + c];
            gk -= gp * sgn * lobe(l, s) * asi[c];
            gas[c] += gp * sgn * (1.0f - k) * lobe(l, s);
            gs += gp * sgn * (1.0f - k) * lobe_ds(l, s) * asi[c];
        }
    }
    if (g_o) g_o[i] = inside ? kPi * go : 0.0f;
    if (g_k) g_k[i] = gk;
    if (g_s) g_s[i] = gs;
    for (int c = 0; c < 3; ++c) {
        if (g_ad) g_ad[3 * i + c] = gad[c];
        if (g_as) g_as[3 * i + c] = gas[c];
    }
}

unsigned row_blocks_sh(int64_t n) { return (unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock); }

template <int K>
void launch_transfer_k(const BvhDev &bv, const Csr &F, int Lt, const float *X, const float *E, const float *R,
                       float *out_a, float *out_b, int mode, hipStream_t st) {
    const unsigned g = row_blocks_sh(F.n);
    hipLaunchKernelGGL(k_transfer_sh<K>, dim3(g), dim3(256), 0, st, bv, F.row_ptr, F.col, F.val, F.n, Lt, X, E, R,
                       out_a, out_b, mode, (int64_t)g, F.order);
}

template <int K>
void launch_sddmm_k(const BvhDev &bv, const Csr &F, int Lt, int nb, const float *Bt, const float *Lt_, const float *R,
                    float *grad_F, hipStream_t st) {
    const unsigned g = row_blocks_sh(F.n);
    hipLaunchKernelGGL(k_sddmm_sh<K>, dim3(g), dim3(256), 0, st, bv, F.row_ptr, F.col, F.n, Lt, nb, Bt, Lt_, R, grad_F,
                       (int64_t)g, F.order);
}

}  // namespace

gsrad_status launch_transfer_sh(const BvhDev &bv, const Csr &F, int Lt, int K, const float *X, const float *E,
                                const float *R, float *out_a, float *out_b, int mode, hipStream_t st) {
    if (F.n == 0) return GSRAD_OK;
    switch (K) {
        case 1: launch_transfer_k<1>(bv, F, Lt, X, E, R, out_a, out_b, mode, st); break;
        case 4: launch_transfer_k<4>(bv, F, Lt, X, E, R, out_a, out_b, mode, st); break;
        case 9: launch_transfer_k<9>(bv, F, Lt, X, E, R, out_a, out_b, mode, st); break;
        case 16: launch_transfer_k<16>(bv, F, Lt, X, E, R, out_a, out_b, mode, st); break;
        default: set_error("SH transfer: K must be 1, 4, 9 or 16"); return GSRAD_EINVAL;
    }
    return check_hip(hipGetLastError(), "SH transfer launch");
}

gsrad_status launch_scale_rows(const float *lam, const float *R, int64_t n, int Lt, int K, float *u, hipStream_t st) {
    const int64_t total = n * Lt * K * 3;
    if (total == 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, lam, R, n, Lt, K * 3, u);
    return check_hip(hipGetLastError(), "SH scale launch");
}

gsrad_status launch_sddmm_sh(const BvhDev &bv, const Csr &F, int Lt, int K, int nb, const float *Btape,
                             const float *Ltape, const float *R, float *grad_F, hipStream_t st) {
    if (F.n == 0 || F.nnz == 0) return GSRAD_OK;
    switch (K) {
        case 1: launch_sddmm_k<1>(bv, F, Lt, nb, Btape, Ltape, R, grad_F, st); break;
        case 4: launch_sddmm_k<4>(bv, F, Lt, nb, Btape, Ltape, R, grad_F, st); break;
        case 9: launch_sddmm_k<9>(bv, F, Lt, nb, Btape, Ltape, R, grad_F, st); break;
        case 16: launch_sddmm_k<16>(bv, F, Lt, nb, Btape, Ltape, R, grad_F, st); break;
        default: set_error("SH sddmm: K must be 1, 4, 9 or 16"); return GSRAD_EINVAL;
    }
    return check_hip(hipGetLastError(), "SH sddmm launch");
}

gsrad_status launch_grad_R(const float *Ltape, const float *Qtape, int64_t n, int Lt, int K, int nb, float *grad_R,
                           hipStream_t st) {
    const int64_t total = n * K * 3;
    hipLaunchKernelGGL(k_grad_R, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, Ltape, Qtape, n, Lt, K * 3,
                       nb, grad_R);
    return check_hip(hipGetLastError(), "SH grad_R launch");
}

gsrad_status launch_brdf_reflectance(const BvhDev &bv, const float *kd, const float *ad, const float *as,
                                     const float *shin, int K, float *R, hipStream_t st) {
    hipLaunchKernelGGL(k_brdf_reflectance, dim3((unsigned)((bv.n + 255) / 256)), dim3(256), 0, st, bv, kd, ad, as, shin,
                       K, R);
    return check_hip(hipGetLastError(), "BRDF reflectance launch");
}

gsrad_status launch_brdf_backward(const BvhDev &bv, const float *kd, const float *ad, const float *as,
                                  const float *shin, int K, const float *G, float *g_o, float *g_k, float *g_ad,
                                  float *g_as, float *g_s, hipStream_t st) {
    hipLaunchKernelGGL(k_brdf_backward, dim3((unsigned)((bv.n + 255) / 256)), dim3(256), 0, st, bv, kd, ad, as, shin, K,
                       G, g_o, g_k, g_ad, g_as, g_s);
    return check_hip(hipGetLastError(), "BRDF backward launch");
}

}  // namespace gsrad
