// Host launchers of the dense BF16 transport kernels (dense.hip).
//
// Layouts: the dense operators are [Np][Np] BF16 row-major with
// Np = dense_pad(n) (zero rows and columns beyond n).  Operands of a
// product with C right-hand-side columns are transposed, [dense_pad(C)][Np]
// BF16 (column c of B as one contiguous row), zero beyond n.
#pragma once

#include "trace_api.h"

namespace gsrad {

int64_t dense_pad(int64_t x);   // next multiple of the 256-wide tile

// One forward bounce on the matrix cores:
//   Q = F X (X given as x_hi [+ x_lo]), B^(k+1) = E + rho Q.
// split: F X = F_hi X_hi + F_hi X_lo + F_lo X_hi (the correction sweep).
// Outputs (each optional): Bout and Q [n][C] FP32, the next operand
// xt_hi / xt_lo [Cp][ldx], a BF16 row copy bb[i][boff + c].
struct DenseBounce {
    const __bf16 *f_hi = nullptr, *f_lo = nullptr;   // [ld][ld]
    int64_t ld = 0;
    const __bf16 *x_hi = nullptr, *x_lo = nullptr;   // [Cp][ldx]
    int64_t ldx = 0;
    bool split = false;
    const float *E = nullptr, *rho = nullptr;
    int64_t n = 0;
    int C = 0;
    float *Bout = nullptr, *Q = nullptr;
    __bf16 *xt_hi = nullptr, *xt_lo = nullptr;
    __bf16 *bb = nullptr, *bb_lo = nullptr;
    int64_t ldbb = 0, boff = 0;
};
gsrad_status launch_dense_bounce(const DenseBounce &a, hipStream_t st);

// One adjoint step: lambda^(k) = F^T Y with Y = rho lambda^(k+1) given as
// y_hi [+ y_lo]; dL/dE += lambda^(k); next operand yt_hi = bf16(rho
// lambda^(k)) transposed; a BF16 row copy p[j][poff + c] of the same.
struct DenseAdjoint {
    const __bf16 *ft_hi = nullptr, *ft_lo = nullptr;   // [ld][ld]
    int64_t ld = 0;
    const __bf16 *y_hi = nullptr, *y_lo = nullptr;     // [Cp][ldx]
    int64_t ldx = 0;
    bool split = false;
    const float *rho = nullptr;
    int64_t n = 0;
    int C = 0;
    float *lam = nullptr, *gE = nullptr;
    __bf16 *yt_hi = nullptr;
    __bf16 *p = nullptr, *p_lo = nullptr;
    int64_t ldp = 0, poff = 0;
};
gsrad_status launch_dense_adjoint(const DenseAdjoint &a, hipStream_t st);

// G[i][j] = sum_k P[i][k] Bb[j][k], k < kpad, with both operands split
// (P_hi Bb_hi + P_hi Bb_lo + P_lo Bb_hi; rows padded to ld_pad, zero beyond
// n), G [n][ldg] FP32.
gsrad_status launch_dense_grad_F(const __bf16 *P, const __bf16 *P_lo, const __bf16 *Bb, const __bf16 *Bb_lo,
                                 int64_t ldk, int64_t kpad, int64_t n, int64_t ld_pad, float *G, int64_t ldg,
                                 hipStream_t st);

gsrad_status launch_dense_scatter(const Csr &F, int64_t ld, __bf16 *f_hi, __bf16 *f_lo, __bf16 *ft_hi,
                                  __bf16 *ft_lo, hipStream_t st);
// out_hi[c][i] = bf16(s x[i][c]) (s = rho[i][c%3] or 1), out_lo = bf16(s x - hi) if given
gsrad_status launch_to_bf16_t(const float *x, const float *rho, int64_t n, int C, __bf16 *hi, __bf16 *lo, int64_t ld,
                              hipStream_t st);
// out[i][off + c] = bf16(s x[i][c]), out_lo = bf16(s x - out) if given
gsrad_status launch_to_bf16_rows(const float *x, const float *rho, int64_t n, int C, __bf16 *out, __bf16 *out_lo,
                                 int64_t ld, int64_t off, hipStream_t st);
// grad_rho[i][col] += sum_{c % 3 == col} lam[i][c] Q[i][c]
gsrad_status launch_grad_rho_acc(const float *lam, const float *Q, int64_t n, int C, float *grad_rho,
                                 hipStream_t st);
// out[e] = G[i][col[e]] over the entries of F
gsrad_status launch_gather_csr(const Csr &F, const float *G, int64_t ld, float *out, hipStream_t st);

}  // namespace gsrad
