// Host launchers of the ray-casting kernels (trace.hip) and the sparse
// kernels (sparse.hip).
#pragma once

#include "gsrad_internal.h"

namespace gsrad {

// device error flag bits
constexpr int kErrStack = 1;   // traversal stack overflow
constexpr int kErrSlab = 2;    // (unused)
constexpr int kErrTable = 4;   // more distinct senders than the aggregation table holds
constexpr int kErrRow = 8;     // row longer than the ELL capacity
constexpr int kErrRecords = 16; // a ray composited more hits than its record slots (recomputed later)

size_t ff_stack_bytes(int threads);
size_t ff_aggregate_smem(int log2h);
// bytes of the ray pools (pools argument) for a chunk of count receivers
size_t ff_pool_list_bytes(int64_t count, int R);
// the chunk's rays, generated and sorted by direction into pools (and the
// trace's pool counters reset); a scene of one surfel gets its zero counts
// here and needs no trace
gsrad_status launch_ray_pools(const BvhDev &bv, int R, uint64_t seed, int64_t s_begin, int64_t count, int by_orig,
                              uint32_t *rcnt, void *pools, hipStream_t st);
// trace of the pools launch_ray_pools made (run it again before a repeat)
gsrad_status launch_ff_trace(const BvhDev &bv, int R, float t_eps, float t_min, int64_t s_begin, int64_t count,
                             int by_orig, uint2 *recs, uint32_t *rcnt, int rcap, int deep, void *pools, int *err,
                             hipStream_t st);
// Rows overflowing a table of 2^log2h entries (a probe chain of 256) are listed in
// redo_list (count in redo_cnt[0], tickets in redo_cnt[1]; room for count
// rows) and aggregated again with 2^log2h_max entries; err[2] counts them.
gsrad_status launch_ff_aggregate(const BvhDev &bv, const uint2 *recs, const uint32_t *rcnt, int rcap, int64_t s_begin,
                                 int64_t count, int by_orig, int R, int topk, int log2h, int log2h_max,
                                 int32_t *redo_list, uint32_t *redo_cnt, int64_t cap_row, int32_t *ell_col,
                                 float *ell_val, uint32_t *row_len, int *err, hipStream_t st);
gsrad_status launch_ell_to_csr(const int32_t *ell_col, const float *ell_val, int64_t cap_row, const int64_t *row_ptr,
                               int64_t n, int32_t *col, float *val, hipStream_t st);
gsrad_status launch_direct(const BvhDev &bv, const float *albedo, const float *lpos, const float *lI, int Lt, int K,
                           float *E, int *err, hipStream_t st);
// Opacity backward accumulators: 8 per-XCD copies of n int64 fixed-point
// sums, then the max |dL/dF| bits and the scale exponent (zero them first).
size_t opacity_acc_bytes(int64_t n);
gsrad_status launch_opacity_scale(const float *gF, int64_t nnz, int64_t n, void *acc, hipStream_t st);
gsrad_status launch_opacity_bwd(const BvhDev &bv, int R, uint64_t seed, float t_eps, float t_min,
                                const int64_t *row_ptr, const int32_t *col, const float *gF, int max_row, float2 *wbuf,
                                void *acc, int pass, const uint32_t *rcnt, int rcap, int *err, hipStream_t st);
gsrad_status launch_opacity_rec(const BvhDev &bv, int R, const uint2 *recs, const uint32_t *rcnt, int rcap,
                                const int64_t *row_ptr, const int32_t *col, const float *gF, int max_row,
                                void *acc, hipStream_t st);
gsrad_status launch_opacity_finish(const BvhDev &bv, const void *acc, const float *grad_rho, const float *albedo,
                                   float *grad_o, float *grad_a, hipStream_t st);
gsrad_status launch_ray_hits(const BvhDev &bv, int R, uint64_t seed, float t_eps, float t_min, const int64_t *recv,
                             int64_t n_recv, int max_hits, float *dirs, int32_t *cnt, int32_t *hj, float *ht,
                             int8_t *hf, float *hT, int *err, hipStream_t st);
gsrad_status launch_reflectance(const BvhDev &bv, const float *albedo, float *rho, hipStream_t st);

// sparse.hip
struct Csr {
    int64_t n = 0, nnz = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const float *val = nullptr;
    // optional order in which the row kernels take the rows (a permutation
    // of 0..n-1, e.g. the receivers' Morton order, so that the rows one XCD
    // runs together gather from nearby columns); results do not depend on it
    const int32_t *order = nullptr;
};

size_t transpose_temp_bytes(int64_t n, int64_t nnz);
gsrad_status csr_transpose(const Csr &A, int64_t *t_row_ptr, int32_t *t_col, float *t_val, void *temp,
                           size_t temp_bytes, hipStream_t st);
// Bout = E + rho * (F Bin), rows of C columns
// Morton-sorted position -> original surfel index (the sorted records' ids)
gsrad_status launch_sorted_order(const BvhDev &bv, int32_t *order, hipStream_t st);
gsrad_status launch_bounce(const Csr &F, int C, const float *Bin, const float *E, const float *rho, float *Bout,
                           hipStream_t st);
// lam_out = F^T (rho * lam_in) given FT = transpose(F); gE += lam_out
gsrad_status launch_adjoint(const Csr &FT, int C, const float *lam_in, const float *rho, float *lam_out, float *gE,
                            hipStream_t st);
// grad_F[e] and grad_rho from the forward tape B^(k) and the adjoint tape
// lambda^(k+1), both [nb][N][C]
gsrad_status launch_sddmm(const Csr &F, int C, int nb, const float *Btape, const float *Ltape, const float *rho,
                          float *grad_F, float *grad_rho, hipStream_t st);
// reciprocity sums over the stored entries (areas [n] FP64): acc[0] +=
// |A_i F_ij - A_j F_ji|, acc[1] += A_i F_ij, acc[2] = max relative difference
gsrad_status launch_reciprocity(const Csr &F, const double *area, double *acc, hipStream_t st);
// FP64 checks: acc[0] = sum r^2, acc[1] = sum B^2, acc[2] = max row sum,
// acc[3] = number of non-finite inputs
gsrad_status launch_check(const Csr &F, int C, const float *rho, const float *E, const float *B, double *acc,
                          hipStream_t st);

}  // namespace gsrad
