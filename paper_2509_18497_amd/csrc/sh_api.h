// Host launchers of the directional (spherical-harmonic) transfer kernels
// (sh.hip) and of the direct light with the BRDF (trace.hip).
#pragma once

#include "gsrad_internal.h"
#include "trace_api.h"

namespace gsrad {

// mode 0: out_a = T X (optional), out_b = E + R (.) (T X)
// mode 1 (F = F^T): out_a = T^T X, out_b += out_a
gsrad_status launch_transfer_sh(const BvhDev &bv, const Csr &F, int Lt, int K, const float *X, const float *E,
                                const float *R, float *out_a, float *out_b, int mode, hipStream_t st);
// u = R (.) lam (rows of Lt lights)
gsrad_status launch_scale_rows(const float *lam, const float *R, int64_t n, int Lt, int K, float *u, hipStream_t st);
gsrad_status launch_sddmm_sh(const BvhDev &bv, const Csr &F, int Lt, int K, int nb, const float *Btape,
                             const float *Ltape, const float *R, float *grad_F, hipStream_t st);
gsrad_status launch_grad_R(const float *Ltape, const float *Qtape, int64_t n, int Lt, int K, int nb, float *grad_R,
                           hipStream_t st);
gsrad_status launch_brdf_reflectance(const BvhDev &bv, const float *kd, const float *ad, const float *as,
                                     const float *shin, int K, float *R, hipStream_t st);
gsrad_status launch_brdf_backward(const BvhDev &bv, const float *kd, const float *ad, const float *as,
                                  const float *shin, int K, const float *G, float *g_o, float *g_k, float *g_ad,
                                  float *g_as, float *g_s, hipStream_t st);
gsrad_status launch_direct_sh(const BvhDev &bv, const float *R, const float *lpos, const float *lI, int Lt, int K,
                              float *E, int *err, hipStream_t st);

// centre-to-centre form factors on a pattern (trace.hip)
gsrad_status launch_ff_center(const BvhDev &bv, const Csr &P, const float *lambda, float *val, int *err,
                              hipStream_t st);
// gradients: accumulators of center_acc_bytes(n) zeroed first; out holds
// 16 device output arrays [n] (fields px py pz tux tuy tuz tvx tvy tvz nx
// ny nz su sv o, then lambda; NULL entries skipped)
struct CenterOutputs {
    float *p[16];
};
size_t center_acc_bytes(int64_t n);
gsrad_status launch_center_backward(const BvhDev &bv, const Csr &F, const float *lambda, const float *gF, void *acc,
                                    const CenterOutputs &out, int *err, hipStream_t st);

// geometry gradients through the ray-cast F from the recorded hits
// (accumulators of center_acc_bytes(n) zeroed first; out.p[0..14])
gsrad_status launch_geometry_rec(const BvhDev &bv, int R, uint64_t seed, const uint2 *recs, const uint32_t *rcnt,
                                 int rcap, const int64_t *row_ptr, const int32_t *col, const float *gF, int max_row,
                                 void *acc, const CenterOutputs &out, hipStream_t st);

// direct-light gradients (accumulators of light_acc_bytes(n, Lt) zeroed
// first; out.p[0..14] surfel fields)
size_t light_acc_bytes(int64_t n, int Lt);
gsrad_status launch_direct_backward(const BvhDev &bv, const float *albedo, const float *lpos, const float *lI, int Lt,
                                    int K, const float *gE, void *acc, float *g_lpos, float *g_lI, float *g_alb,
                                    const CenterOutputs &out, int *err, hipStream_t st);

// Monte-Carlo TD(0) solver (trace.hip): device buffers owned by the handle
struct McBuffers {
    float *cent = nullptr, *gnrm = nullptr, *L = nullptr;   // [G][3], [G][3], [G]
    uint32_t *key = nullptr, *ids = nullptr, *skey = nullptr, *members = nullptr, *count = nullptr;
    int64_t *goff = nullptr;                                  // [G + 1]
    void *rtemp = nullptr, *stemp = nullptr;
    size_t rtemp_bytes = 0, stemp_bytes = 0;
    float *S = nullptr, *S2 = nullptr, *B = nullptr, *delta = nullptr, *var = nullptr;   // [n][C], [n]
    uint32_t *D = nullptr, *q = nullptr, *maxbits = nullptr;
    int32_t *recv = nullptr;
    int64_t *cdf = nullptr;                                   // [n + 1]
};
gsrad_status mc_kmeans(const BvhDev &bv, int G, int iters, McBuffers &mb, hipStream_t st);
gsrad_status mc_step(const BvhDev &bv, const McBuffers &mb, int G, float rmin2, const float *lambda, const float *rho,
                     const float *E, const float *B, int Lt, int K, uint64_t seed, int step, const int32_t *recv,
                     float *delta, int *err, hipStream_t st);
gsrad_status mc_solve(const BvhDev &bv, const McBuffers &mb, int G, float rmin2, const float *lambda,
                      const float *rho, const float *E, int Lt, int K, int T, uint64_t seed, float *B_out,
                      int *err, hipStream_t st);

}  // namespace gsrad
