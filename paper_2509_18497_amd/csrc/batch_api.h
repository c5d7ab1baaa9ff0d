// Host launchers of the batched (ragged) transport kernels (batch.hip).
#pragma once

#include "trace_api.h"

namespace gsrad {

// Device view of a batch of scenes sharing one block-diagonal F.
struct BatchDev {
    int64_t rows = 0;               // sum of the scenes' rows
    int32_t scenes = 0;
    const int64_t *row_off = nullptr;   // [scenes + 1] first row of each scene
    const int64_t *val_off = nullptr;   // [scenes + 1] first value of each scene's [N_s][C_s] block
    const int32_t *scene_C = nullptr;   // [scenes] columns C_s = Lt_s * K * 3
    int32_t *row_scene = nullptr;       // [rows] scene of each row (filled by batch_order_rows)
    const int64_t *order = nullptr;     // [rows] the order the persistent kernels take rows in: each ray-cast
                                        // scene's rows in Morton order, scene after scene, else by cost
};

size_t batch_order_temp_bytes(int64_t rows);
// row_scene and order from the scene table and F's row lengths
gsrad_status batch_order_rows(const BatchDev &bd, const int64_t *row_ptr, void *temp, size_t temp_bytes,
                              hipStream_t st);
// bounce: out = E + rho * (F in);  adjoint (F given as F^T): out = F^T (rho in), gE += out.
// One persistent launch; lpr = lanes per row (16, 32 or 64).  counter: one device uint32.
// in: FP32 rows, or BF16 rows when in_bf16 (FP32 sums either way).
gsrad_status launch_ragged_spmm(const BatchDev &bd, const Csr &F, int lpr, bool adjoint, const void *in, bool in_bf16,
                                const float *E, const float *rho, float *out, float *gE, uint32_t *counter,
                                hipStream_t st);
// grad_F at the stored entries and grad_rho from the tapes [nb][vals]
// (max_C: the largest C_s of the batch)
gsrad_status launch_ragged_sddmm(const BatchDev &bd, const Csr &F, int nb, int64_t vals, int max_C, const float *Bt,
                                 const float *Lt, const float *rho, float *grad_F, float *grad_rho, uint32_t *counter,
                                 hipStream_t st);

}  // namespace gsrad

namespace gsrad {

// out[k] = in[k] + add (index shifts of the block-diagonal CSR)
gsrad_status launch_offset_copy_i32(const int32_t *in, int64_t n, int32_t add, int32_t *out, hipStream_t st);
gsrad_status launch_offset_copy_i64(const int64_t *in, int64_t n, int64_t add, int64_t *out, hipStream_t st);
// out[k] = (int64) in[k] + add
gsrad_status launch_offset_widen(const int32_t *in, int64_t n, int64_t add, int64_t *out, hipStream_t st);
// plain copy as a kernel (usable inside a captured graph)
gsrad_status launch_copy_f32(const float *in, int64_t n, float *out, hipStream_t st);
// out[k] = BF16 of in[k] (round to nearest even; out is __bf16[n])
gsrad_status launch_round_bf16(const float *in, int64_t n, void *out, hipStream_t st);

}  // namespace gsrad
