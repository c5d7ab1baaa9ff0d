// Batched transport over scenes of uneven size: the scenes' form factors
// form one block-diagonal F (global row and column indices), scene s owns
// rows [row_off[s], row_off[s+1]) and C_s = Lt_s * K * 3 columns, so B, E
// and the gradients are ragged: scene s's rows are a [N_s][C_s] block at
// val_off[s] of one array.
//
// Each bounce (and each adjoint step) is ONE persistent launch over all
// scenes: groups of LPR lanes take rows from a work queue (eight ranges,
// one per XCD, drained by the others once their own is done), so scenes of
// 2k and 65k surfels and 8 or 100 lights share the chip without tail
// effects.  The queue holds each ray-cast scene's rows in the receivers'
// Morton order, scene after scene (rows that one XCD takes together gather
// from nearby columns), else all rows by cost (entries x columns, largest
// first).
// LPR (lanes per row: 64, 32 or 16) is the tile shape the autotuner picks;
// every variant accumulates each output in the same order (the row's
// entries in CSR order), so the choice never changes a result bit.
#include "gsrad_internal.h"
#include "batch_api.h"

namespace gsrad {

namespace {

// Work-queue position -> row, for a group of LPR lanes: one lane takes the
// next index and the group shares it.  The queue is cut into eight equal
// ranges with a counter each; a group takes from the range of the XCD it
// runs on first (consecutive rows of the order, nearby receivers of one
// scene, share that XCD's L2) and from the others once it is drained.
// Every position below `rows` is handed out exactly once; `rows` means done.
template <int LPR>
__device__ __forceinline__ int64_t next_row(uint32_t *counter, int64_t rows, int lane_in_group, int group_base) {
    int q = (int)rows;
    if (lane_in_group == 0) {
        const int xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7;   // HW_REG_XCC_ID
        for (int t = 0; t < 8; ++t) {
            const int x = (xcc + t) & 7;
            const int64_t lo = rows * x / 8, len = rows * (x + 1) / 8 - lo;
            const uint32_t idx = atomicAdd(counter + x, 1u);
            if ((int64_t)idx < len) {
                q = (int)(lo + idx);
                break;
            }
        }
    }
    return (int64_t)__shfl(q, group_base, 64);
}

// out = E + rho * (F in) on the rows of all scenes (bounce), or
// out = F^T (rho in) and gE += out (adjoint, FT given as F, rho applied to
// the gathered rows).
// The gathered rows `in` are FP32, or BF16 (IN = __bf16) in the BF16 mode of
// the batched transport; the sums are FP32 either way.
// column chunks per pass over a row's entries: eight for FP32 rows, one for
// BF16 rows (measured on 64 uneven rooms with 8-100 lights: FP32 bounces
// 4.7 s with one chunk, 3.5 s with four, 3.2 s with eight; BF16 rows 3.0 s
// with one, 3.3 s with two, 4.8 s with four)
template <typename IN> constexpr int kChunks = sizeof(IN) == 2 ? 1 : 8;

template <int LPR, bool ADJ, typename IN>
__global__ void __launch_bounds__(256) k_ragged_spmm(BatchDev bd, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const float *__restrict__ val,
                                                     const IN *__restrict__ in, const float *__restrict__ E,
                                                     const float *__restrict__ rho, float *__restrict__ out,
                                                     float *__restrict__ gE, uint32_t *counter) {
    const int lane = __lane_id();
    const int lig = lane % LPR;                 // lane in group
    const int gbase = lane - lig;               // first lane of the group
    for (;;) {
        const int64_t q = next_row<LPR>(counter, bd.rows, lig, gbase);
        if (q >= bd.rows) break;
        const int64_t row = bd.order[q];
        const int s = bd.row_scene[row];
        const int C = bd.scene_C[s];
        const int64_t r0 = bd.row_off[s], base = bd.val_off[s];
        const int64_t lr = row - r0;
        const int64_t b = row_ptr[row], e = row_ptr[row + 1];
        // kChunks column chunks of LPR per pass over the row's entries: the
        // entries are read and broadcast once for all of them, and their
        // gathers are in flight together; each column's sum is the same
        // sequence of FMAs in CSR order as with one chunk per pass
        for (int c0 = 0; c0 < C; c0 += kChunks<IN> * LPR) {
            int cc[kChunks<IN>], colour[kChunks<IN>];
            bool on[kChunks<IN>], has[kChunks<IN>];
            float acc[kChunks<IN>];
#pragma unroll
            for (int h = 0; h < kChunks<IN>; ++h) {
                const int c = c0 + h * LPR + lig;
                has[h] = c0 + h * LPR < C;   // the chunk holds columns (uniform over the row's lanes)
                on[h] = c < C;
                cc[h] = on[h] ? c : 0;   // lanes past C gather column 0 and discard it
                colour[h] = cc[h] % 3;
                acc[h] = 0.0f;
            }
            for (int64_t k0 = b; k0 < e; k0 += LPR) {
                const int64_t kk = k0 + lig;
                const int jv = kk < e ? col[kk] : (int)r0;
                const float vv = kk < e ? val[kk] : 0.0f;
                const int m = (int)min<int64_t>(LPR, e - k0);
                int t = 0;
                // eight entries' gathers in flight per chunk, added in CSR order
                for (; t + 8 <= m; t += 8) {
                    float w[kChunks<IN>][8], x[kChunks<IN>][8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int64_t j = __shfl(jv, gbase + t + u, 64);
                        const float v = __shfl(vv, gbase + t + u, 64);
#pragma unroll
                        for (int h = 0; h < kChunks<IN>; ++h) {
                            w[h][u] = v;
                            if (ADJ) w[h][u] *= rho[j * 3 + colour[h]];
                            x[h][u] = has[h] ? (float)in[base + (j - r0) * C + cc[h]] : 0.0f;
                        }
                    }
#pragma unroll
                    for (int h = 0; h < kChunks<IN>; ++h)
#pragma unroll
                        for (int u = 0; u < 8; ++u) acc[h] = __builtin_fmaf(w[h][u], x[h][u], acc[h]);
                }
                for (; t < m; ++t) {
                    const int64_t j = __shfl(jv, gbase + t, 64);
                    const float v = __shfl(vv, gbase + t, 64);
#pragma unroll
                    for (int h = 0; h < kChunks<IN>; ++h) {
                        float w = v;
                        if (ADJ) w *= rho[j * 3 + colour[h]];
                        const float x = has[h] ? (float)in[base + (j - r0) * C + cc[h]] : 0.0f;
                        acc[h] = __builtin_fmaf(w, x, acc[h]);
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < kChunks<IN>; ++h) {
                if (on[h]) {
                    const int c = c0 + h * LPR + lig;
                    const int64_t o = base + lr * C + c;
                    if (ADJ) {
                        out[o] = acc[h];
                        gE[o] += acc[h];
                    } else {
                        out[o] = __builtin_fmaf(rho[row * 3 + colour[h]], acc[h], E[o]);
                    }
                }
            }
        }
    }
}

// grad_F[e] = sum_k sum_c rho_row,c%3 lam^(k+1)[row][c] B^(k)[j][c] and
// grad_rho[row][colour] = sum_e F[e] sum_k sum_{c of colour} (same), one
// wave per row (tapes [nb][vals]).
constexpr int kSddE = 12;   // entries per pass (measured on 64 uneven rooms: 1 entry 10.6 s, 2: 7.9, 4: 6.5, 8: 5.8, 12: 5.6, 16: 5.4 s with 206 VGPRs)

__global__ void __launch_bounds__(256) k_ragged_sddmm(BatchDev bd, const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const float *__restrict__ val, int nb, int64_t vals,
                                                      const float *__restrict__ Bt, const float *__restrict__ Lt,
                                                      const float *__restrict__ rho, float *__restrict__ grad_F,
                                                      float *__restrict__ grad_rho, uint32_t *counter) {
    const int lane = __lane_id();
    for (;;) {
        const int64_t q = next_row<64>(counter, bd.rows, lane, 0);
        if (q >= bd.rows) break;
        const int64_t row = bd.order[q];
        const int s = bd.row_scene[row];
        const int C = bd.scene_C[s];
        const int64_t r0 = bd.row_off[s], base = bd.val_off[s];
        const int64_t lr = row - r0;
        const int64_t b = row_ptr[row], e = row_ptr[row + 1];
        const float rr0 = rho[row * 3 + 0], rr1 = rho[row * 3 + 1], rr2 = rho[row * 3 + 2];
        float gr0 = 0.0f, gr1 = 0.0f, gr2 = 0.0f;
        // kSddE entries per pass: the row's lambda value of a (column, bounce)
        // is read once for all of them, and their gathers are in flight
        // together; each entry's sums run in the order of one at a time
        for (int64_t k = b; k < e; k += kSddE) {
            const int m = (int)min<int64_t>(kSddE, e - k);
            int64_t jj[kSddE];
#pragma unroll
            for (int u = 0; u < kSddE; ++u) jj[u] = (u < m ? col[k + u] : col[k]) - r0;
            float s0[kSddE], s1[kSddE], s2[kSddE];
#pragma unroll
            for (int u = 0; u < kSddE; ++u) s0[u] = s1[u] = s2[u] = 0.0f;
            for (int c = lane; c < C; c += 64) {
                float sum[kSddE];
#pragma unroll
                for (int u = 0; u < kSddE; ++u) sum[u] = 0.0f;
                for (int t = 0; t < nb; ++t) {
                    const float l = Lt[t * vals + base + lr * C + c];
#pragma unroll
                    for (int u = 0; u < kSddE; ++u)
                        sum[u] = __builtin_fmaf(l, Bt[t * vals + base + jj[u] * C + c], sum[u]);
                }
                const int colour = c % 3;
#pragma unroll
                for (int u = 0; u < kSddE; ++u) {
                    s0[u] += colour == 0 ? sum[u] : 0.0f;
                    s1[u] += colour == 1 ? sum[u] : 0.0f;
                    s2[u] += colour == 2 ? sum[u] : 0.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < kSddE; ++u) {
                if (u < m) {
                    float a0 = s0[u], a1 = s1[u], a2 = s2[u];
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) {
                        a0 += __shfl_xor(a0, o, 64);
                        a1 += __shfl_xor(a1, o, 64);
                        a2 += __shfl_xor(a2, o, 64);
                    }
                    if (lane == 0 && grad_F) grad_F[k + u] = rr0 * a0 + rr1 * a1 + rr2 * a2;
                    const float f = val[k + u];
                    gr0 = __builtin_fmaf(f, a0, gr0);
                    gr1 = __builtin_fmaf(f, a1, gr1);
                    gr2 = __builtin_fmaf(f, a2, gr2);
                }
            }
        }
        if (lane == 0 && grad_rho) {
            grad_rho[row * 3 + 0] = gr0;
            grad_rho[row * 3 + 1] = gr1;
            grad_rho[row * 3 + 2] = gr2;
        }
    }
}

// The same sums for scenes with up to 8 bounces and C <= 128: each lane
// keeps its (at most two) columns of lambda^(k+1)[row] in registers for
// every k, and four entries are gathered at a time.  Per lane the column
// chunks and bounces are added in the order of k_ragged_sddmm, and the
// reductions are the same, so both give the same bits.
constexpr int kFastNb = 8;

__global__ void __launch_bounds__(256) k_ragged_sddmm_fast(BatchDev bd, const int64_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ col,
                                                           const float *__restrict__ val, int nb, int64_t vals,
                                                           const float *__restrict__ Bt, const float *__restrict__ Lt,
                                                           const float *__restrict__ rho, float *__restrict__ grad_F,
                                                           float *__restrict__ grad_rho, uint32_t *counter) {
    const int lane = __lane_id();
    for (;;) {
        const int64_t q = next_row<64>(counter, bd.rows, lane, 0);
        if (q >= bd.rows) break;
        const int64_t row = bd.order[q];
        const int s = bd.row_scene[row];
        const int C = bd.scene_C[s];
        const int64_t r0 = bd.row_off[s], base = bd.val_off[s];
        const int64_t lr = row - r0;
        const bool on0 = lane < C, on1 = lane + 64 < C;
        const int c0 = on0 ? lane : 0, c1 = on1 ? lane + 64 : 0;
        const int col0 = c0 % 3, col1 = c1 % 3;
        float l0[kFastNb], l1[kFastNb];
#pragma unroll
        for (int t = 0; t < kFastNb; ++t) {
            l0[t] = (t < nb && on0) ? Lt[t * vals + base + lr * C + c0] : 0.0f;
            l1[t] = (t < nb && on1) ? Lt[t * vals + base + lr * C + c1] : 0.0f;
        }
        const int64_t b = row_ptr[row], e = row_ptr[row + 1];
        const float rr0 = rho[row * 3 + 0], rr1 = rho[row * 3 + 1], rr2 = rho[row * 3 + 2];
        float gr0 = 0.0f, gr1 = 0.0f, gr2 = 0.0f;
        constexpr int kE = 4;
        for (int64_t k0 = b; k0 < e; k0 += kE) {
            const int m = (int)min<int64_t>(kE, e - k0);
            float a0[kE], a1[kE];
#pragma unroll
            for (int u = 0; u < kE; ++u) {
                const int64_t j = (u < m ? col[k0 + u] : col[k0]) - r0;
                float x0[kFastNb], x1[kFastNb];
#pragma unroll
                for (int t = 0; t < kFastNb; ++t) {
                    x0[t] = t < nb ? Bt[t * vals + base + j * C + c0] : 0.0f;
                    x1[t] = (t < nb && on1) ? Bt[t * vals + base + j * C + c1] : 0.0f;
                }
                float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
                for (int t = 0; t < kFastNb; ++t)
                    if (t < nb) {
                        s0 = __builtin_fmaf(l0[t], x0[t], s0);
                        s1 = __builtin_fmaf(l1[t], x1[t], s1);
                    }
                a0[u] = on0 ? s0 : 0.0f;
                a1[u] = on1 ? s1 : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kE; ++u) {
                if (u >= m) break;
                // chunk 0 then chunk 1, as the column loop of k_ragged_sddmm adds them
                float s0 = col0 == 0 ? a0[u] : 0.0f;
                float s1 = col0 == 1 ? a0[u] : 0.0f;
                float s2 = col0 == 2 ? a0[u] : 0.0f;
                if (on1) {
                    s0 += col1 == 0 ? a1[u] : 0.0f;
                    s1 += col1 == 1 ? a1[u] : 0.0f;
                    s2 += col1 == 2 ? a1[u] : 0.0f;
                }
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    s0 += __shfl_xor(s0, o, 64);
                    s1 += __shfl_xor(s1, o, 64);
                    s2 += __shfl_xor(s2, o, 64);
                }
                const int64_t k = k0 + u;
                if (lane == 0 && grad_F) grad_F[k] = rr0 * s0 + rr1 * s1 + rr2 * s2;
                const float f = val[k];
                gr0 = __builtin_fmaf(f, s0, gr0);
                gr1 = __builtin_fmaf(f, s1, gr1);
                gr2 = __builtin_fmaf(f, s2, gr2);
            }
        }
        if (lane == 0 && grad_rho) {
            grad_rho[row * 3 + 0] = gr0;
            grad_rho[row * 3 + 1] = gr1;
            grad_rho[row * 3 + 2] = gr2;
        }
    }
}

__global__ void k_reset_counter(uint32_t *counter) {
    if (threadIdx.x < 8) counter[threadIdx.x] = 0u;
}

// row -> scene and the per-row cost (entries x columns) used for ordering
__global__ void __launch_bounds__(256) k_row_cost(BatchDev bd, const int64_t *__restrict__ row_ptr,
                                                  uint32_t *__restrict__ keys, uint32_t *__restrict__ ids) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= bd.rows) return;
    int lo = 0, hi = bd.scenes - 1;
    while (lo < hi) {   // last scene with row_off <= r
        const int mid = (lo + hi + 1) >> 1;
        if (bd.row_off[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    bd.row_scene[r] = lo;
    const uint64_t cost = (uint64_t)(row_ptr[r + 1] - row_ptr[r] + 1) * (uint64_t)bd.scene_C[lo];
    // descending cost: sort ascending on the complement, saturated to 32 bits
    keys[r] = ~(uint32_t)min<uint64_t>(cost, 0xffffffffull);
    ids[r] = (uint32_t)r;
}

__global__ void __launch_bounds__(256) k_copy_u32_to_i64(const uint32_t *__restrict__ a, int64_t n,
                                                         int64_t *__restrict__ b) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < n) b[r] = a[r];
}

inline unsigned persistent_blocks() { return 256 * 8; }   // 8 workgroups of 4 waves per CU

}  // namespace

gsrad_status batch_order_rows(const BatchDev &bd, const int64_t *row_ptr, void *temp, size_t temp_bytes,
                              hipStream_t st) {
    const int64_t n = bd.rows;
    if (n == 0) return GSRAD_OK;
    char *p = static_cast<char *>(temp);
    auto carve = [&](size_t bytes) {
        char *r = p;
        p += (bytes + 255) / 256 * 256;
        return r;
    };
    uint32_t *keys = reinterpret_cast<uint32_t *>(carve((size_t)n * 4));
    uint32_t *ids = reinterpret_cast<uint32_t *>(carve((size_t)n * 4));
    uint32_t *skeys = reinterpret_cast<uint32_t *>(carve((size_t)n * 4));
    uint32_t *sids = reinterpret_cast<uint32_t *>(carve((size_t)n * 4));
    const size_t rbytes = radix_temp_bytes(n);
    void *rtemp = carve(rbytes);
    if ((size_t)(p - static_cast<char *>(temp)) > temp_bytes) {
        set_error("batch ordering: temp too small");
        return GSRAD_EINVAL;
    }
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_row_cost, dim3(g), dim3(256), 0, st, bd, row_ptr, keys, ids);
    gsrad_status s = radix_sort_pairs(keys, ids, skeys, sids, n, 32, rtemp, rbytes, st);
    if (s != GSRAD_OK) return s;
    hipLaunchKernelGGL(k_copy_u32_to_i64, dim3(g), dim3(256), 0, st, sids, n, const_cast<int64_t *>(bd.order));
    return check_hip(hipGetLastError(), "batch ordering");
}

size_t batch_order_temp_bytes(int64_t n) { return 4 * ((size_t)n * 4 + 256) + radix_temp_bytes(n) + 256; }

gsrad_status launch_ragged_spmm(const BatchDev &bd, const Csr &F, int lpr, bool adjoint, const void *in, bool in_bf16,
                                const float *E, const float *rho, float *out, float *gE, uint32_t *counter,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
    const dim3 grid(persistent_blocks()), block(256);
#define RAGGED(L, A)                                                                                                 \
    do {                                                                                                             \
        if (in_bf16)                                                                                                 \
            hipLaunchKernelGGL((k_ragged_spmm<L, A, __bf16>), grid, block, 0, st, bd, F.row_ptr, F.col, F.val,      \
                               static_cast<const __bf16 *>(in), E, rho, out, gE, counter);                         \
        else                                                                                                         \
            hipLaunchKernelGGL((k_ragged_spmm<L, A, float>), grid, block, 0, st, bd, F.row_ptr, F.col, F.val,       \
                               static_cast<const float *>(in), E, rho, out, gE, counter);                          \
    } while (0)
    if (lpr == 64) {
        if (adjoint) RAGGED(64, true);
        else RAGGED(64, false);
    } else if (lpr == 32) {
        if (adjoint) RAGGED(32, true);
        else RAGGED(32, false);
    } else if (lpr == 16) {
        if (adjoint) RAGGED(16, true);
        else RAGGED(16, false);
    } else {
        set_error("ragged product: lanes per row must be 16, 32 or 64");
        return GSRAD_EINVAL;
    }
#undef RAGGED
    return check_hip(hipGetLastError(), "ragged product launch");
}

gsrad_status launch_ragged_sddmm(const BatchDev &bd, const Csr &F, int nb, int64_t vals, int max_C, const float *Bt,
                                 const float *Lt, const float *rho, float *grad_F, float *grad_rho, uint32_t *counter,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
    if (nb <= kFastNb && max_C <= 128)
        hipLaunchKernelGGL(k_ragged_sddmm_fast, dim3(persistent_blocks()), dim3(256), 0, st, bd, F.row_ptr, F.col,
                           F.val, nb, vals, Bt, Lt, rho, grad_F, grad_rho, counter);
    else
        hipLaunchKernelGGL(k_ragged_sddmm, dim3(persistent_blocks()), dim3(256), 0, st, bd, F.row_ptr, F.col, F.val,
                           nb, vals, Bt, Lt, rho, grad_F, grad_rho, counter);
    return check_hip(hipGetLastError(), "ragged sddmm launch");
}

}  // namespace gsrad

namespace gsrad {

namespace {

__global__ void __launch_bounds__(256) k_offset_copy_i32(const int32_t *__restrict__ in, int64_t n, int32_t add,
                                                         int32_t *__restrict__ out) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        out[k] = in[k] + add;
}

__global__ void __launch_bounds__(256) k_offset_copy_i64(const int64_t *__restrict__ in, int64_t n, int64_t add,
                                                         int64_t *__restrict__ out) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        out[k] = in[k] + add;
}

__global__ void __launch_bounds__(256) k_offset_widen(const int32_t *__restrict__ in, int64_t n, int64_t add,
                                                      int64_t *__restrict__ out) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        out[k] = (int64_t)in[k] + add;
}

__global__ void __launch_bounds__(256) k_copy_f32(const float *__restrict__ in, int64_t n, float *__restrict__ out) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) out[k] = in[k];
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

}  // namespace

gsrad_status launch_offset_copy_i32(const int32_t *in, int64_t n, int32_t add, int32_t *out, hipStream_t st) {
    if (n <= 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_offset_copy_i32, dim3(grid_for(n)), dim3(256), 0, st, in, n, add, out);
    return check_hip(hipGetLastError(), "offset copy launch");
}

gsrad_status launch_offset_widen(const int32_t *in, int64_t n, int64_t add, int64_t *out, hipStream_t st) {
    if (n <= 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_offset_widen, dim3(grid_for(n)), dim3(256), 0, st, in, n, add, out);
    return check_hip(hipGetLastError(), "offset widen launch");
}

gsrad_status launch_offset_copy_i64(const int64_t *in, int64_t n, int64_t add, int64_t *out, hipStream_t st) {
    if (n <= 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_offset_copy_i64, dim3(grid_for(n)), dim3(256), 0, st, in, n, add, out);
    return check_hip(hipGetLastError(), "offset copy launch");
}

__global__ void __launch_bounds__(256) k_round_bf16(const float *__restrict__ in, int64_t n, __bf16 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (__bf16)in[i];   // round to nearest even
}

gsrad_status launch_round_bf16(const float *in, int64_t n, void *out, hipStream_t st) {
    if (n <= 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, n,
                       static_cast<__bf16 *>(out));
    return check_hip(hipGetLastError(), "bf16 rounding launch");
}

gsrad_status launch_copy_f32(const float *in, int64_t n, float *out, hipStream_t st) {
    if (n <= 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n)), dim3(256), 0, st, in, n, out);
    return check_hip(hipGetLastError(), "copy launch");
}

}  // namespace gsrad
