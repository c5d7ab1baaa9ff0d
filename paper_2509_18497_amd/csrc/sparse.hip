// Sparse transport kernels: CSR transpose (stable, deterministic), the
// bounce SpMM B <- E + rho * (F B), its adjoint on F^T, the sampled
// dense-dense product that yields dL/dF and dL/drho, and FP64 checks.
//
// Rows of B, E and the gradients hold C = Lt*K*3 contiguous floats; one
// wave64 owns one output row and its lanes own columns, so every gathered
// row of B is read with one coalesced access per wave.
#include "gsrad_internal.h"
#include "trace_api.h"

namespace gsrad {

namespace {

constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t g) {
    const int64_t x = b & 7, q = b >> 3, per = g >> 3, rem = g & 7;
    return x * per + (x < rem ? x : rem) + q;
}

__global__ void __launch_bounds__(256) k_expand_rows(const int64_t *__restrict__ row_ptr, int64_t n,
                                                     uint32_t *__restrict__ rows, uint32_t *__restrict__ keys_col,
                                                     const int32_t *__restrict__ col, uint32_t *__restrict__ ids) {
    const int64_t row = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / 64;
    if (row >= n) return;
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    for (int64_t k = b + __lane_id(); k < e; k += 64) {
        rows[k] = (uint32_t)row;
        keys_col[k] = (uint32_t)col[k];
        ids[k] = (uint32_t)k;
    }
}

// Row pointers of the transpose from the column-sorted keys: position p of
// the sorted list starts every column c with keys[p-1] < c <= keys[p]
// (keys[-1] = -1, keys[nnz] = n), so each of the n + 1 pointers is written
// exactly once.
__global__ void __launch_bounds__(256) k_col_bounds(const uint32_t *__restrict__ keys, int64_t nnz, int64_t n,
                                                    int64_t *__restrict__ t_row_ptr) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p > nnz) return;
    const int64_t a = p == 0 ? -1 : (int64_t)keys[p - 1];
    const int64_t b = p == nnz ? n : (int64_t)keys[p];
    for (int64_t c = a + 1; c <= b; ++c) t_row_ptr[c] = p;
}

__global__ void __launch_bounds__(256) k_transpose_gather(const uint32_t *__restrict__ sorted_ids,
                                                          const uint32_t *__restrict__ rows,
                                                          const float *__restrict__ val, int64_t nnz,
                                                          int32_t *__restrict__ t_col, float *__restrict__ t_val) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nnz) return;
    const uint32_t e = sorted_ids[k];
    t_col[k] = (int32_t)rows[e];
    t_val[k] = val[e];
}

// sum over the entries e in [b, e_end) of w_e * in[col_e][c] in CSR order,
// w_e = val_e (bounce) or val_e * rho[col_e][c % 3] (adjoint).  The wave
// reads 64 entries at a time and issues eight row gathers before it adds
// them, so eight loads are in flight per wave; the additions keep the CSR
// order, so the result is the plain sequential sum.  Lanes past C gather
// column 0 and discard it.
template <bool ADJ>
__device__ __forceinline__ float gather_row(const int32_t *__restrict__ col, const float *__restrict__ val,
                                            int64_t b, int64_t e_end, const float *__restrict__ in,
                                            const float *__restrict__ rho, int C, int c, int lane) {
    const int cc = c < C ? c : 0;
    const int colour = cc % 3;
    float acc = 0.0f;
    for (int64_t k0 = b; k0 < e_end; k0 += 64) {
        const int64_t kk = k0 + lane;
        const int jv = kk < e_end ? col[kk] : 0;
        const float vv = kk < e_end ? val[kk] : 0.0f;
        const int m = (int)min<int64_t>(64, e_end - k0);
        int q = 0;
        for (; q + 8 <= m; q += 8) {
            float w[8], x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = __builtin_amdgcn_readlane(jv, q + u);
                w[u] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), q + u));
                if (ADJ) w[u] *= rho[(int64_t)j * 3 + colour];
                x[u] = in[(int64_t)j * C + cc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = __builtin_fmaf(w[u], x[u], acc);
        }
        for (; q < m; ++q) {
            const int j = __builtin_amdgcn_readlane(jv, q);
            float w = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), q));
            if (ADJ) w *= rho[(int64_t)j * 3 + colour];
            acc = __builtin_fmaf(w, in[(int64_t)j * C + cc], acc);
        }
    }
    return acc;
}

// The same sums for NCH column chunks of 64 at once (columns c0 + 64 h +
// lane): the entries are read and broadcast once for all chunks and their
// gathers are in flight together; each column's FMAs keep the order of
// gather_row, so the results are the same bits.
template <bool ADJ, int NCH>
__device__ __forceinline__ void gather_rows(const int32_t *__restrict__ col, const float *__restrict__ val,
                                            int64_t b, int64_t e_end, const float *__restrict__ in,
                                            const float *__restrict__ rho, int C, int c0, int lane,
                                            float (&acc)[NCH]) {
    int cc[NCH], colour[NCH];
    bool has[NCH];
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
        const int c = c0 + 64 * h + lane;
        has[h] = c0 + 64 * h < C;
        cc[h] = c < C ? c : 0;
        colour[h] = cc[h] % 3;
        acc[h] = 0.0f;
    }
    for (int64_t k0 = b; k0 < e_end; k0 += 64) {
        const int64_t kk = k0 + lane;
        const int jv = kk < e_end ? col[kk] : 0;
        const float vv = kk < e_end ? val[kk] : 0.0f;
        const int m = (int)min<int64_t>(64, e_end - k0);
        int q = 0;
        for (; q + 8 <= m; q += 8) {
            float w[NCH][8], x[NCH][8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = __builtin_amdgcn_readlane(jv, q + u);
                const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), q + u));
#pragma unroll
                for (int h = 0; h < NCH; ++h) {
                    w[h][u] = v;
                    if (ADJ) w[h][u] *= rho[(int64_t)j * 3 + colour[h]];
                    x[h][u] = has[h] ? in[(int64_t)j * C + cc[h]] : 0.0f;
                }
            }
#pragma unroll
            for (int h = 0; h < NCH; ++h)
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[h] = __builtin_fmaf(w[h][u], x[h][u], acc[h]);
        }
        for (; q < m; ++q) {
            const int j = __builtin_amdgcn_readlane(jv, q);
            const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), q));
#pragma unroll
            for (int h = 0; h < NCH; ++h) {
                float w = v;
                if (ADJ) w *= rho[(int64_t)j * 3 + colour[h]];
                acc[h] = __builtin_fmaf(w, has[h] ? in[(int64_t)j * C + cc[h]] : 0.0f, acc[h]);
            }
        }
    }
}

constexpr int kRowChunks = 8;   // column chunks of 64 per pass when C > 64 (100 lights, C = 2700: one 6.6 s, four 5.5 s, eight 5.25 s per FP32 solve + backward)

// B_out[row] = E[row] + rho[row] * sum_e val[e] * B_in[col[e]]; NCH column
// chunks of 64 per pass (one for C <= 64, whose kernel keeps few registers)
template <int NCH>
__global__ void __launch_bounds__(256) k_bounce(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                const float *__restrict__ val, int64_t n, int C,
                                                const float *__restrict__ Bin, const float *__restrict__ E,
                                                const float *__restrict__ rho, float *__restrict__ Bout,
                                                int64_t nblocks, const int32_t *__restrict__ order) {
    const int64_t idx = xcd_block(blockIdx.x, nblocks) * kWavesPerBlock + threadIdx.x / 64;
    if (idx >= n) return;
    const int64_t row = order ? (int64_t)order[idx] : idx;
    const int lane = __lane_id();
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    if (NCH == 1) {
        for (int c0 = 0; c0 < C; c0 += 64) {
            const int c = c0 + lane;
            const float acc = gather_row<false>(col, val, b, e, Bin, nullptr, C, c, lane);
            if (c < C) Bout[row * C + c] = __builtin_fmaf(rho[row * 3 + c % 3], acc, E[row * C + c]);
        }
        return;
    }
    for (int c0 = 0; c0 < C; c0 += 64 * NCH) {
        float acc[NCH];
        gather_rows<false, NCH>(col, val, b, e, Bin, nullptr, C, c0, lane, acc);
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
            const int c = c0 + 64 * h + lane;
            if (c < C) Bout[row * C + c] = __builtin_fmaf(rho[row * 3 + c % 3], acc[h], E[row * C + c]);
        }
    }
}

// lam_out[row] = sum_e val[e] * rho[col] * lam_in[col];  gE[row] += lam_out[row]
template <int NCH>
__global__ void __launch_bounds__(256) k_adjoint(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                 const float *__restrict__ val, int64_t n, int C,
                                                 const float *__restrict__ lam_in, const float *__restrict__ rho,
                                                 float *__restrict__ lam_out, float *__restrict__ gE,
                                                 int64_t nblocks, const int32_t *__restrict__ order) {
    const int64_t idx = xcd_block(blockIdx.x, nblocks) * kWavesPerBlock + threadIdx.x / 64;
    if (idx >= n) return;
    const int64_t row = order ? (int64_t)order[idx] : idx;
    const int lane = __lane_id();
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    if (NCH == 1) {
        for (int c0 = 0; c0 < C; c0 += 64) {
            const int c = c0 + lane;
            const float acc = gather_row<true>(col, val, b, e, lam_in, rho, C, c, lane);
            if (c < C) {
                lam_out[row * C + c] = acc;
                gE[row * C + c] += acc;
            }
        }
        return;
    }
    for (int c0 = 0; c0 < C; c0 += 64 * NCH) {
        float acc[NCH];
        gather_rows<true, NCH>(col, val, b, e, lam_in, rho, C, c0, lane, acc);
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
            const int c = c0 + 64 * h + lane;
            if (c < C) {
                lam_out[row * C + c] = acc[h];
                gE[row * C + c] += acc[h];
            }
        }
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kSddE = 12;   // entries per pass of the general SDDMM (16: slower, 206 VGPRs)

// For each stored entry e = (row, j):
//   s_c = sum_k sum_{cols of colour c} lam^(k+1)[row] * B^(k)[j]
//   grad_F[e] = sum_c rho[row, c] s_c ;  grad_rho[row, c] = sum_e F[e] s_c
__global__ void __launch_bounds__(256) k_sddmm(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                               const float *__restrict__ val, int64_t n, int C, int nb,
                                               const float *__restrict__ Bt, const float *__restrict__ Lt,
                                               const float *__restrict__ rho, float *__restrict__ grad_F,
                                               float *__restrict__ grad_rho, int64_t nblocks, const int32_t *__restrict__ order) {
    const int64_t idx = xcd_block(blockIdx.x, nblocks) * kWavesPerBlock + threadIdx.x / 64;
    if (idx >= n) return;
    const int64_t row = order ? (int64_t)order[idx] : idx;
    const int lane = __lane_id();
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    const int64_t NC = n * (int64_t)C;
    const float r0 = rho[row * 3 + 0], r1 = rho[row * 3 + 1], r2 = rho[row * 3 + 2];
    float gr0 = 0.0f, gr1 = 0.0f, gr2 = 0.0f;
    // kSddE entries per pass: the row's lambda value of a (column, bounce) is
    // read once for all of them, and their gathers are in flight together;
    // each entry's sums run in the order of one entry at a time
    for (int64_t k = b; k < e; k += kSddE) {
        const int m = (int)min<int64_t>(kSddE, e - k);
        int64_t jj[kSddE];
#pragma unroll
        for (int u = 0; u < kSddE; ++u) jj[u] = u < m ? col[k + u] : col[k];
        float s0[kSddE], s1[kSddE], s2[kSddE];
#pragma unroll
        for (int u = 0; u < kSddE; ++u) s0[u] = s1[u] = s2[u] = 0.0f;
        for (int c = lane; c < C; c += 64) {
            float sum[kSddE];
#pragma unroll
            for (int u = 0; u < kSddE; ++u) sum[u] = 0.0f;
            for (int q = 0; q < nb; ++q) {
                const float l = Lt[q * NC + row * C + c];
#pragma unroll
                for (int u = 0; u < kSddE; ++u) sum[u] = __builtin_fmaf(l, Bt[q * NC + jj[u] * C + c], sum[u]);
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
                const float a0 = wave_sum(s0[u]), a1 = wave_sum(s1[u]), a2 = wave_sum(s2[u]);
                if (lane == 0 && grad_F) grad_F[k + u] = r0 * a0 + r1 * a1 + r2 * a2;
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

// The same sums for up to 8 bounces and C <= 64 (one column per lane): each
// lane keeps its column of rho_row-free lambda^(k+1)[row] for every k in
// registers, and four entries are gathered at a time (32 loads in flight)
// before their per-colour sums are reduced over the wave.  Per entry and
// lane the bounce sum runs in the same order, and the reductions and the
// grad_rho accumulation are those of k_sddmm, so both give the same bits.
constexpr int kSddmmMaxNb = 8;

__global__ void __launch_bounds__(256) k_sddmm_fast(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, const float *__restrict__ val,
                                                    int64_t n, int C, int nb, const float *__restrict__ Bt,
                                                    const float *__restrict__ Lt, const float *__restrict__ rho,
                                                    float *__restrict__ grad_F, float *__restrict__ grad_rho,
                                                    int64_t nblocks, const int32_t *__restrict__ order) {
    const int64_t idx = xcd_block(blockIdx.x, nblocks) * kWavesPerBlock + threadIdx.x / 64;
    if (idx >= n) return;
    const int64_t row = order ? (int64_t)order[idx] : idx;
    const int lane = __lane_id();
    const bool on = lane < C;
    const int c = on ? lane : 0;
    const int colour = c % 3;
    const int64_t NC = n * (int64_t)C;
    float lr[kSddmmMaxNb];
#pragma unroll
    for (int q = 0; q < kSddmmMaxNb; ++q) lr[q] = (q < nb && on) ? Lt[q * NC + row * C + c] : 0.0f;
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    const float r0 = rho[row * 3 + 0], r1 = rho[row * 3 + 1], r2 = rho[row * 3 + 2];
    float gr0 = 0.0f, gr1 = 0.0f, gr2 = 0.0f;
    constexpr int kE = 4;
    for (int64_t k0 = b; k0 < e; k0 += kE) {
        const int m = (int)min<int64_t>(kE, e - k0);
        float sv[kE];
#pragma unroll
        for (int u = 0; u < kE; ++u) {
            const int64_t j = u < m ? col[k0 + u] : col[k0];
            float x[kSddmmMaxNb];
#pragma unroll
            for (int q = 0; q < kSddmmMaxNb; ++q) x[q] = q < nb ? Bt[q * NC + j * C + c] : 0.0f;
            float sum = 0.0f;
#pragma unroll
            for (int q = 0; q < kSddmmMaxNb; ++q)
                if (q < nb) sum = __builtin_fmaf(lr[q], x[q], sum);
            sv[u] = on ? sum : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kE; ++u) {
            if (u >= m) break;
            float s0 = colour == 0 ? sv[u] : 0.0f;
            float s1 = colour == 1 ? sv[u] : 0.0f;
            float s2 = colour == 2 ? sv[u] : 0.0f;
            s0 = wave_sum(s0);
            s1 = wave_sum(s1);
            s2 = wave_sum(s2);
            const int64_t k = k0 + u;
            if (lane == 0 && grad_F) grad_F[k] = r0 * s0 + r1 * s1 + r2 * s2;
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

// FP64 residual of the fixed point and the other checks.
__global__ void __launch_bounds__(256) k_check(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                               const float *__restrict__ val, int64_t n, int C,
                                               const float *__restrict__ rho, const float *__restrict__ E,
                                               const float *__restrict__ B, double *acc) {
    const int64_t row = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / 64;
    if (row >= n) return;
    const int lane = __lane_id();
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    double r2 = 0.0, b2 = 0.0, bad = 0.0, rs = 0.0;
    for (int c = lane; c < C; c += 64) {
        double s = 0.0;
        for (int64_t k = b; k < e; ++k) s += (double)val[k] * (double)B[(int64_t)col[k] * C + c];
        const double Bi = B[row * C + c], Ei = E[row * C + c], ri = rho[row * 3 + c % 3];
        if (!isfinite(Bi) || !isfinite(Ei) || !isfinite(ri)) bad += 1.0;
        const double r = Ei + ri * s - Bi;
        r2 += r * r;
        b2 += Bi * Bi;
    }
    for (int64_t k = b + lane; k < e; k += 64) rs += (double)val[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        r2 += __shfl_xor(r2, o, 64);
        b2 += __shfl_xor(b2, o, 64);
        bad += __shfl_xor(bad, o, 64);
        rs += __shfl_xor(rs, o, 64);
    }
    if (lane == 0) {
        unsafeAtomicAdd(&acc[0], r2);
        unsafeAtomicAdd(&acc[1], b2);
        unsafeAtomicAdd(&acc[3], bad);
        // max of non-negative doubles through their bit patterns
        atomicMax(reinterpret_cast<unsigned long long *>(&acc[2]), (unsigned long long)__double_as_longlong(rs));
    }
}

// Reciprocity of the estimated operator (A_i F_ij = A_j F_ji for the exact
// form factors, App. E areas): per stored entry the FP64 difference with
// its mirror entry F_ji (binary search in row j; 0 if not stored).
// acc[0] += |A_i F_ij - A_j F_ji|, acc[1] += A_i F_ij,
// acc[2] = max |A_i F_ij - A_j F_ji| / max(A_i F_ij, A_j F_ji) (bit order).
__global__ void __launch_bounds__(256) k_reciprocity(const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const float *__restrict__ val,
                                                     int64_t n, const double *__restrict__ area, double *acc) {
    const int64_t row = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / 64;
    if (row >= n) return;
    const int lane = __lane_id();
    double sd = 0.0, sf = 0.0, mx = 0.0;
    const double ai = area[row];
    for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += 64) {
        const int64_t j = col[k];
        int64_t lo = row_ptr[j], hi = row_ptr[j + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (col[mid] < row) lo = mid + 1;
            else hi = mid;
        }
        const double fji = (lo < row_ptr[j + 1] && col[lo] == row) ? (double)val[lo] : 0.0;
        const double a = ai * (double)val[k], b = area[j] * fji;
        const double d = fabs(a - b);
        sd += d;
        sf += a;
        const double m = fmax(a, b);
        if (m > 0.0) mx = fmax(mx, d / m);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        sd += __shfl_xor(sd, o, 64);
        sf += __shfl_xor(sf, o, 64);
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    if (lane == 0) {
        unsafeAtomicAdd(&acc[0], sd);
        unsafeAtomicAdd(&acc[1], sf);
        atomicMax(reinterpret_cast<unsigned long long *>(&acc[2]), (unsigned long long)__double_as_longlong(mx));
    }
}

inline unsigned row_blocks(int64_t n) { return (unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock); }

}  // namespace

size_t transpose_temp_bytes(int64_t n, int64_t nnz) {
    size_t b = 0;
    b += 4 * ((size_t)nnz * 4 + 256);       // rows, keys, ids, sorted keys
    b += (size_t)nnz * 4 + 256;             // sorted ids
    b += radix_temp_bytes(nnz) + 256;
    return b;
}

static inline char *carve(char *&p, size_t bytes) {
    char *r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
}

gsrad_status csr_transpose(const Csr &A, int64_t *t_row_ptr, int32_t *t_col, float *t_val, void *temp,
                           size_t temp_bytes, hipStream_t st) {
    const int64_t n = A.n, nnz = A.nnz;
    char *p = static_cast<char *>(temp);
    uint32_t *rows = reinterpret_cast<uint32_t *>(carve(p, (size_t)nnz * 4));
    uint32_t *keys = reinterpret_cast<uint32_t *>(carve(p, (size_t)nnz * 4));
    uint32_t *ids = reinterpret_cast<uint32_t *>(carve(p, (size_t)nnz * 4));
    uint32_t *skeys = reinterpret_cast<uint32_t *>(carve(p, (size_t)nnz * 4));
    uint32_t *sids = reinterpret_cast<uint32_t *>(carve(p, (size_t)nnz * 4));
    const size_t rbytes = radix_temp_bytes(nnz);
    void *rtemp = carve(p, rbytes);
    if ((size_t)(p - static_cast<char *>(temp)) > temp_bytes) {
        set_error("transpose: temp too small");
        return GSRAD_EINVAL;
    }
    gsrad_status s;
    if (nnz > 0) {
        hipLaunchKernelGGL(k_expand_rows, dim3(row_blocks(n)), dim3(256), 0, st, A.row_ptr, n, rows, keys, A.col, ids);
        int bits = 1;
        while (bits < 32 && ((int64_t)1 << bits) < n) ++bits;
        s = radix_sort_pairs(keys, ids, skeys, sids, nnz, bits, rtemp, rbytes, st);
        if (s != GSRAD_OK) return s;
        hipLaunchKernelGGL(k_transpose_gather, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, sids, rows,
                           A.val, nnz, t_col, t_val);
    }
    hipLaunchKernelGGL(k_col_bounds, dim3((unsigned)((nnz + 1 + 255) / 256)), dim3(256), 0, st, skeys, nnz, n,
                       t_row_ptr);
    return check_hip(hipGetLastError(), "transpose");
}

gsrad_status launch_bounce(const Csr &F, int C, const float *Bin, const float *E, const float *rho, float *Bout,
                           hipStream_t st) {
    const unsigned g = row_blocks(F.n);
    hipLaunchKernelGGL(C <= 64 ? k_bounce<1> : k_bounce<kRowChunks>, dim3(g), dim3(256), 0, st, F.row_ptr, F.col, F.val, F.n, C, Bin, E, rho, Bout,
                       (int64_t)g, F.order);
    return check_hip(hipGetLastError(), "bounce launch");
}

gsrad_status launch_adjoint(const Csr &FT, int C, const float *lam_in, const float *rho, float *lam_out, float *gE,
                            hipStream_t st) {
    const unsigned g = row_blocks(FT.n);
    hipLaunchKernelGGL(C <= 64 ? k_adjoint<1> : k_adjoint<kRowChunks>, dim3(g), dim3(256), 0, st, FT.row_ptr, FT.col, FT.val, FT.n, C, lam_in, rho,
                       lam_out, gE, (int64_t)g, FT.order);
    return check_hip(hipGetLastError(), "adjoint launch");
}

gsrad_status launch_sddmm(const Csr &F, int C, int nb, const float *Btape, const float *Ltape, const float *rho,
                          float *grad_F, float *grad_rho, hipStream_t st) {
    const unsigned g = row_blocks(F.n);
    if (C <= 64 && nb <= kSddmmMaxNb)
        hipLaunchKernelGGL(k_sddmm_fast, dim3(g), dim3(256), 0, st, F.row_ptr, F.col, F.val, F.n, C, nb, Btape, Ltape,
                           rho, grad_F, grad_rho, (int64_t)g, F.order);
    else
        hipLaunchKernelGGL(k_sddmm, dim3(g), dim3(256), 0, st, F.row_ptr, F.col, F.val, F.n, C, nb, Btape, Ltape, rho,
                           grad_F, grad_rho, (int64_t)g, F.order);
    return check_hip(hipGetLastError(), "sddmm launch");
}

gsrad_status launch_reciprocity(const Csr &F, const double *area, double *acc, hipStream_t st) {
    if (F.n == 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_reciprocity, dim3(row_blocks(F.n)), dim3(256), 0, st, F.row_ptr, F.col, F.val, F.n, area, acc);
    return check_hip(hipGetLastError(), "reciprocity launch");
}

gsrad_status launch_check(const Csr &F, int C, const float *rho, const float *E, const float *B, double *acc,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_check, dim3(row_blocks(F.n)), dim3(256), 0, st, F.row_ptr, F.col, F.val, F.n, C, rho, E, B,
                       acc);
    return check_hip(hipGetLastError(), "check launch");
}

}  // namespace gsrad
