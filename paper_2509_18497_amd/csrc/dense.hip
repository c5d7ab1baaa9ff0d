// Dense transport on the matrix cores: the bounce and adjoint products
// F B and F^T (rho * lambda) with F stored as BF16 and FP32 accumulation
// (v_mfma_f32_32x32x16_bf16), and the dense dL/dF = sum_k (rho lambda^(k+1))
// (B^(k))^T on split (hi + lo) operands.  Every product is one "NT" GEMM kernel: both operands are
// row-major with the reduction index contiguous, C[i][j] = sum_k A[i][k] B[j][k].
//
// Tiles: a 256-thread workgroup computes a 256 x 256 block of C, its four
// waves 128 x 128 each (4 x 4 MFMA tiles of 32 x 32, 256 accumulators per
// lane), K advanced 64 at a time through a double-buffered LDS stage
// (rows padded to 72 BF16 = 144 B, which keeps the 16-byte fragment reads
// of 16 consecutive rows on distinct banks).  Tiles are numbered row-block
// major and handed to the XCDs in contiguous ranges, so the workgroups that
// share an A row-block (the large operand) run on one XCD and share its L2.
//
// A K range may be split into up to three segments with their own A and B
// (the correction sweep sums F_hi X_hi + F_hi X_lo + F_lo X_hi in one pass).
#include "gsrad_internal.h"
#include "dense_api.h"

namespace gsrad {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 16-byte register chunk

constexpr int kBM = 256, kBN = 256, kBK = 64;
constexpr int kPitch = kBK + 8;   // LDS row pitch (BF16 elements)
constexpr size_t kGemmSmem = (size_t)2 * (kBM + kBN) * kPitch * sizeof(__bf16);

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t g) {
    const int64_t x = b & 7, q = b >> 3, per = g >> 3, rem = g & 7;
    return x * per + (x < rem ? x : rem) + q;
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

// Four BF16 values of consecutive rows i..i+3 of column c of a transposed
// [c][i] array, as one 8-byte store when all four rows exist.
__device__ __forceinline__ void store_t4(__bf16 *base, int64_t ld, int64_t c, int64_t i, int nvalid, const __bf16 (&v)[4]) {
    __bf16 *p = base + c * ld + i;
    if (nvalid == 4) {
        union {
            __bf16 h[4];
            uint2 u;
        } pk;
        pk.h[0] = v[0];
        pk.h[1] = v[1];
        pk.h[2] = v[2];
        pk.h[3] = v[3];
        *reinterpret_cast<uint2 *>(p) = pk.u;
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r < nvalid) p[r] = v[r];
    }
}

// Forward bounce epilogue: Q = acc = (F B^(k))[i][c], B^(k+1) = E + rho Q.
struct EpiBounce {
    const float *E, *rho;
    int64_t n;
    int C;
    float *Bout;          // [n][C] FP32, or null
    float *Q;             // [n][C] FP32 tape slot, or null
    __bf16 *xt_hi;        // next operand, transposed [Cp][ldx], or null
    __bf16 *xt_lo;        // its low part (B - hi), or null
    int64_t ldx;
    __bf16 *bb, *bb_lo;   // [n][ldbb] BF16 copy (hi, lo) of B^(k+1) at column offset boff, or null
    int64_t ldbb, boff;
    __device__ __forceinline__ void operator()(int64_t i, int64_t c, const float (&v)[4]) const {
        if (c >= C) return;
        const int nv = (int)min<int64_t>(4, n - i);
        if (nv <= 0) return;
        __bf16 hi[4], lo[4];
        const int colour = (int)(c % 3);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            hi[r] = lo[r] = to_bf16(0.0f);
            if (r >= nv) continue;
            const int64_t ii = i + r;
            const float q = v[r];
            const float b = __builtin_fmaf(rho[ii * 3 + colour], q, E[ii * C + c]);
            if (Bout) Bout[ii * C + c] = b;
            if (Q) Q[ii * C + c] = q;
            hi[r] = to_bf16(b);
            lo[r] = to_bf16(b - from_bf16(hi[r]));
            if (bb) {
                bb[ii * ldbb + boff + c] = hi[r];
                bb_lo[ii * ldbb + boff + c] = lo[r];
            }
        }
        if (xt_hi) store_t4(xt_hi, ldx, c, i, nv, hi);
        if (xt_lo) store_t4(xt_lo, ldx, c, i, nv, lo);
    }
};

// Adjoint epilogue: lambda^(k) = acc = (F^T (rho lambda^(k+1)))[j][c];
// dL/dE += lambda^(k); next operand rho * lambda^(k) (transposed BF16) and
// its BF16 copy for the dense dL/dF.
struct EpiAdjoint {
    const float *rho;
    int64_t n;
    int C;
    float *lam;           // [n][C] FP32
    float *gE;            // [n][C] FP32, accumulated
    __bf16 *yt_hi;        // [Cp][ldx], or null
    int64_t ldx;
    __bf16 *p, *p_lo;     // [n][ldp] (hi, lo) at column offset poff, or null
    int64_t ldp, poff;
    __device__ __forceinline__ void operator()(int64_t i, int64_t c, const float (&v)[4]) const {
        if (c >= C) return;
        const int nv = (int)min<int64_t>(4, n - i);
        if (nv <= 0) return;
        __bf16 hi[4];
        const int colour = (int)(c % 3);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            hi[r] = to_bf16(0.0f);
            if (r >= nv) continue;
            const int64_t ii = i + r;
            const float l = v[r];
            lam[ii * C + c] = l;
            gE[ii * C + c] += l;
            const float y = rho[ii * 3 + colour] * l;
            hi[r] = to_bf16(y);
            if (p) {
                p[ii * ldp + poff + c] = hi[r];
                p_lo[ii * ldp + poff + c] = to_bf16(y - from_bf16(hi[r]));
            }
        }
        if (yt_hi) store_t4(yt_hi, ldx, c, i, nv, hi);
    }
};

// Plain FP32 store of C[i][j] for i < m, j < ncol.
struct EpiStore {
    float *out;
    int64_t ld, m, ncol;
    __device__ __forceinline__ void operator()(int64_t i, int64_t j, const float (&v)[4]) const {
        if (j >= ncol) return;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (i + r < m) out[(i + r) * ld + j] = v[r];
    }
};

// Epilogue of one 32 x 32 accumulator tile: register r of lane l holds
// row (r/4)*8 + (l/32)*4 + r%4 and column l%32 of the tile; i, j are the
// lane's first row and its column.
template <class Epi>
__device__ __forceinline__ void epi_tile(const Epi &epi, const f32x16 &a, int64_t i, int64_t j) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float v[4] = {a[g * 4 + 0], a[g * 4 + 1], a[g * 4 + 2], a[g * 4 + 3]};
        epi(i + g * 8, j, v);
    }
}

struct Segs {
    const __bf16 *a[3];
    const __bf16 *b[3];
};

template <class Epi>
__global__ void __launch_bounds__(256) k_gemm_nt(Segs sg, int nseg, int64_t lda, int64_t ldb, int64_t kpad,
                                                 int tiles_n, int64_t ntiles, Epi epi) {
    extern __shared__ __align__(16) unsigned char gemm_smem[];
    __bf16 *As = reinterpret_cast<__bf16 *>(gemm_smem);   // [2][kBM][kPitch]
    __bf16 *Bs = As + 2 * kBM * kPitch;                     // [2][kBN][kPitch]
    const int64_t t = xcd_block(blockIdx.x, ntiles);
    const int64_t bm = t / tiles_n, bn = t % tiles_n;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int kt_per = (int)(kpad / kBK);
    const int KT = nseg * kt_per;
    u32x4 ra[8], rb[8];
    f32x16 acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;
    const int frow = lane & 31, fk = 8 * (lane >> 5);
    // global -> registers of K tile kt (select, not index, the segment's
    // operands: a dynamic index into the argument struct would put it in
    // scratch memory)
#define GEMM_GLOAD(kt)                                                                                   \
    do {                                                                                                 \
        const int s_ = (kt) / kt_per;                                                                    \
        const int64_t k0_ = (int64_t)((kt) - s_ * kt_per) * kBK;                                         \
        const __bf16 *A_ = (s_ == 0 ? sg.a[0] : s_ == 1 ? sg.a[1] : sg.a[2]) + bm * kBM * lda + k0_;     \
        const __bf16 *B_ = (s_ == 0 ? sg.b[0] : s_ == 1 ? sg.b[1] : sg.b[2]) + bn * kBN * ldb + k0_;     \
        const __bf16 *a_ = A_ + (tid >> 3) * lda + (tid & 7) * 8;                                        \
        const __bf16 *b_ = B_ + (tid >> 3) * ldb + (tid & 7) * 8;                                        \
        ra[0] = *reinterpret_cast<const u32x4 *>(a_);                                                    \
        ra[1] = *reinterpret_cast<const u32x4 *>(a_ + 32 * lda);                                         \
        ra[2] = *reinterpret_cast<const u32x4 *>(a_ + 64 * lda);                                         \
        ra[3] = *reinterpret_cast<const u32x4 *>(a_ + 96 * lda);                                         \
        ra[4] = *reinterpret_cast<const u32x4 *>(a_ + 128 * lda);                                        \
        ra[5] = *reinterpret_cast<const u32x4 *>(a_ + 160 * lda);                                        \
        ra[6] = *reinterpret_cast<const u32x4 *>(a_ + 192 * lda);                                        \
        ra[7] = *reinterpret_cast<const u32x4 *>(a_ + 224 * lda);                                        \
        rb[0] = *reinterpret_cast<const u32x4 *>(b_);                                                    \
        rb[1] = *reinterpret_cast<const u32x4 *>(b_ + 32 * ldb);                                         \
        rb[2] = *reinterpret_cast<const u32x4 *>(b_ + 64 * ldb);                                         \
        rb[3] = *reinterpret_cast<const u32x4 *>(b_ + 96 * ldb);                                         \
        rb[4] = *reinterpret_cast<const u32x4 *>(b_ + 128 * ldb);                                        \
        rb[5] = *reinterpret_cast<const u32x4 *>(b_ + 160 * ldb);                                        \
        rb[6] = *reinterpret_cast<const u32x4 *>(b_ + 192 * ldb);                                        \
        rb[7] = *reinterpret_cast<const u32x4 *>(b_ + 224 * ldb);                                        \
    } while (0)
#define GEMM_LSTORE(buf)                                                                                 \
    do {                                                                                                 \
        __bf16 *la_ = As + ((buf) * kBM + (tid >> 3)) * kPitch + (tid & 7) * 8;                          \
        __bf16 *lb_ = Bs + ((buf) * kBN + (tid >> 3)) * kPitch + (tid & 7) * 8;                          \
        *reinterpret_cast<u32x4 *>(la_) = ra[0];                                                         \
        *reinterpret_cast<u32x4 *>(la_ + 32 * kPitch) = ra[1];                                           \
        *reinterpret_cast<u32x4 *>(la_ + 64 * kPitch) = ra[2];                                           \
        *reinterpret_cast<u32x4 *>(la_ + 96 * kPitch) = ra[3];                                           \
        *reinterpret_cast<u32x4 *>(la_ + 128 * kPitch) = ra[4];                                          \
        *reinterpret_cast<u32x4 *>(la_ + 160 * kPitch) = ra[5];                                          \
        *reinterpret_cast<u32x4 *>(la_ + 192 * kPitch) = ra[6];                                          \
        *reinterpret_cast<u32x4 *>(la_ + 224 * kPitch) = ra[7];                                          \
        *reinterpret_cast<u32x4 *>(lb_) = rb[0];                                                         \
        *reinterpret_cast<u32x4 *>(lb_ + 32 * kPitch) = rb[1];                                           \
        *reinterpret_cast<u32x4 *>(lb_ + 64 * kPitch) = rb[2];                                           \
        *reinterpret_cast<u32x4 *>(lb_ + 96 * kPitch) = rb[3];                                           \
        *reinterpret_cast<u32x4 *>(lb_ + 128 * kPitch) = rb[4];                                          \
        *reinterpret_cast<u32x4 *>(lb_ + 160 * kPitch) = rb[5];                                          \
        *reinterpret_cast<u32x4 *>(lb_ + 192 * kPitch) = rb[6];                                          \
        *reinterpret_cast<u32x4 *>(lb_ + 224 * kPitch) = rb[7];                                          \
    } while (0)
    GEMM_GLOAD(0);
    GEMM_LSTORE(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < KT) GEMM_GLOAD(kt + 1);
        const __bf16 *Ab = As + buf * kBM * kPitch + (wm * 128 + frow) * kPitch + fk;
        const __bf16 *Bb = Bs + buf * kBN * kPitch + (wn * 128 + frow) * kPitch + fk;
        // fragments of the next 16-wide K step are read while the sixteen
        // MFMAs of the current one run (two register sets)
        bf16x8 af[2][4], bf[2][4];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) af[0][mi] = *reinterpret_cast<const bf16x8 *>(Ab + mi * 32 * kPitch);
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) bf[0][ni] = *reinterpret_cast<const bf16x8 *>(Bb + ni * 32 * kPitch);
#pragma unroll
        for (int ks = 0; ks < kBK / 16; ++ks) {
            const int cur = ks & 1, nxt = cur ^ 1;
            if (ks + 1 < kBK / 16) {
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
                    af[nxt][mi] = *reinterpret_cast<const bf16x8 *>(Ab + mi * 32 * kPitch + (ks + 1) * 16);
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    bf[nxt][ni] = *reinterpret_cast<const bf16x8 *>(Bb + ni * 32 * kPitch + (ks + 1) * 16);
            }
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] =
                        __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[cur][mi], bf[cur][ni], acc[mi][ni], 0, 0, 0);
        }
        // issue order: the first step's eight LDS reads, then each step's
        // sixteen MFMAs with the next step's reads slotted between the first
        // eight of them
        __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
#pragma unroll
        for (int ks = 0; ks + 1 < kBK / 16; ++ks) {
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
        if (kt + 1 < KT) GEMM_LSTORE(buf ^ 1);
        __syncthreads();
    }
#undef GEMM_GLOAD
#undef GEMM_LSTORE
    // accumulator register r of lane l holds row (r/4)*8 + (l/32)*4 + r%4,
    // column l%32 of its 32 x 32 tile
    const int64_t i0 = bm * kBM + wm * 128 + (lane >> 5) * 4, j0 = bn * kBN + wn * 128 + (lane & 31);
    // sixteen explicit tile calls: a loop over the accumulator array that
    // the compiler does not unroll would leave it in scratch memory
#define GEMM_EPI(mi, ni) epi_tile(epi, acc[mi][ni], i0 + (mi) * 32, j0 + (ni) * 32)
    GEMM_EPI(0, 0); GEMM_EPI(0, 1); GEMM_EPI(0, 2); GEMM_EPI(0, 3);
    GEMM_EPI(1, 0); GEMM_EPI(1, 1); GEMM_EPI(1, 2); GEMM_EPI(1, 3);
    GEMM_EPI(2, 0); GEMM_EPI(2, 1); GEMM_EPI(2, 2); GEMM_EPI(2, 3);
    GEMM_EPI(3, 0); GEMM_EPI(3, 1); GEMM_EPI(3, 2); GEMM_EPI(3, 3);
#undef GEMM_EPI
}

// Dense BF16 copies of F (rows i) and F^T (rows j) from the CSR: the value
// rounded to BF16 (hi) and the rounded remainder (lo), so hi + lo carries
// 16 significant bits.  The arrays are zero except at the stored entries.
__global__ void __launch_bounds__(256) k_dense_scatter(const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col, const float *__restrict__ val,
                                                       int64_t n, int64_t ld, __bf16 *f_hi, __bf16 *f_lo,
                                                       __bf16 *ft_hi, __bf16 *ft_lo) {
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (row >= n) return;
    for (int64_t e = row_ptr[row] + __lane_id(); e < row_ptr[row + 1]; e += 64) {
        const int64_t j = col[e];
        const float v = val[e];
        const __bf16 h = to_bf16(v);
        const __bf16 l = to_bf16(v - from_bf16(h));
        f_hi[row * ld + j] = h;
        f_lo[row * ld + j] = l;
        ft_hi[j * ld + row] = h;
        ft_lo[j * ld + row] = l;
    }
}

// Transposed BF16 operand from an FP32 [n][C] array (optionally scaled by
// rho per colour): out_hi[c][i] = bf16(s x), out_lo[c][i] = bf16(s x - hi).
// 32 x 32 tiles through LDS so both sides are accessed row by row.
__global__ void __launch_bounds__(256) k_to_bf16_t(const float *__restrict__ x, const float *__restrict__ rho,
                                                   int64_t n, int C, __bf16 *out_hi, __bf16 *out_lo, int64_t ld) {
    __shared__ float tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32;
    const int c0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + r;
        const int c = c0 + tx;
        float v = 0.0f;
        if (i < n && c < C) {
            v = x[i * C + c];
            if (rho) v *= rho[i * 3 + c % 3];
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int c = c0 + r;
        const int64_t i = i0 + tx;
        if (c < C && i < n) {
            const float v = tile[tx][r];
            const __bf16 h = to_bf16(v);
            out_hi[c * ld + i] = h;
            if (out_lo) out_lo[c * ld + i] = to_bf16(v - from_bf16(h));
        }
    }
}

// Row-major BF16 copy (hi and lo parts) of an FP32 [n][C] array
// (optionally scaled by rho) into columns [off, off + C) of out [n][ld].
__global__ void __launch_bounds__(256) k_to_bf16_rows(const float *__restrict__ x, const float *__restrict__ rho,
                                                      int64_t n, int C, __bf16 *out, __bf16 *out_lo, int64_t ld,
                                                      int64_t off) {
    const int64_t total = n * C;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / C;
        const int c = (int)(e - i * C);
        float v = x[e];
        if (rho) v *= rho[i * 3 + c % 3];
        const __bf16 h = to_bf16(v);
        out[i * ld + off + c] = h;
        if (out_lo) out_lo[i * ld + off + c] = to_bf16(v - from_bf16(h));
    }
}

// grad_rho[i][col] += sum over c with c % 3 == col of lam[i][c] * Q[i][c]
// (one wave per row).
__global__ void __launch_bounds__(256) k_grad_rho_acc(const float *__restrict__ lam, const float *__restrict__ Q,
                                                      int64_t n, int C, float *__restrict__ grad_rho) {
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (row >= n) return;
    const int lane = __lane_id();
    float s[3] = {0.0f, 0.0f, 0.0f};
    for (int c = lane; c < C; c += 64) {
        const float p = lam[row * C + c] * Q[row * C + c];
        const int k = c % 3;
        s[0] += k == 0 ? p : 0.0f;
        s[1] += k == 1 ? p : 0.0f;
        s[2] += k == 2 ? p : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int o = 32; o >= 1; o >>= 1) s[k] += __shfl_xor(s[k], o, 64);
    if (lane < 3) grad_rho[row * 3 + lane] += s[lane];
}

// grad_F[e] = G[i][col[e]] for the stored entries of row i (one wave per row).
__global__ void __launch_bounds__(256) k_gather_csr(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, int64_t n,
                                                    const float *__restrict__ G, int64_t ld, float *__restrict__ out) {
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (row >= n) return;
    for (int64_t e = row_ptr[row] + __lane_id(); e < row_ptr[row + 1]; e += 64) out[e] = G[row * ld + col[e]];
}

template <class Epi>
gsrad_status launch_gemm(const Segs &sg, int nseg, int64_t lda, int64_t ldb, int64_t kpad, int64_t m_pad,
                         int64_t n_pad, const Epi &epi, hipStream_t st) {
    if (m_pad % kBM || n_pad % kBN || kpad % kBK || lda % 8 || ldb % 8 || nseg < 1 || nseg > 3) {
        set_error("dense product: operand shapes are not padded to the tile sizes");
        return GSRAD_EINVAL;
    }
    const int tiles_n = (int)(n_pad / kBN);
    const int64_t ntiles = (m_pad / kBM) * tiles_n;
    gsrad_status e = check_hip(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_gemm_nt<Epi>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmSmem),
                               "dense product LDS attribute");
    if (e != GSRAD_OK) return e;
    hipLaunchKernelGGL(k_gemm_nt<Epi>, dim3((unsigned)ntiles), dim3(256), kGemmSmem, st, sg, nseg, lda, ldb, kpad,
                       tiles_n, ntiles, epi);
    return check_hip(hipGetLastError(), "dense product launch");
}

}  // namespace

int64_t dense_pad(int64_t x) { return (x + 255) / 256 * 256; }

gsrad_status launch_dense_scatter(const Csr &F, int64_t ld, __bf16 *f_hi, __bf16 *f_lo, __bf16 *ft_hi, __bf16 *ft_lo,
                                  hipStream_t st) {
    if (F.n == 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_dense_scatter, dim3((unsigned)((F.n + 3) / 4)), dim3(256), 0, st, F.row_ptr, F.col, F.val,
                       F.n, ld, f_hi, f_lo, ft_hi, ft_lo);
    return check_hip(hipGetLastError(), "dense scatter launch");
}

gsrad_status launch_to_bf16_t(const float *x, const float *rho, int64_t n, int C, __bf16 *hi, __bf16 *lo, int64_t ld,
                              hipStream_t st) {
    if (n == 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_to_bf16_t, dim3((unsigned)((n + 31) / 32), (unsigned)((C + 31) / 32)), dim3(256), 0, st, x,
                       rho, n, C, hi, lo, ld);
    return check_hip(hipGetLastError(), "bf16 transpose launch");
}

gsrad_status launch_to_bf16_rows(const float *x, const float *rho, int64_t n, int C, __bf16 *out, __bf16 *out_lo,
                                 int64_t ld, int64_t off, hipStream_t st) {
    if (n == 0) return GSRAD_OK;
    const int64_t total = n * C;
    const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_to_bf16_rows, dim3(g), dim3(256), 0, st, x, rho, n, C, out, out_lo, ld, off);
    return check_hip(hipGetLastError(), "bf16 rows launch");
}

gsrad_status launch_grad_rho_acc(const float *lam, const float *Q, int64_t n, int C, float *grad_rho,
                                 hipStream_t st) {
    if (n == 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_grad_rho_acc, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, lam, Q, n, C, grad_rho);
    return check_hip(hipGetLastError(), "grad_rho launch");
}

gsrad_status launch_gather_csr(const Csr &F, const float *G, int64_t ld, float *out, hipStream_t st) {
    if (F.n == 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_gather_csr, dim3((unsigned)((F.n + 3) / 4)), dim3(256), 0, st, F.row_ptr, F.col, F.n, G, ld,
                       out);
    return check_hip(hipGetLastError(), "gather launch");
}

gsrad_status launch_dense_bounce(const DenseBounce &a, hipStream_t st) {
    Segs sg = {};
    int nseg = 1;
    sg.a[0] = a.f_hi;
    sg.b[0] = a.x_hi;
    if (a.split) {
        sg.a[1] = a.f_hi;
        sg.b[1] = a.x_lo;
        sg.a[2] = a.f_lo;
        sg.b[2] = a.x_hi;
        nseg = 3;
    }
    EpiBounce epi{a.E, a.rho, a.n, a.C, a.Bout, a.Q, a.xt_hi, a.xt_lo, a.ldx, a.bb, a.bb_lo, a.ldbb, a.boff};
    return launch_gemm(sg, nseg, a.ld, a.ldx, a.ld, a.ld, dense_pad(a.C), epi, st);
}

gsrad_status launch_dense_adjoint(const DenseAdjoint &a, hipStream_t st) {
    Segs sg = {};
    int nseg = 1;
    sg.a[0] = a.ft_hi;
    sg.b[0] = a.y_hi;
    if (a.split) {
        sg.a[1] = a.ft_hi;
        sg.b[1] = a.y_lo;
        sg.a[2] = a.ft_lo;
        sg.b[2] = a.y_hi;
        nseg = 3;
    }
    EpiAdjoint epi{a.rho, a.n, a.C, a.lam, a.gE, a.yt_hi, a.ldx, a.p, a.p_lo, a.ldp, a.poff};
    return launch_gemm(sg, nseg, a.ld, a.ldx, a.ld, a.ld, dense_pad(a.C), epi, st);
}

gsrad_status launch_dense_grad_F(const __bf16 *P, const __bf16 *P_lo, const __bf16 *Bb, const __bf16 *Bb_lo,
                                 int64_t ldk, int64_t kpad, int64_t n, int64_t ld_pad, float *G, int64_t ldg,
                                 hipStream_t st) {
    Segs sg = {};
    sg.a[0] = P;
    sg.b[0] = Bb;
    sg.a[1] = P;
    sg.b[1] = Bb_lo;
    sg.a[2] = P_lo;
    sg.b[2] = Bb;
    EpiStore epi{G, ldg, n, n};
    return launch_gemm(sg, 3, ldk, ldk, kpad, ld_pad, ld_pad, epi, st);
}

}  // namespace gsrad
