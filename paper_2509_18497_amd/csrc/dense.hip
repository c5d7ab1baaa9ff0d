// Dense transport on the matrix cores: the bounce and adjoint products
// F B and F^T (rho * lambda) with F stored as BF16 and FP32 accumulation
// (v_mfma_f32_32x32x16_bf16), and the dense dL/dF = sum_k (rho lambda^(k+1))
// (B^(k))^T on split (hi + lo) operands.  Every product is one "NT" GEMM kernel: both operands are
// row-major with the reduction index contiguous, C[i][j] = sum_k A[i][k] B[j][k].
//
// Tiles: a 256-thread workgroup computes a 256 x 256 block of C, its four
// waves 128 x 128 each (4 x 4 MFMA tiles of 32 x 32, 256 accumulators per
// lane), K advanced 64 at a time through two LDS stages filled by direct
// global -> LDS buffer loads (no staging registers): the next K tile is in
// flight while the current one is multiplied.  LDS rows are unpadded with
// their 16-byte chunks XOR-permuted per row, which keeps the fragment reads
// of consecutive rows on distinct banks.  Tiles are numbered row-block
// major and handed to the XCDs in contiguous ranges, so the workgroups that
// share an A row-block (the large operand) run on one XCD and share its L2;
// the dL/dF product, whose operands are equally large, uses bands of eight
// tile rows instead.
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
typedef __attribute__((address_space(3))) void lds_void;
constexpr int kWaitVm0 = 0x0F70;   // s_waitcnt vmcnt(0), other counters unconstrained

constexpr int kBM = 256, kBN = 256, kBK = 64;
constexpr int kRowBytes = kBK * 2;                         // one LDS row: 8 chunks of 16 bytes
constexpr int kStageBytes = (kBM + kBN) * kRowBytes;      // A then B of one K tile (64 KiB)
constexpr size_t kGemmSmem = (size_t)2 * kStageBytes;     // two stages
constexpr int kBufFlags = 0x00020000;                     // raw buffer resource (stride 0) on CDNA

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

// LDS rows hold their eight 16-byte K chunks permuted: logical chunk q of
// tile row r sits at chunk q ^ swz(r), swz(r) = (r ^ (r >> 3)) & 7, so the
// fragment reads of 8 (or 16) consecutive rows at one logical chunk touch
// every bank once, without padding (the direct global -> LDS loads write
// 64 lanes x 16 bytes contiguously).
__device__ __forceinline__ int swz(int r) { return (r ^ (r >> 3)) & 7; }

// The 64-wide K tile of one wave's 128 x 128 block out of one stage: four
// 16-wide steps of sixteen 32 x 32 x 16 MFMAs, each step's fragments read
// while the previous step multiplies (two register sets).  Ab/Bb address
// the wave's row frow of A and B; fsw = swz(frow) (rows 32 mi + frow add
// 4 (mi & 1) to it), h = the lane's K half.
__device__ __forceinline__ void gemm_k_tile(const unsigned char *Ab, const unsigned char *Bb, int fsw, int h,
                                            f32x16 (&acc)[4][4]) {
    bf16x8 af[2][4], bf[2][4];
#define GEMM_FRAG(ks, i) (16 * ((2 * (ks) + h) ^ fsw ^ (((i) & 1) << 2)) + (i) * 32 * kRowBytes)
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) af[0][mi] = *reinterpret_cast<const bf16x8 *>(Ab + GEMM_FRAG(0, mi));
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) bf[0][ni] = *reinterpret_cast<const bf16x8 *>(Bb + GEMM_FRAG(0, ni));
#pragma unroll
    for (int ks = 0; ks < kBK / 16; ++ks) {
        const int cur = ks & 1, nxt = cur ^ 1;
        if (ks + 1 < kBK / 16) {
#pragma unroll
            for (int mi = 0; mi < 4; ++mi)
                af[nxt][mi] = *reinterpret_cast<const bf16x8 *>(Ab + GEMM_FRAG(ks + 1, mi));
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                bf[nxt][ni] = *reinterpret_cast<const bf16x8 *>(Bb + GEMM_FRAG(ks + 1, ni));
        }
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                acc[mi][ni] =
                    __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[cur][mi], bf[cur][ni], acc[mi][ni], 0, 0, 0);
    }
#undef GEMM_FRAG
}

struct Segs {
    const __bf16 *a[3];
    const __bf16 *b[3];
};

template <class Epi>
__global__ void __launch_bounds__(256) k_gemm_nt(Segs sg, int nseg, int64_t lda, int64_t ldb, int64_t kpad,
                                                 int tiles_n, int64_t ntiles, int group_m, Epi epi) {
    extern __shared__ __align__(16) unsigned char gemm_smem[];   // [2 stages][A 256 rows | B 256 rows]
    const int64_t t = xcd_block(blockIdx.x, ntiles);
    int64_t bm, bn;
    if (group_m > 0) {
        // column-major within bands of group_m tile rows: the 32 tiles an
        // XCD runs at once share group_m A blocks and 32/group_m B blocks
        const int64_t band = (int64_t)group_m * tiles_n, g = t / band, first = g * group_m;
        const int64_t rows = min(ntiles / tiles_n - first, (int64_t)group_m), r = t - g * band;
        bm = first + r % rows;
        bn = r / rows;
    } else {
        bm = t / tiles_n;
        bn = t % tiles_n;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = w >> 1, wn = w & 1;
    const int kt_per = (int)(kpad / kBK);
    const int KT = nseg * kt_per;
    f32x16 acc[4][4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][ni][r] = 0.0f;
    // Direct global -> LDS loads: wave w brings rows 64 w .. 64 w + 63 of
    // the A and the B tile, eight rows (1 KiB) per instruction; lane l
    // fills row 64 w + 8 i + l / 8, physical chunk l % 8, so it fetches the
    // logical chunk (l % 8) ^ swz(row) = (l % 8) ^ (l / 8) ^ i.  One buffer
    // resource per segment operand based at the workgroup's first row
    // (selected, not indexed: a dynamic index into the argument struct
    // would put it in scratch memory), the row step and K offset in SGPRs.
    const int lr = lane >> 3, lc = lane & 7;
    const int nra = kBM * (int)lda * 2, nrb = kBN * (int)ldb * 2;
#define GEMM_LOAD(kt, stage)                                                                             \
    do {                                                                                                 \
        const int s_ = (kt) / kt_per;                                                                    \
        const int k0_ = ((kt) - s_ * kt_per) * kBK * 2;                                                  \
        const __bf16 *A_ = (s_ == 0 ? sg.a[0] : s_ == 1 ? sg.a[1] : sg.a[2]) + bm * kBM * lda;           \
        const __bf16 *B_ = (s_ == 0 ? sg.b[0] : s_ == 1 ? sg.b[1] : sg.b[2]) + bn * kBN * ldb;           \
        const __amdgpu_buffer_rsrc_t ar_ = __builtin_amdgcn_make_buffer_rsrc((void *)A_, 0, nra, kBufFlags); \
        const __amdgpu_buffer_rsrc_t br_ = __builtin_amdgcn_make_buffer_rsrc((void *)B_, 0, nrb, kBufFlags); \
        unsigned char *ls_ = gemm_smem + (stage) * kStageBytes + w * 64 * kRowBytes;                     \
        GEMM_LOAD_ROWS(0); GEMM_LOAD_ROWS(1); GEMM_LOAD_ROWS(2); GEMM_LOAD_ROWS(3);                      \
        GEMM_LOAD_ROWS(4); GEMM_LOAD_ROWS(5); GEMM_LOAD_ROWS(6); GEMM_LOAD_ROWS(7);                      \
    } while (0)
#define GEMM_LOAD_ROWS(i)                                                                                \
    do {                                                                                                 \
        const int r_ = w * 64 + 8 * (i);                                                                 \
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ar_, (lds_void *)(ls_ + 8 * (i) * kRowBytes), 16,       \
                                                 lr * (int)lda * 2 + 16 * (lc ^ lr ^ (i)),               \
                                                 r_ * (int)lda * 2 + k0_, 0, 0);                         \
        __builtin_amdgcn_raw_ptr_buffer_load_lds(br_, (lds_void *)(ls_ + kBM * kRowBytes + 8 * (i) * kRowBytes), \
                                                 16, lr * (int)ldb * 2 + 16 * (lc ^ lr ^ (i)),           \
                                                 r_ * (int)ldb * 2 + k0_, 0, 0);                         \
    } while (0)
    const int frow = lane & 31, h = lane >> 5, fsw = swz(frow);
    const unsigned char *Aw = gemm_smem + (wm * 128 + frow) * kRowBytes;
    const unsigned char *Bw = gemm_smem + kBM * kRowBytes + (wn * 128 + frow) * kRowBytes;
    GEMM_LOAD(0, 0);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int st = kt & 1;
        // the next tile (the last one again at the end: in bounds, unused)
        // goes into the other stage, free since the previous barrier
        GEMM_LOAD(min(kt + 1, KT - 1), st ^ 1);
        gemm_k_tile(Aw + st * kStageBytes, Bw + st * kStageBytes, fsw, h, acc);
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
    }
#undef GEMM_LOAD_ROWS
#undef GEMM_LOAD
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
                         int64_t n_pad, const Epi &epi, hipStream_t st, int group_m = 0) {
    if (m_pad % kBM || n_pad % kBN || kpad % kBK || lda % 8 || ldb % 8 || nseg < 1 || nseg > 3) {
        set_error("dense product: operand shapes are not padded to the tile sizes");
        return GSRAD_EINVAL;
    }
    // buffer offsets within a 256-row block are 32-bit
    if (kpad > lda || kpad > ldb || lda > (1 << 22) || ldb > (1 << 22)) {
        set_error("dense product: rows longer than 2^22 elements or shorter than the reduction");
        return GSRAD_EINVAL;
    }
    const int tiles_n = (int)(n_pad / kBN);
    const int64_t ntiles = (m_pad / kBM) * tiles_n;
    gsrad_status e = check_hip(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_gemm_nt<Epi>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemmSmem),
                               "dense product LDS attribute");
    if (e != GSRAD_OK) return e;
    hipLaunchKernelGGL(k_gemm_nt<Epi>, dim3((unsigned)ntiles), dim3(256), kGemmSmem, st, sg, nseg, lda, ldb, kpad,
                       tiles_n, ntiles, group_m, epi);
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
    // both operands are n_pad x kpad: bands of 8 tile rows keep the blocks
    // that run together few enough to be read from L2
    return launch_gemm(sg, 3, ldk, ldk, kpad, ld_pad, ld_pad, epi, st, 8);
}

}  // namespace gsrad
