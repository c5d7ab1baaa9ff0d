// Device-wide exclusive scan and stable LSD radix sort (digits of up to 9
// bits) for wave64.  Used for Morton-code ordering of the surfels and for the
// deterministic CSR transpose of F.
#include "gsrad_internal.h"

namespace gsrad {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kWaves = kSortThreads / 64;
constexpr int kMaxDigitBits = 9;
constexpr int kMaxBins = 1 << kMaxDigitBits;   // two per thread

__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (blockDim == 256).
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total) {
    __shared__ T wsum[kScanThreads / 64];
    const int lane = lane_id(), w = threadIdx.x / 64;
    const T inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

template <typename In>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const In *__restrict__ in, uint64_t *__restrict__ sums,
                                                            int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += (uint64_t)in[i];
    }
    uint64_t tot;
    block_exclusive_scan<uint64_t>(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = offset[tile] + exclusive prefix within the tile; out[n] = total.
template <typename In>
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const In *in, int64_t *out,
                                                            const uint64_t *__restrict__ tile_off, int64_t n,
                                                            int write_total) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? (uint64_t)in[i] : 0;
        s += v[k];
    }
    uint64_t tot;
    uint64_t run = block_exclusive_scan<uint64_t>(s, &tot) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i < n) out[i] = (int64_t)run;
        run += v[k];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) {
        const uint64_t off = tile_off ? tile_off[blockIdx.x] : 0;
        out[n] = (int64_t)(off + tot);
    }
}

// exclusive scan of uint64 tile sums in place (recursive levels)
gsrad_status scan_u64_inplace(uint64_t *data, int64_t n, char *temp, size_t temp_bytes, hipStream_t st);

int64_t n_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

}  // namespace

size_t scan_temp_bytes(int64_t n) {
    size_t bytes = 0;
    int64_t m = n;
    do {
        m = n_tiles(m);
        bytes += ((size_t)(m + 1) * sizeof(uint64_t) + 255) / 256 * 256;
    } while (m > 1);
    return bytes + 4096;
}

namespace {

// Scans `data` (uint64, n values) into exclusive prefix form, in place:
// every thread of k_tile_scan reads and writes only its own items.
gsrad_status scan_u64_inplace(uint64_t *data, int64_t n, char *temp, size_t temp_bytes, hipStream_t st) {
    if (n <= 0) return GSRAD_OK;
    const int64_t nt = n_tiles(n);
    int64_t *out = reinterpret_cast<int64_t *>(data);
    if (nt == 1) {
        hipLaunchKernelGGL(k_tile_scan<uint64_t>, dim3(1), dim3(kScanThreads), 0, st, data, out, nullptr, n, 0);
        return check_hip(hipGetLastError(), "scan launch");
    }
    uint64_t *sums = reinterpret_cast<uint64_t *>(temp);
    char *rest = temp + ((size_t)(nt + 1) * sizeof(uint64_t) + 255) / 256 * 256;
    if ((size_t)(rest - temp) > temp_bytes) {
        set_error("scan: temp too small");
        return GSRAD_EINVAL;
    }
    hipLaunchKernelGGL(k_tile_sums<uint64_t>, dim3((unsigned)nt), dim3(kScanThreads), 0, st, data, sums, n);
    gsrad_status s = scan_u64_inplace(sums, nt, rest, temp_bytes - (size_t)(rest - temp), st);
    if (s != GSRAD_OK) return s;
    hipLaunchKernelGGL(k_tile_scan<uint64_t>, dim3((unsigned)nt), dim3(kScanThreads), 0, st, data, out, sums, n, 0);
    return check_hip(hipGetLastError(), "scan launch");
}

}  // namespace

gsrad_status exclusive_scan_u32_i64(const uint32_t *in, int64_t *out, int64_t n, void *temp, size_t temp_bytes,
                                    hipStream_t st) {
    if (n <= 0) {
        return check_hip(hipMemsetAsync(out, 0, sizeof(int64_t), st), "scan memset");
    }
    const int64_t nt = n_tiles(n);
    char *t = static_cast<char *>(temp);
    uint64_t *sums = reinterpret_cast<uint64_t *>(t);
    char *rest = t + ((size_t)(nt + 1) * sizeof(uint64_t) + 255) / 256 * 256;
    if (nt > 1) {
        hipLaunchKernelGGL(k_tile_sums<uint32_t>, dim3((unsigned)nt), dim3(kScanThreads), 0, st, in, sums, n);
        gsrad_status s = scan_u64_inplace(sums, nt, rest, temp_bytes - (size_t)(rest - t), st);
        if (s != GSRAD_OK) return s;
    }
    hipLaunchKernelGGL(k_tile_scan<uint32_t>, dim3((unsigned)nt), dim3(kScanThreads), 0, st, in, out,
                       nt > 1 ? sums : nullptr, n, 1);
    return check_hip(hipGetLastError(), "scan launch");
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
namespace {

__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                             int dbits, uint32_t *__restrict__ hist, int64_t nb) {
    __shared__ uint32_t cnt[kMaxBins];
    const uint32_t mask = (1u << dbits) - 1u;
    const int bins = 1 << dbits;
    for (int d = threadIdx.x; d < bins; d += kSortThreads) cnt[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < bins; d += kSortThreads) hist[(int64_t)d * nb + blockIdx.x] = cnt[d];
}

// Stable scatter: the item order inside a tile is (round, thread), which is
// the input order, and ranks are assigned in that order.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(const uint32_t *__restrict__ keys,
                                                                const uint32_t *__restrict__ vals, uint32_t *kout,
                                                                uint32_t *vout, int64_t n, int shift, int dbits,
                                                                const int64_t *__restrict__ off, int64_t nb) {
    __shared__ uint32_t running[kMaxBins];
    __shared__ uint32_t wcnt[kWaves][kMaxBins];
    __shared__ int64_t goff[kMaxBins];
    const int tid = threadIdx.x, lane = lane_id(), w = tid / 64;
    const uint32_t mask = (1u << dbits) - 1u;
    const int bins = 1 << dbits;
    for (int d = tid; d < bins; d += kSortThreads) {
        running[d] = 0;
        goff[d] = off[(int64_t)d * nb + blockIdx.x];
#pragma unroll
        for (int k = 0; k < kWaves; ++k) wcnt[k][d] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + tid;
        const bool valid = i < n;
        uint32_t key = 0, val = 0, dig = 0;
        if (valid) {
            key = keys[i];
            val = vals[i];
            dig = (key >> shift) & mask;
        }
        // lanes of the wave with the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < dbits; ++b) {
            const uint64_t bal = __ballot(valid && ((dig >> b) & 1u));
            peers &= ((dig >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank_w = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank_w == 0) wcnt[w][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = running[dig];
            for (int k = 0; k < w; ++k) before += wcnt[k][dig];
            const int64_t pos = goff[dig] + (int64_t)(before + rank_w);
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        for (int d = tid; d < bins; d += kSortThreads) {
            uint32_t add = 0;
#pragma unroll
            for (int k = 0; k < kWaves; ++k) {
                add += wcnt[k][d];
                wcnt[k][d] = 0;
            }
            running[d] += add;
        }
        __syncthreads();
    }
}

}  // namespace

size_t radix_temp_bytes(int64_t n) {
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t m = (int64_t)kMaxBins * nb;
    size_t b = 0;
    b += (size_t)m * sizeof(uint32_t) + 256;              // histogram
    b += (size_t)(m + 1) * sizeof(int64_t) + 256;         // offsets
    b += 2 * ((size_t)n * sizeof(uint32_t) + 256);        // ping-pong keys/vals
    b += 2 * ((size_t)n * sizeof(uint32_t) + 256);
    b += scan_temp_bytes(m);
    return b;
}

static inline char *align_up(char *p, size_t a) {
    return reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(p) + a - 1) & ~(uintptr_t)(a - 1));
}

gsrad_status radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                              uint32_t *vals_out, int64_t n, int bits, void *temp, size_t temp_bytes,
                              hipStream_t st) {
    if (n <= 0) return GSRAD_OK;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    // passes of at most 9-bit digits, as few as the key bits need (17-bit
    // keys: two of 9 bits instead of three of 8), the digits of equal width
    const int passes = bits <= 0 ? 1 : (bits + kMaxDigitBits - 1) / kMaxDigitBits;
    const int dbits = bits <= 0 ? 1 : (bits + passes - 1) / passes;
    const int64_t m = ((int64_t)1 << dbits) * nb;
    char *p = static_cast<char *>(temp);
    char *end = p + temp_bytes;
    uint32_t *hist = reinterpret_cast<uint32_t *>(p);
    p = align_up(p + (size_t)m * sizeof(uint32_t), 256);
    int64_t *off = reinterpret_cast<int64_t *>(p);
    p = align_up(p + (size_t)(m + 1) * sizeof(int64_t), 256);
    uint32_t *ka = reinterpret_cast<uint32_t *>(p);
    p = align_up(p + (size_t)n * sizeof(uint32_t), 256);
    uint32_t *va = reinterpret_cast<uint32_t *>(p);
    p = align_up(p + (size_t)n * sizeof(uint32_t), 256);
    uint32_t *kb = reinterpret_cast<uint32_t *>(p);
    p = align_up(p + (size_t)n * sizeof(uint32_t), 256);
    uint32_t *vb = reinterpret_cast<uint32_t *>(p);
    p = align_up(p + (size_t)n * sizeof(uint32_t), 256);
    if (p > end) {
        set_error("radix sort: temp too small");
        return GSRAD_EINVAL;
    }
    const size_t scan_bytes = (size_t)(end - p);
    const uint32_t *ksrc = keys_in;
    const uint32_t *vsrc = vals_in;
    for (int pass = 0; pass < passes; ++pass) {
        const bool last = pass == passes - 1;
        uint32_t *kdst = last ? keys_out : ((pass & 1) ? kb : ka);
        uint32_t *vdst = last ? vals_out : ((pass & 1) ? vb : va);
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ksrc, n, dbits * pass, dbits,
                           hist, nb);
        gsrad_status s = exclusive_scan_u32_i64(hist, off, m, p, scan_bytes, st);
        if (s != GSRAD_OK) return s;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, st, ksrc, vsrc, kdst, vdst, n,
                           dbits * pass, dbits, off, nb);
        s = check_hip(hipGetLastError(), "radix scatter");
        if (s != GSRAD_OK) return s;
        ksrc = kdst;
        vsrc = vdst;
    }
    return GSRAD_OK;
}

}  // namespace gsrad
