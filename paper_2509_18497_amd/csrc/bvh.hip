// Surfel preparation and linear BVH construction.
//
// 1. bounds of the centres (exact FP32 min/max) -> default t_eps
// 2. 30-bit Morton codes of the centres, stable radix sort (index ties)
// 3. Karras (HPG 2012) binary radix tree over the sorted codes
// 4. bottom-up refit of 3-sigma ellipse bounds (atomic arrival counters)
// 5. packing: each internal node stores both children's boxes (64 B)
#include "gsrad_internal.h"
#include "bvh_build.h"

namespace gsrad {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float clamp_op(float o) {
    if (!(o > 0.0f)) return 0.0f;
    return o < kOpacityMax ? o : kOpacityMax;
}

__global__ void __launch_bounds__(kThreads) k_bounds_partial(const float *__restrict__ px, const float *__restrict__ py,
                                                             const float *__restrict__ pz, int64_t n,
                                                             float *__restrict__ part) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const float v[3] = {px[i], py[i], pz[i]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], v[k]);
            hi[k] = fmaxf(hi[k], v[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        for (int o = 32; o >= 1; o >>= 1) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], o, 64));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o, 64));
        }
    }
    __shared__ float s[kThreads / 64][6];
    const int w = threadIdx.x / 64;
    if (__lane_id() == 0) {
        for (int k = 0; k < 3; ++k) {
            s[w][k] = lo[k];
            s[w][3 + k] = hi[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        float v = s[0][threadIdx.x];
        for (int q = 1; q < kThreads / 64; ++q) v = threadIdx.x < 3 ? fminf(v, s[q][threadIdx.x]) : fmaxf(v, s[q][threadIdx.x]);
        part[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

// bounds[0..2] = lo, [3..5] = hi, [6] = t_eps = 1e-5 * diag, [7] = diag
__global__ void k_bounds_final(const float *__restrict__ part, int nparts, float *__restrict__ bounds) {
    if (threadIdx.x != 0) return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int p = 0; p < nparts; ++p)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], part[p * 6 + k]);
            hi[k] = fmaxf(hi[k], part[p * 6 + 3 + k]);
        }
    const float ex = __fsub_rn(hi[0], lo[0]), ey = __fsub_rn(hi[1], lo[1]), ez = __fsub_rn(hi[2], lo[2]);
    const float diag = sqrt_rn(__builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, __fmul_rn(ex, ex))));
    for (int k = 0; k < 3; ++k) {
        bounds[k] = lo[k];
        bounds[3 + k] = hi[k];
    }
    bounds[6] = __fmul_rn(1e-5f, diag);
    bounds[7] = diag;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t quant10(float x, float lo, float hi) {
    const float ext = hi - lo;
    if (!(ext > 0.0f)) return 0u;
    float q = (x - lo) / ext * 1024.0f;
    q = fminf(fmaxf(q, 0.0f), 1023.0f);
    return (uint32_t)q;
}

__global__ void __launch_bounds__(kThreads) k_morton(const float *__restrict__ px, const float *__restrict__ py,
                                                     const float *__restrict__ pz, int64_t n,
                                                     const float *__restrict__ bounds, uint32_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = quant10(px[i], bounds[0], bounds[3]);
    const uint32_t y = quant10(py[i], bounds[1], bounds[4]);
    const uint32_t z = quant10(pz[i], bounds[2], bounds[5]);
    keys[i] = (spread10(x) << 2) | (spread10(y) << 1) | spread10(z);
    vals[i] = (uint32_t)i;
}

// Per sorted position s (original index j = order[s]): the traversal
// record, the outward-rounded 3-sigma ellipse bounds, the inverse
// permutation, and the per-surfel constants in original order.
__global__ void __launch_bounds__(kThreads) k_records(gsrad_surfels sf, const uint32_t *__restrict__ order,
                                                      const float *__restrict__ bounds, SurfRec *__restrict__ rec,
                                                      float *__restrict__ leafbox, int32_t *__restrict__ inv,
                                                      float *__restrict__ cst, float *__restrict__ opc,
                                                      float *__restrict__ opraw, double *__restrict__ area,
                                                      float *__restrict__ dado) {
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= sf.n) return;
    const int64_t j = order[s];
    const float px = sf.px[j], py = sf.py[j], pz = sf.pz[j];
    const float tux = sf.tux[j], tuy = sf.tuy[j], tuz = sf.tuz[j];
    const float tvx = sf.tvx[j], tvy = sf.tvy[j], tvz = sf.tvz[j];
    const float nx = sf.nx[j], ny = sf.ny[j], nz = sf.nz[j];
    const float su = sf.su[j], sv = sf.sv[j];
    const float oraw = sf.opacity[j];
    const float o = clamp_op(oraw);
    // c = -ln(1 - o), evaluated in FP64 and rounded once to FP32
    const float c = (float)(-log1p(-(double)o));
    SurfRec r;
    r.a = make_float4(px, py, pz, __fdiv_rn(1.0f, su));
    r.b = make_float4(nx, ny, nz, __fdiv_rn(1.0f, sv));
    r.c = make_float4(tux, tuy, tuz, c);
    r.d = make_float4(tvx, tvy, tvz, __uint_as_float((uint32_t)j));
    rec[s] = r;
    inv[j] = (int32_t)s;
    cst[j] = c;
    opc[j] = o;
    opraw[j] = oraw;
    // 3-sigma ellipse half extents, inflated so the FP32 hit decision can
    // never accept a point outside the box
    const float teps = bounds[6];
    const float p[3] = {px, py, pz};
    const float tu[3] = {tux, tuy, tuz}, tv[3] = {tvx, tvy, tvz};
    for (int k = 0; k < 3; ++k) {
        const float a = su * tu[k], b = sv * tv[k];
        const float h = 3.0f * sqrtf(a * a + b * b) * 1.0002f + teps + 4e-7f * fabsf(p[k]);
        leafbox[s * 6 + k] = p[k] - h;
        leafbox[s * 6 + 3 + k] = p[k] + h;
    }
    // App. E effective area in FP64: (2 pi / 3.4) s_u s_v Ein(c),
    // Ein(c) = sum_{k>=1} (-1)^(k+1) c^k / (k k!)
    const double cd = -log1p(-(double)o);
    double term = cd, sum = 0.0;
    for (int k = 1; k < 80; ++k) {
        const double add = term / (double)k;
        sum += add;
        term *= -cd / (double)(k + 1);
        if (fabs(add) < 1e-18 * fabs(sum)) break;
    }
    const double a0 = (2.0 * 3.14159265358979323846 / 3.4) * (double)su * (double)sv;
    area[j] = a0 * sum;
    // dA/do = a0 dEin/dc dc/do = a0 (1 - e^-c)/c / (1 - o), inside the clamp
    const bool inside = oraw > 0.0f && oraw < kOpacityMax;
    dado[j] = inside ? (float)(a0 * (cd > 1e-12 ? -expm1(-cd) / cd : 1.0) / (1.0 - (double)o)) : 0.0f;
}

__device__ __forceinline__ int delta(const uint32_t *__restrict__ keys, int64_t n, int64_t a, int64_t b) {
    if (b < 0 || b >= n) return -1;
    const uint32_t ka = keys[a], kb = keys[b];
    if (ka == kb) return 32 + __clz((uint32_t)(a ^ b));
    return __clz(ka ^ kb);
}

// Binary radix tree (Karras 2012): internal node i covers a key range
// [min(i,j), max(i,j)] split at gamma.
__global__ void __launch_bounds__(kThreads) k_karras(const uint32_t *__restrict__ keys, int64_t n,
                                                     Node *__restrict__ nodes, int32_t *__restrict__ leaf_parent) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(keys, n, i, i - d);
    int64_t lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = delta(keys, n, i, j);
    int64_t s = 0;
    int64_t step = l;
    do {
        step = (step + 1) >> 1;
        if (s + step < l && delta(keys, n, i, i + (s + step) * d) > dnode) s += step;
    } while (step > 1);
    const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int c0, c1;
    if (lo == gamma) {
        c0 = ~(int)gamma;
        leaf_parent[gamma] = (int32_t)i;
    } else {
        c0 = (int)gamma;
        nodes[gamma].ch.z = (int)i;
    }
    if (hi == gamma + 1) {
        c1 = ~(int)(gamma + 1);
        leaf_parent[gamma + 1] = (int32_t)i;
    } else {
        c1 = (int)(gamma + 1);
        nodes[gamma + 1].ch.z = (int)i;
    }
    nodes[i].ch.x = c0;
    nodes[i].ch.y = c1;
    nodes[i].ch.w = 0;
    if (i == 0) nodes[0].ch.z = -1;
}

__device__ __forceinline__ float ld_coherent(const float *p) {
    return __uint_as_float(__hip_atomic_load(reinterpret_cast<const uint32_t *>(p), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ int ld_coherent_i(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(float *p, float v) {
    __hip_atomic_store(reinterpret_cast<uint32_t *>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent_i(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bottom-up: the second child to arrive at a node computes its box (and
// subtree height) and walks on; box unions are exact, so the result does
// not depend on arrival order.
__global__ void __launch_bounds__(kThreads) k_refit(const Node *__restrict__ nodes,
                                                    const int32_t *__restrict__ leaf_parent,
                                                    const float *__restrict__ leafbox, float *nodebox,
                                                    int *nodeheight, int *counter, int *height_out, int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s >= n) return;
    int node = leaf_parent[s];
    while (node >= 0) {
        __threadfence();
        const int old = atomicAdd(&counter[node], 1);
        if (old == 0) return;
        __threadfence();
        const int c[2] = {nodes[node].ch.x, nodes[node].ch.y};
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int h = 0;
        for (int q = 0; q < 2; ++q) {
            const float *b = c[q] < 0 ? leafbox + (int64_t)(~c[q]) * 6 : nodebox + (int64_t)c[q] * 6;
            const int hc = c[q] < 0 ? 0 : ld_coherent_i(nodeheight + c[q]);
            h = max(h, hc + 1);
            for (int k = 0; k < 3; ++k) {
                lo[k] = fminf(lo[k], c[q] < 0 ? b[k] : ld_coherent(b + k));
                hi[k] = fmaxf(hi[k], c[q] < 0 ? b[3 + k] : ld_coherent(b + 3 + k));
            }
        }
        for (int k = 0; k < 3; ++k) {
            st_coherent(nodebox + (int64_t)node * 6 + k, lo[k]);
            st_coherent(nodebox + (int64_t)node * 6 + 3 + k, hi[k]);
        }
        st_coherent_i(nodeheight + node, h);
        if (node == 0) {
            *height_out = h;
            return;
        }
        node = nodes[node].ch.z;
    }
}

__global__ void __launch_bounds__(kThreads) k_pack(Node *__restrict__ nodes, const float *__restrict__ leafbox,
                                                   const float *__restrict__ nodebox, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n - 1) return;
    const int c0 = nodes[i].ch.x, c1 = nodes[i].ch.y;
    const float *b0 = c0 < 0 ? leafbox + (int64_t)(~c0) * 6 : nodebox + (int64_t)c0 * 6;
    const float *b1 = c1 < 0 ? leafbox + (int64_t)(~c1) * 6 : nodebox + (int64_t)c1 * 6;
    nodes[i].b0 = make_float4(b0[0], b0[1], b0[2], b0[3]);
    nodes[i].b1 = make_float4(b0[4], b0[5], b1[0], b1[1]);
    nodes[i].b2 = make_float4(b1[2], b1[3], b1[4], b1[5]);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

__global__ void __launch_bounds__(kThreads) k_sorted_order(const SurfRec *__restrict__ rec, int64_t n,
                                                          int32_t *__restrict__ order) {
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (s < n) order[s] = (int32_t)__float_as_uint(rec[s].d.w);
}

}  // namespace

size_t bvh_temp_bytes(int64_t n) {
    size_t b = 0;
    b += 4 * ((size_t)n * 4 + 256);                   // keys/vals in and out
    b += radix_temp_bytes(n) + 256;
    b += (size_t)n * 6 * sizeof(float) + 256;         // node boxes
    b += (size_t)n * sizeof(int) * 2 + 512;           // heights, counters
    b += 1024 * 6 * sizeof(float) + 256;              // bounds partials
    return b;
}

static inline char *carve(char *&p, size_t bytes) {
    char *r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
}

gsrad_status bvh_build(const gsrad_surfels &sf, BvhBuffers &B, hipStream_t st) {
    const int64_t n = sf.n;
    char *p = static_cast<char *>(B.temp);
    uint32_t *k_in = reinterpret_cast<uint32_t *>(carve(p, (size_t)n * 4));
    uint32_t *v_in = reinterpret_cast<uint32_t *>(carve(p, (size_t)n * 4));
    uint32_t *k_out = reinterpret_cast<uint32_t *>(carve(p, (size_t)n * 4));
    uint32_t *v_out = reinterpret_cast<uint32_t *>(carve(p, (size_t)n * 4));
    const size_t rbytes = radix_temp_bytes(n);
    void *rtemp = carve(p, rbytes);
    float *nodebox = reinterpret_cast<float *>(carve(p, (size_t)n * 6 * sizeof(float)));
    int *height = reinterpret_cast<int *>(carve(p, (size_t)n * sizeof(int)));
    int *counter = reinterpret_cast<int *>(carve(p, (size_t)n * sizeof(int)));
    float *part = reinterpret_cast<float *>(carve(p, 1024 * 6 * sizeof(float)));
    if ((size_t)(p - static_cast<char *>(B.temp)) > B.temp_bytes) {
        set_error("bvh: temp too small");
        return GSRAD_EINVAL;
    }
    const int nparts = (int)std::min<int64_t>(1024, (n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_bounds_partial, dim3(nparts), dim3(kThreads), 0, st, sf.px, sf.py, sf.pz, n, part);
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(64), 0, st, part, nparts, B.bounds);
    hipLaunchKernelGGL(k_morton, dim3(nblk(n)), dim3(kThreads), 0, st, sf.px, sf.py, sf.pz, n, B.bounds, k_in, v_in);
    gsrad_status s = check_hip(hipGetLastError(), "bvh morton");
    if (s != GSRAD_OK) return s;
    s = radix_sort_pairs(k_in, v_in, k_out, v_out, n, 30, rtemp, rbytes, st);
    if (s != GSRAD_OK) return s;
    hipLaunchKernelGGL(k_records, dim3(nblk(n)), dim3(kThreads), 0, st, sf, v_out, B.bounds, B.rec, B.leafbox, B.inv,
                       B.cst, B.opc, B.opraw, B.area, B.dado);
    if (n >= 2) {
        hipLaunchKernelGGL(k_karras, dim3(nblk(n - 1)), dim3(kThreads), 0, st, k_out, n, B.nodes, B.leaf_parent);
        s = check_hip(hipMemsetAsync(counter, 0, (size_t)n * sizeof(int), st), "bvh memset");
        if (s != GSRAD_OK) return s;
        hipLaunchKernelGGL(k_refit, dim3(nblk(n)), dim3(kThreads), 0, st, B.nodes, B.leaf_parent, B.leafbox, nodebox,
                           height, counter, B.height, n);
        hipLaunchKernelGGL(k_pack, dim3(nblk(n - 1)), dim3(kThreads), 0, st, B.nodes, B.leafbox, nodebox, n);
    }
    return check_hip(hipGetLastError(), "bvh build");
}

gsrad_status launch_sorted_order(const BvhDev &bv, int32_t *order, hipStream_t st) {
    if (bv.n == 0) return GSRAD_OK;
    hipLaunchKernelGGL(k_sorted_order, dim3(nblk(bv.n)), dim3(kThreads), 0, st, bv.rec, bv.n, order);
    return check_hip(hipGetLastError(), "sorted order launch");
}

}  // namespace gsrad
