// Internal declarations shared by the HIP translation units of libgsrad.
// Device-side definitions of the ray generator and the hit decision live
// here so that the form-factor, direct-light and backward kernels take
// exactly the same FP32 decisions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsrad.h"

namespace gsrad {

// ---------------------------------------------------------------------------
// constants of the method
// ---------------------------------------------------------------------------
constexpr float kOpacityMax = 0.9999f;   // o clamp: c = -ln(1-o) stays finite
constexpr float kSupportR2 = 9.0f;       // 3-sigma cut of the surfel support
constexpr float kGrazing = 1e-6f;        // |d . n| must exceed this
constexpr float kKernelExp = 1.7f;       // G^3.4 = exp(-1.7 (u^2+v^2)), App. E
constexpr int kRayMaxAttempts = 64;      // rejection-sampling bound
constexpr double kFixScale = 1099511627776.0;   // 2^40: fixed point of weights
constexpr float kFixScaleF = 1099511627776.0f;

// ---------------------------------------------------------------------------
// data layouts in HBM
// ---------------------------------------------------------------------------
// One surfel as the traversal reads it: 64 bytes, one cache line half.
//   a = (px, py, pz, 1/s_u)   b = (nx, ny, nz, 1/s_v)
//   c = (tux, tuy, tuz, c)    d = (tvx, tvy, tvz, original index as bits)
struct __align__(16) SurfRec {
    float4 a, b, c, d;
};

// Internal node of the binary BVH with both children's boxes inline (64 B).
//   b0 = (lo0.x, lo0.y, lo0.z, hi0.x)
//   b1 = (hi0.y, hi0.z, lo1.x, lo1.y)
//   b2 = (lo1.z, hi1.x, hi1.y, hi1.z)
//   ch = (child0, child1, parent, 0); child >= 0: internal node index,
//        child < 0: leaf ~sorted_position.
struct __align__(16) Node {
    float4 b0, b1, b2;
    int4 ch;
};

struct BvhDev {
    int64_t n;
    const SurfRec *rec;      // [n] in sorted (Morton) order
    const Node *nodes;       // [n-1]
    const int32_t *inv;      // [n] original index -> sorted position
    const float *c;          // [n] opacity constant c_j, original order
    const float *op;         // [n] clamped opacity, original order
    const float *raw_op;     // [n] opacity as given, original order
    const float *bounds;     // [8]: lo.xyz, hi.xyz, t_eps, diag
    const double *area;      // [n] App. E effective area, original order
    const float *dado;       // [n] d area / d opacity, original order
    float leaf_box_r;        // unused padding for alignment
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3, uint64_t k0,
                                              uint64_t k1, uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t h0 = __umul64hi(M0, x0), l0 = M0 * x0;
        const uint64_t h1 = __umul64hi(M1, x2), l1 = M1 * x2;
        const uint64_t y0 = h1 ^ x1 ^ k0, y2 = h0 ^ x3 ^ k1;
        x0 = y0;
        x1 = l1;
        x2 = y2;
        x3 = l0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

// Correctly rounded FP32 square root: the FP64 square root rounded to FP32
// (double rounding from 53 to 24 bits is harmless for sqrt, Figueroa 1995).
__device__ __forceinline__ float sqrt_rn(float x) { return (float)__builtin_sqrt((double)x); }

// Cosine-weighted hemisphere direction of ray r of receiver i: uniform
// points of the unit disc (rejection from the square) lifted to the
// hemisphere (Malley's method).  Every FP32 step is written out so the
// result is a fixed function of the inputs:
//   x = float(w >> 40) * 2^-23 - 1  (exact),  accept x*x + y*y < 1,
//   z = sqrt(1 - (x*x + y*y)) (correctly rounded),
//   d = fma(z, n, fma(y, t_v, x * t_u)).
__device__ __forceinline__ int ray_direction(float tux, float tuy, float tuz, float tvx, float tvy, float tvz,
                                             float nx, float ny, float nz, uint64_t ray, uint64_t recv,
                                             uint64_t seed, uint64_t tag, float &dx, float &dy, float &dz) {
    for (int a = 0; a < kRayMaxAttempts; ++a) {
        uint64_t w[4];
        philox4x64_10(ray, recv, (uint64_t)a, tag, seed, 0ULL, w);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float x = __fsub_rn(__fmul_rn((float)(uint32_t)(w[2 * p] >> 40), 0x1p-23f), 1.0f);
            const float y = __fsub_rn(__fmul_rn((float)(uint32_t)(w[2 * p + 1] >> 40), 0x1p-23f), 1.0f);
            const float xx = __fmul_rn(x, x);
            const float yy = __fmul_rn(y, y);
            const float s2 = __fadd_rn(xx, yy);
            if (s2 < 1.0f) {
                const float z = sqrt_rn(__fsub_rn(1.0f, s2));
                dx = __builtin_fmaf(z, nx, __builtin_fmaf(y, tvx, __fmul_rn(x, tux)));
                dy = __builtin_fmaf(z, ny, __builtin_fmaf(y, tvy, __fmul_rn(x, tuy)));
                dz = __builtin_fmaf(z, nz, __builtin_fmaf(y, tvz, __fmul_rn(x, tuz)));
                return a;
            }
        }
    }
    dx = nx;
    dy = ny;
    dz = nz;
    return kRayMaxAttempts;
}

// The disc sample (x, y) and z = sqrt(1 - x^2 - y^2) behind ray_direction's
// direction d = x t_u + y t_v + z n (same draws and roundings).
__device__ __forceinline__ void ray_sample(uint64_t ray, uint64_t recv, uint64_t seed, uint64_t tag, float &x_out,
                                           float &y_out, float &z_out) {
    for (int a = 0; a < kRayMaxAttempts; ++a) {
        uint64_t w[4];
        philox4x64_10(ray, recv, (uint64_t)a, tag, seed, 0ULL, w);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float x = __fsub_rn(__fmul_rn((float)(uint32_t)(w[2 * p] >> 40), 0x1p-23f), 1.0f);
            const float y = __fsub_rn(__fmul_rn((float)(uint32_t)(w[2 * p + 1] >> 40), 0x1p-23f), 1.0f);
            const float s2 = __fadd_rn(__fmul_rn(x, x), __fmul_rn(y, y));
            if (s2 < 1.0f) {
                x_out = x;
                y_out = y;
                z_out = sqrt_rn(__fsub_rn(1.0f, s2));
                return;
            }
        }
    }
    x_out = 0.0f;
    y_out = 0.0f;
    z_out = 1.0f;
}

// Hit decision (FP32, fixed order).  Returns true and (t, r2, front) when
// the ray o + t d crosses surfel `s` with t_lo < t (< t_hi if bounded) and
// u^2 + v^2 <= 9.
__device__ __forceinline__ bool hit_test(const SurfRec &s, float ox, float oy, float oz, float dx, float dy,
                                         float dz, float t_lo, float t_hi, bool bounded, float &t, float &r2,
                                         bool &front) {
    const float den = __builtin_fmaf(dz, s.b.z, __builtin_fmaf(dy, s.b.y, __fmul_rn(dx, s.b.x)));
    if (!(fabsf(den) > kGrazing)) return false;
    const float qx = __fsub_rn(s.a.x, ox), qy = __fsub_rn(s.a.y, oy), qz = __fsub_rn(s.a.z, oz);
    const float num = __builtin_fmaf(qz, s.b.z, __builtin_fmaf(qy, s.b.y, __fmul_rn(qx, s.b.x)));
    t = __fdiv_rn(num, den);
    if (!(t > t_lo)) return false;
    if (bounded && !(t < t_hi)) return false;
    const float hx = __builtin_fmaf(t, dx, -qx), hy = __builtin_fmaf(t, dy, -qy), hz = __builtin_fmaf(t, dz, -qz);
    const float u = __fmul_rn(__builtin_fmaf(hz, s.c.z, __builtin_fmaf(hy, s.c.y, __fmul_rn(hx, s.c.x))), s.a.w);
    const float v = __fmul_rn(__builtin_fmaf(hz, s.d.z, __builtin_fmaf(hy, s.d.y, __fmul_rn(hx, s.d.x))), s.b.w);
    r2 = __builtin_fmaf(v, v, __fmul_rn(u, u));
    if (!(r2 <= kSupportR2)) return false;
    front = den < 0.0f;
    return true;
}

// e^y for y <= 0 from correctly rounded FP32 steps only, so that the
// compositing cut (the first hit that leaves T < t_min) is one fixed
// function of the hit list: Cody-Waite reduction y = k ln2 + r with
// k = rint(y log2 e) and ln2 split into a 15-bit head (exact products)
// and an FP32 tail, the degree-7 Taylor polynomial of e^r (|r| <= ln2/2,
// truncation 3e-9) by Horner with fma, then an exact scaling by 2^k.
// Within 1 ulp of e^y on (-80, 0]; 0 at or below -80.
__device__ __forceinline__ float exp_fx(float y) {
    if (!(y > -80.0f)) return 0.0f;
    const float k = rintf(__fmul_rn(y, 1.44269504088896341f));
    float r = __builtin_fmaf(k, -0x1.62e4p-1f, y);
    r = __builtin_fmaf(k, -1.42860682030941723212e-6f, r);
    float p = 1.0f / 5040.0f;
    p = __builtin_fmaf(p, r, 1.0f / 720.0f);
    p = __builtin_fmaf(p, r, 1.0f / 120.0f);
    p = __builtin_fmaf(p, r, 1.0f / 24.0f);
    p = __builtin_fmaf(p, r, 1.0f / 6.0f);
    p = __builtin_fmaf(p, r, 0.5f);
    p = __builtin_fmaf(p, r, 1.0f);
    p = __builtin_fmaf(p, r, 1.0f);
    return __builtin_ldexpf(p, (int)k);
}

// u^2 + v^2 at a composited hit from the FP64 intersection of the FP32 ray
// with the surfel's plane, rounded once to FP32.  The FP32 hit decision
// loses the hit point's offset from the centre to cancellation when the
// centre is many radii away (h = t d - q with |q| >> |h|); the kernel
// value that weights the hit is taken from this exact evaluation instead.
// Fixed operation order, scales by the stored FP32 reciprocals 1/s:
//   den = d.n, q = p - o, t = (q.n)/den, h = t d - q,
//   u = (h.t_u)(1/s_u), v = (h.t_v)(1/s_v), r2 = u u + v v.
__device__ __forceinline__ float hit_r2_exact(const SurfRec &s, float ox, float oy, float oz, float dx, float dy,
                                              float dz) {
    const double nx = s.b.x, ny = s.b.y, nz = s.b.z;
    const double qx = (double)s.a.x - (double)ox, qy = (double)s.a.y - (double)oy, qz = (double)s.a.z - (double)oz;
    const double den = (double)dx * nx + (double)dy * ny + (double)dz * nz;
    const double t = (qx * nx + qy * ny + qz * nz) / den;
    const double hx = t * dx - qx, hy = t * dy - qy, hz = t * dz - qz;
    const double u = (hx * s.c.x + hy * s.c.y + hz * s.c.z) * (double)s.a.w;
    const double v = (hx * s.d.x + hy * s.d.y + hz * s.d.z) * (double)s.b.w;
    return (float)(u * u + v * v);
}

// Kernel value at a hit: gamma = e^(-1.7 r2), App. E (product rounded once).
__device__ __forceinline__ float kernel_gamma(float r2) { return exp_fx(-__fmul_rn(kKernelExp, r2)); }

// Transmittance factor of one composited hit with opacity constant c and
// kernel value g: e^(-c g), the product c g rounded once.
__device__ __forceinline__ float transmit(float c, float g) { return exp_fx(-__fmul_rn(c, g)); }

// Ray / box slab test with slack so that every hit point the FP32 surfel
// test can accept lies inside the tested interval.
__device__ __forceinline__ bool slab(float lox, float loy, float loz, float hix, float hiy, float hiz, float ox,
                                     float oy, float oz, float ix, float iy, float iz, float t0, float t1,
                                     float &tn) {
    // (lo - o) / d as fma(lo, 1/d, -o/d): one operation per plane (o/d is
    // loop-invariant); its rounding, a few 1e-8 of |o| in distance, is far
    // inside the boxes' inflation (4e-7 |p| + t_eps)
    const float ox_ = ox * ix, oy_ = oy * iy, oz_ = oz * iz;
    const float ax = __builtin_fmaf(lox, ix, -ox_), bx = __builtin_fmaf(hix, ix, -ox_);
    const float ay = __builtin_fmaf(loy, iy, -oy_), by = __builtin_fmaf(hiy, iy, -oy_);
    const float az = __builtin_fmaf(loz, iz, -oz_), bz = __builtin_fmaf(hiz, iz, -oz_);
    const float tmin = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t0));
    const float tmax = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), t1));
    tn = tmin;
    return tmin <= tmax * 1.00001f + 1e-30f;
}

__device__ __forceinline__ float safe_inv(float d) {
    return fabsf(d) > 1e-30f ? 1.0f / d : copysignf(1e30f, d);
}

// ---------------------------------------------------------------------------
// host-side helpers (defined in abi.cpp / kernels' translation units)
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
gsrad_status check_hip(hipError_t e, const char *what);

// scan_sort.hip
size_t scan_temp_bytes(int64_t n);
// exclusive prefix sum of n uint32 counts into int64 out[n+1] (out[n] = total)
gsrad_status exclusive_scan_u32_i64(const uint32_t *in, int64_t *out, int64_t n, void *temp, size_t temp_bytes,
                                    hipStream_t st);
size_t radix_temp_bytes(int64_t n);
// stable sort of (key, value) by the low `bits` of key; results in keys_out/vals_out
gsrad_status radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out,
                              uint32_t *vals_out, int64_t n, int bits, void *temp, size_t temp_bytes, hipStream_t st);

}  // namespace gsrad
