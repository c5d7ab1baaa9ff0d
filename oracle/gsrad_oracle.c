/*
 * gsrad_oracle.c -- plain, slow FP64 CPU oracle for surfel-to-surfel light
 * transport with alpha-composited visibility.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant generator with the GPU path; both sides
 * implement the same published definitions independently.
 *
 * What it computes (paper: "Differentiable Light Transport with Gaussian
 * Surfels via Adapted Radiosity"):
 *   - surfel opacity profile alpha(u,v) = 1 - exp(-c exp(-1.7 (u^2+v^2))),
 *     c = -ln(1-o): App. E opacity of the geometry field with the geometry
 *     value g folded into c = 0.03279 g^3.4, so that o = alpha(0,0);
 *     support cut at u^2+v^2 <= 9 (3 sigma);
 *   - cosine-weighted hemisphere rays from each receiver centre (App. B,
 *     the hemisphere integral of the rendering equation with the receiver
 *     weighting kernel a Dirac delta at p_i, Sec. 5.3 / Eq. before-final-
 *     radiosity), drawn with Philox4x64-10 (Salmon et al., SC'11);
 *   - per-ray depth-sorted alpha compositing (Eq. L_I): weight of the q-th
 *     hit w_q = alpha_q prod_{k<q}(1-alpha_k); back faces occlude but do not
 *     reflect (Sec. 5.1 "two-sided primitive with reflective front and
 *     non-reflective back faces"); self hits are disabled (Sec. 5.1);
 *   - form factors F_ij = (1/R) sum_rays sum_{hits on j, front} w  (Eq.
 *     final-radiosity with a Lambertian BRDF: the cosine-weighted estimator
 *     of the decay integral);
 *   - direct light from point lights (Eq. forward rendering equation, direct
 *     illumination; point lights as infinitesimal emitters, Sec. 5.1/5.3);
 *   - the compositing backward for opacity gradients through recorded hits
 *     (Eq. dl-dgeo-0, decay-term part, restricted to opacity).
 *
 * Hit decisions (which surfel a ray hits, and the depth order) and the
 * compositing cut (after which hit a ray stops) are integers decided by
 * floating point, so this oracle takes them in the FP32 operation sequence
 * the GPU kernel uses (definitions "D_hit" and "D_stop" below); all weights,
 * sums and gradients are then evaluated in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    const float *px, *py, *pz, *tux, *tuy, *tuz, *tvx, *tvy, *tvz, *nx, *ny, *nz, *su, *sv, *op;
    int64_t n;
} orc_scene;

#define ORC_PI 3.14159265358979323846
#define ORC_RAY_MAX_ATTEMPTS 64
#define ORC_OPACITY_MAX 0.9999f
#define ORC_SUPPORT_R2 9.0f
#define ORC_GRAZING 1e-6f

/* ------------------------------------------------------------------------
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): 10 rounds of two 64x64->128 multiplies with a
 * Weyl-sequence key schedule.
 * ---------------------------------------------------------------------- */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t h0, l0, h1, l1;
        mulhilo64(M0, x0, &h0, &l0);
        mulhilo64(M1, x2, &h1, &l1);
        uint64_t y0 = h1 ^ x1 ^ k0, y1 = l1, y2 = h0 ^ x3 ^ k1, y3 = l0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------
 * Ray generation, definition "D_ray".  Receiver i, ray r, stream tag:
 *   counter = (r, i, attempt, tag), key = (seed, 0);
 *   each Philox block gives two candidate points (w0,w1), (w2,w3) of the
 *   square, x = float(w >> 40) * 2^-23 - 1 (exact in FP32);
 *   accept the first with x*x + y*y < 1 (each product and the sum rounded);
 *   z = sqrt(1 - (x*x + y*y)) correctly rounded;
 *   d = fma(z, n, fma(y, t_v, x * t_u)) per component.
 * Uniform points of the unit disc lifted to the hemisphere are
 * cosine-distributed (Malley's method), so (1/R) sum_r g(d_r) estimates
 * (1/pi) * integral over the hemisphere of g(w) cos(theta) dw.
 * ---------------------------------------------------------------------- */
int orc_ray_direction(const orc_scene *s, int64_t i, uint64_t r, uint64_t seed, uint64_t tag, float d[3]) {
    const float tux = s->tux[i], tuy = s->tuy[i], tuz = s->tuz[i];
    const float tvx = s->tvx[i], tvy = s->tvy[i], tvz = s->tvz[i];
    const float nx = s->nx[i], ny = s->ny[i], nz = s->nz[i];
    for (uint64_t a = 0; a < ORC_RAY_MAX_ATTEMPTS; ++a) {
        uint64_t ctr[4] = {r, (uint64_t)i, a, tag}, key[2] = {seed, 0}, w[4];
        orc_philox4x64_10(ctr, key, w);
        for (int p = 0; p < 2; ++p) {
            float x = (float)(uint32_t)(w[2 * p] >> 40) * 0x1p-23f - 1.0f;
            float y = (float)(uint32_t)(w[2 * p + 1] >> 40) * 0x1p-23f - 1.0f;
            float xx = x * x;
            float yy = y * y;
            float s2 = xx + yy;
            if (s2 < 1.0f) {
                float z = sqrtf(1.0f - s2);
                d[0] = fmaf(z, nx, fmaf(y, tvx, x * tux));
                d[1] = fmaf(z, ny, fmaf(y, tvy, x * tuy));
                d[2] = fmaf(z, nz, fmaf(y, tvz, x * tuz));
                return (int)a;
            }
        }
    }
    d[0] = nx; d[1] = ny; d[2] = nz;
    return ORC_RAY_MAX_ATTEMPTS;
}

/* t_eps = 1e-5 * diagonal of the bounding box of the surfel centres, FP32:
 * e = max - min per axis, diag = sqrt(fma(ez,ez, fma(ey,ey, ex*ex))). */
float orc_default_t_eps(const orc_scene *s) {
    if (s->n <= 0) return 0.0f;
    float lo[3] = {s->px[0], s->py[0], s->pz[0]}, hi[3] = {s->px[0], s->py[0], s->pz[0]};
    for (int64_t j = 1; j < s->n; ++j) {
        float v[3] = {s->px[j], s->py[j], s->pz[j]};
        for (int k = 0; k < 3; ++k) {
            if (v[k] < lo[k]) lo[k] = v[k];
            if (v[k] > hi[k]) hi[k] = v[k];
        }
    }
    float ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    float diag = sqrtf(fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
    return 1e-5f * diag;
}

/* ------------------------------------------------------------------------
 * Hit decision, definition "D_hit" (FP32, fixed operation order):
 *   den = fma(dz,nz, fma(dy,ny, dx*nx));  reject unless |den| > 1e-6
 *   q   = p_j - o                          (componentwise)
 *   num = fma(qz,nz, fma(qy,ny, qx*nx))
 *   t   = num / den                        (correctly rounded)
 *   reject unless t > t_lo  (and t < t_hi for bounded rays)
 *   h   = fma(t, d, -q)                    (hit point minus centre)
 *   u   = fma(hz,tuz, fma(hy,tuy, hx*tux)) * (1/s_u)   (1/s_u rounded once)
 *   v   = same with t_v, s_v
 *   accept iff fma(v, v, u*u) <= 9
 * front face iff den < 0 (the ray arrives on the side the normal points to).
 * ---------------------------------------------------------------------- */
typedef struct {
    float t;
    int32_t j;
    int32_t front;
} orc_hit;

static int hit_test(const orc_scene *s, const float o[3], const float d[3], int64_t j, float t_lo, float t_hi,
                    int bounded, orc_hit *out) {
    const float nx = s->nx[j], ny = s->ny[j], nz = s->nz[j];
    float den = fmaf(d[2], nz, fmaf(d[1], ny, d[0] * nx));
    if (!(fabsf(den) > ORC_GRAZING)) return 0;
    float qx = s->px[j] - o[0], qy = s->py[j] - o[1], qz = s->pz[j] - o[2];
    float num = fmaf(qz, nz, fmaf(qy, ny, qx * nx));
    float t = num / den;
    if (!(t > t_lo)) return 0;
    if (bounded && !(t < t_hi)) return 0;
    float hx = fmaf(t, d[0], -qx), hy = fmaf(t, d[1], -qy), hz = fmaf(t, d[2], -qz);
    float isu = 1.0f / s->su[j], isv = 1.0f / s->sv[j];
    float u = fmaf(hz, s->tuz[j], fmaf(hy, s->tuy[j], hx * s->tux[j])) * isu;
    float v = fmaf(hz, s->tvz[j], fmaf(hy, s->tvy[j], hx * s->tvx[j])) * isv;
    float r2 = fmaf(v, v, u * u);
    if (!(r2 <= ORC_SUPPORT_R2)) return 0;
    out->t = t;
    out->j = (int32_t)j;
    out->front = den < 0.0f;
    return 1;
}

static int hit_cmp(const void *a, const void *b) {
    const orc_hit *x = (const orc_hit *)a, *y = (const orc_hit *)b;
    if (x->t < y->t) return -1;
    if (x->t > y->t) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

/* Clamped peak opacity (o <= 0.9999 keeps c = -ln(1-o) finite). */
static float clamp_opacity(float o) {
    if (!(o > 0.0f)) return 0.0f;
    return o < ORC_OPACITY_MAX ? o : ORC_OPACITY_MAX;
}

/* ------------------------------------------------------------------------
 * Compositing cut, definition "D_stop" (fixed operations).  The ray keeps
 * an FP32 transmittance T32 = 1 and, per hit in (t, j) order,
 *   c32   = -log1p(-o_j) evaluated in FP64, rounded to FP32 once
 *   r2s   = u^2 + v^2 of the FP64 intersection, rounded to FP32 once:
 *           den = d.n, q = p - o, t = (q.n)/den, h = t d - q,
 *           u = (h.t_u) * fl32(1/s_u), v = (h.t_v) * fl32(1/s_v)
 *           (FP64 operations in this order, sums left to right)
 *   g32   = exp_fx(-(1.7f * r2s))
 *   T32   = T32 * exp_fx(-(c32 * g32))    (each product rounded)
 * and stops after the first hit that leaves T32 < t_min.
 * exp_fx(y), y <= 0: e^y by Cody-Waite reduction y = k ln2 + r with
 *   k = rint(y * log2(e)),  r = fma(k, -ln2_hi, y),  r = fma(k, -ln2_lo, r),
 *   ln2_hi = 0x1.62e4p-1 (exact, 15 bits), ln2_lo = ln2 - ln2_hi in FP32,
 * the degree-7 Taylor polynomial of e^r by Horner with fma (coefficients
 * 1/n! rounded to FP32), and an exact scaling by 2^k; 0 for y <= -80.
 * Every step is a correctly rounded FP32 operation, so any implementation
 * of these steps returns the same bits (about 2 ulp from e^y).
 * ---------------------------------------------------------------------- */
float orc_exp_fx(float y) {
    if (!(y > -80.0f)) return 0.0f;
    float k = rintf(y * 1.44269504088896341f);
    float r = fmaf(k, -0x1.62e4p-1f, y);
    r = fmaf(k, -1.42860682030941723212e-6f, r);
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)k);
}

static float stop_factor(const orc_scene *s, const float o[3], const float d[3], const orc_hit *h) {
    const int64_t j = h->j;
    double nx = s->nx[j], ny = s->ny[j], nz = s->nz[j];
    double qx = (double)s->px[j] - (double)o[0], qy = (double)s->py[j] - (double)o[1],
           qz = (double)s->pz[j] - (double)o[2];
    double den = (double)d[0] * nx + (double)d[1] * ny + (double)d[2] * nz;
    double t = (qx * nx + qy * ny + qz * nz) / den;
    double hx = t * d[0] - qx, hy = t * d[1] - qy, hz = t * d[2] - qz;
    float isu = 1.0f / s->su[j], isv = 1.0f / s->sv[j];
    double u = (hx * s->tux[j] + hy * s->tuy[j] + hz * s->tuz[j]) * (double)isu;
    double v = (hx * s->tvx[j] + hy * s->tvy[j] + hz * s->tvz[j]) * (double)isv;
    float r2s = (float)(u * u + v * v);
    float c32 = (float)(-log1p(-(double)clamp_opacity(s->op[j])));
    float g32 = orc_exp_fx(-(1.7f * r2s));
    return orc_exp_fx(-(c32 * g32));
}

/* FP64 kernel value at the hit: gamma = exp(-1.7 (u^2+v^2)) from the exact
 * (FP64) intersection of the FP32 ray with surfel j's plane. */
static double hit_gamma64(const orc_scene *s, const float o[3], const float d[3], int64_t j) {
    double nx = s->nx[j], ny = s->ny[j], nz = s->nz[j];
    double qx = (double)s->px[j] - o[0], qy = (double)s->py[j] - o[1], qz = (double)s->pz[j] - o[2];
    double den = d[0] * nx + d[1] * ny + d[2] * nz;
    double t = (qx * nx + qy * ny + qz * nz) / den;
    double hx = t * d[0] - qx, hy = t * d[1] - qy, hz = t * d[2] - qz;
    double u = (hx * s->tux[j] + hy * s->tuy[j] + hz * s->tuz[j]) / (double)s->su[j];
    double v = (hx * s->tvx[j] + hy * s->tvy[j] + hz * s->tvz[j]) / (double)s->sv[j];
    return exp(-1.7 * (u * u + v * v));
}

/* All hits of one ray, sorted by (t, j).  Returns the count; grows *buf. */
static int64_t collect_hits(const orc_scene *s, const float o[3], const float d[3], int64_t skip, float t_lo,
                            float t_hi, int bounded, orc_hit **buf, int64_t *cap) {
    int64_t m = 0;
    for (int64_t j = 0; j < s->n; ++j) {
        if (j == skip) continue;
        orc_hit h;
        if (hit_test(s, o, d, j, t_lo, t_hi, bounded, &h)) {
            if (m == *cap) {
                *cap = *cap ? 2 * *cap : 64;
                *buf = (orc_hit *)realloc(*buf, (size_t)*cap * sizeof(orc_hit));
            }
            (*buf)[m++] = h;
        }
    }
    qsort(*buf, (size_t)m, sizeof(orc_hit), hit_cmp);
    return m;
}

/* One ray, fully described: every hit in depth order with its FP64 alpha,
 * transmittance in front of it and weight; n_comp = how many are composited
 * before the transmittance falls below t_min.  Returns the number of hits
 * (all of them, also those behind the cut) or -(needed) if cap is short. */
int64_t orc_trace_ray(const orc_scene *s, int64_t i, uint64_t r, uint64_t seed, float t_eps, float t_min,
                      int64_t cap, float *t_out, int32_t *j_out, int8_t *front_out, double *alpha_out,
                      double *T_out, float *T32_out, int64_t *n_comp, float d_out[3]) {
    float o[3] = {s->px[i], s->py[i], s->pz[i]}, d[3];
    orc_ray_direction(s, i, r, seed, 0, d);
    if (d_out) { d_out[0] = d[0]; d_out[1] = d[1]; d_out[2] = d[2]; }
    orc_hit *buf = NULL;
    int64_t bcap = 0;
    int64_t m = collect_hits(s, o, d, i, t_eps, 0.0f, 0, &buf, &bcap);
    if (m > cap) { free(buf); return -m; }
    double T = 1.0;
    float T32 = 1.0f;
    int64_t nc = m;
    int stopped = 0;
    for (int64_t q = 0; q < m; ++q) {
        int64_t j = buf[q].j;
        double c = -log1p(-(double)clamp_opacity(s->op[j]));
        double g = hit_gamma64(s, o, d, j);
        t_out[q] = buf[q].t;
        j_out[q] = buf[q].j;
        front_out[q] = (int8_t)buf[q].front;
        alpha_out[q] = -expm1(-c * g);
        T_out[q] = T;
        if (T32_out) T32_out[q] = T32;
        T *= exp(-c * g);
        T32 = T32 * stop_factor(s, o, d, &buf[q]);
        if (!stopped && T32 < t_min) { nc = q + 1; stopped = 1; }
    }
    *n_comp = nc;
    free(buf);
    return m;
}

/* ------------------------------------------------------------------------
 * Form-factor rows.  For each listed receiver i:
 *   F_ij = (1/R) sum_r sum_{composited front hits q on j} alpha_q T_q
 * with T_1 = 1, T_{q+1} = T_q (1 - alpha_q), compositing stops after the
 * first hit that leaves T < t_min.  With topk > 0 only the topk largest
 * entries (value descending, j ascending) are kept, without renormalising.
 * Output row k occupies cols/vals[k*cap_row .. k*cap_row + count[k]),
 * columns ascending.  diag[k*4 + {0,1,2,3}] = (sum of all front weights)/R
 * before truncation, (sum of back-face weights)/R, (1/R) sum_r (1 - T_r),
 * max hits composited on one ray.  Returns -1 if a row exceeds cap_row
 * (count then holds the size needed), else 0.
 * ---------------------------------------------------------------------- */
typedef struct {
    double v;
    int32_t j;
} orc_entry;

static int entry_desc(const void *a, const void *b) {
    const orc_entry *x = (const orc_entry *)a, *y = (const orc_entry *)b;
    if (x->v > y->v) return -1;
    if (x->v < y->v) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

static int entry_by_j(const void *a, const void *b) {
    const orc_entry *x = (const orc_entry *)a, *y = (const orc_entry *)b;
    return (x->j > y->j) - (x->j < y->j);
}

int orc_ff_rows(const orc_scene *s, const int64_t *recv, int64_t n_recv, int32_t R, uint64_t seed, float t_eps,
                float t_min, int32_t topk, int64_t cap_row, int32_t *cols, double *vals, int64_t *count, double *diag,
                int32_t n_threads) {
    int status = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
        double *acc = (double *)calloc((size_t)s->n, sizeof(double));
        int32_t *touched = (int32_t *)malloc((size_t)(s->n > 0 ? s->n : 1) * sizeof(int32_t));
        char *seen = (char *)calloc((size_t)s->n, 1);
        orc_hit *buf = NULL;
        int64_t bcap = 0;
        orc_entry *ent = (orc_entry *)malloc((size_t)(s->n > 0 ? s->n : 1) * sizeof(orc_entry));
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < n_recv; ++k) {
            int64_t i = recv[k];
            int64_t nt = 0;
            double back = 0.0, opaque = 0.0, maxh = 0.0;
            float o[3] = {s->px[i], s->py[i], s->pz[i]};
            for (int32_t r = 0; r < R; ++r) {
                float d[3];
                orc_ray_direction(s, i, (uint64_t)r, seed, 0, d);
                int64_t m = collect_hits(s, o, d, i, t_eps, 0.0f, 0, &buf, &bcap);
                double T = 1.0;
                float T32 = 1.0f;
                int64_t q = 0;
                for (; q < m; ++q) {
                    int64_t j = buf[q].j;
                    double c = -log1p(-(double)clamp_opacity(s->op[j]));
                    double g = hit_gamma64(s, o, d, j);
                    double a = -expm1(-c * g);
                    double w = a * T;
                    if (buf[q].front) {
                        if (!seen[j]) { seen[j] = 1; touched[nt++] = (int32_t)j; }
                        acc[j] += w;
                    } else {
                        back += w;
                    }
                    T *= exp(-c * g);
                    T32 = T32 * stop_factor(s, o, d, &buf[q]);
                    if (T32 < t_min) { ++q; break; }
                }
                if ((double)q > maxh) maxh = (double)q;
                opaque += 1.0 - T;
            }
            double front_sum = 0.0;
            for (int64_t e = 0; e < nt; ++e) {
                int32_t j = touched[e];
                ent[e].j = j;
                ent[e].v = acc[j] / (double)R;
                front_sum += ent[e].v;
                acc[j] = 0.0;
                seen[j] = 0;
            }
            int64_t keep = nt;
            if (topk > 0 && nt > topk) {
                qsort(ent, (size_t)nt, sizeof(orc_entry), entry_desc);
                keep = topk;
            }
            qsort(ent, (size_t)keep, sizeof(orc_entry), entry_by_j);
            count[k] = keep;
            if (diag) {
                diag[4 * k + 0] = front_sum;
                diag[4 * k + 1] = back / (double)R;
                diag[4 * k + 2] = opaque / (double)R;
                diag[4 * k + 3] = maxh;
            }
            if (keep > cap_row) {
#pragma omp atomic write
                status = -1;
                continue;
            }
            for (int64_t e = 0; e < keep; ++e) {
                cols[k * cap_row + e] = ent[e].j;
                vals[k * cap_row + e] = ent[e].v;
            }
        }
        free(acc);
        free(touched);
        free(seen);
        free(buf);
        free(ent);
    }
    return status;
}

/* ------------------------------------------------------------------------
 * Direct light (Eq. forward rendering equation, direct illumination, with
 * the receiver kernel a Dirac delta at p_i and the light an isotropic point
 * emitter of radiant intensity I):  only the DC coefficient is non-zero for
 * a Lambertian receiver (App. A: c_00 = 4 a for k = 1, so the DC output is
 * 4 a Y00 times the incident radiance), giving
 *   E_i,l,00,c = o_i a_i,c (2/sqrt(pi)) I_l max(0, n_i . w) / r^2 * T_il
 * with w the unit direction to the light, r its distance and T the product
 * of (1 - alpha) over every surfel the segment p_i -> x_l crosses (both
 * faces occlude; D_hit with d = x_l - p_i, t in (t_eps/|d|, 1)).
 * E_out is [n_recv][Lt][K][3]; coefficients with l >= 1 are 0.
 * ---------------------------------------------------------------------- */
void orc_direct_light(const orc_scene *s, const float *albedo, const float *lpos, const float *lI, int32_t Lt,
                      int32_t K, float t_eps, const int64_t *recv, int64_t n_recv, double *E_out, double *T_out,
                      int32_t n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
        orc_hit *buf = NULL;
        int64_t bcap = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < n_recv; ++k) {
            int64_t i = recv[k];
            float o[3] = {s->px[i], s->py[i], s->pz[i]};
            double oc = (double)clamp_opacity(s->op[i]);
            for (int32_t l = 0; l < Lt; ++l) {
                double *E = E_out + ((k * Lt + l) * K) * 3;
                for (int32_t c = 0; c < K * 3; ++c) E[c] = 0.0;
                float d[3] = {lpos[3 * l + 0] - o[0], lpos[3 * l + 1] - o[1], lpos[3 * l + 2] - o[2]};
                double r2 = (double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2];
                double cosv = ((double)s->nx[i] * d[0] + (double)s->ny[i] * d[1] + (double)s->nz[i] * d[2]) / sqrt(r2);
                if (T_out) T_out[k * Lt + l] = 0.0;
                if (!(cosv > 0.0) || !(r2 > 0.0)) continue;
                float len = sqrtf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])));
                float t_lo = t_eps / len;
                int64_t m = collect_hits(s, o, d, i, t_lo, 1.0f, 1, &buf, &bcap);
                double T = 1.0;
                for (int64_t q = 0; q < m; ++q) {
                    int64_t j = buf[q].j;
                    double c = -log1p(-(double)clamp_opacity(s->op[j]));
                    T *= exp(-c * hit_gamma64(s, o, d, j));
                }
                if (T_out) T_out[k * Lt + l] = T;
                double base = oc * (2.0 / sqrt(ORC_PI)) * (double)lI[l] * cosv / r2 * T;
                for (int c = 0; c < 3; ++c) E[c] = base * (double)albedo[3 * i + c];
            }
        }
        free(buf);
    }
}

/* ------------------------------------------------------------------------
 * Compositing backward (Eq. dl-dgeo-0 restricted to opacity; the decay
 * term is the only place o_j enters F).  For receiver i and each ray, with
 * composited hits q = 1..m, G_q = gF[i, j_q] / R on front hits (0 on back
 * hits and on entries dropped from the row):
 *   F-part of the loss on this ray:  sum_q G_q w_q,  w_q = alpha_q T_q
 *   dL/dalpha_q = G_q T_q - (sum_{p>q} G_p w_p) / (1 - alpha_q)
 *   dalpha/do   = gamma (1-o)^(gamma-1),  gamma = exp(-1.7 (u^2+v^2))
 *                 (0 where the opacity clamp is active)
 * accumulated into grad_o[j_q].  gF is given as CSR over the listed
 * receivers (row k of (gptr, gcol, gval) belongs to recv[k]).  The hit set
 * and the cut are those of the forward pass.
 * ---------------------------------------------------------------------- */
void orc_opacity_backward(const orc_scene *s, const int64_t *recv, int64_t n_recv, const int64_t *gptr,
                          const int32_t *gcol, const double *gval, int32_t R, uint64_t seed, float t_eps,
                          float t_min, double *grad_o, int32_t n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *part = (double *)calloc((size_t)nth * (size_t)s->n, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *go = part + (size_t)tid * (size_t)s->n;
        double *G = (double *)calloc((size_t)s->n, sizeof(double));
        orc_hit *buf = NULL;
        int64_t bcap = 0;
        double *a = NULL, *T = NULL, *gw = NULL, *gam = NULL;
        int64_t acap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < n_recv; ++k) {
            int64_t i = recv[k];
            for (int64_t e = gptr[k]; e < gptr[k + 1]; ++e) G[gcol[e]] = gval[e] / (double)R;
            float o[3] = {s->px[i], s->py[i], s->pz[i]};
            for (int32_t r = 0; r < R; ++r) {
                float d[3];
                orc_ray_direction(s, i, (uint64_t)r, seed, 0, d);
                int64_t m = collect_hits(s, o, d, i, t_eps, 0.0f, 0, &buf, &bcap);
                if (m > acap) {
                    acap = m;
                    a = (double *)realloc(a, (size_t)acap * sizeof(double));
                    T = (double *)realloc(T, (size_t)acap * sizeof(double));
                    gw = (double *)realloc(gw, (size_t)acap * sizeof(double));
                    gam = (double *)realloc(gam, (size_t)acap * sizeof(double));
                }
                double Tc = 1.0;
                float T32 = 1.0f;
                int64_t mc = 0;
                for (int64_t q = 0; q < m; ++q) {
                    int64_t j = buf[q].j;
                    double c = -log1p(-(double)clamp_opacity(s->op[j]));
                    gam[q] = hit_gamma64(s, o, d, j);
                    a[q] = -expm1(-c * gam[q]);
                    T[q] = Tc;
                    gw[q] = buf[q].front ? G[j] * a[q] * Tc : 0.0;
                    Tc *= exp(-c * gam[q]);
                    T32 = T32 * stop_factor(s, o, d, &buf[q]);
                    mc = q + 1;
                    if (T32 < t_min) break;
                }
                double suffix = 0.0;
                for (int64_t q = mc - 1; q >= 0; --q) {
                    int64_t j = buf[q].j;
                    double Gq = buf[q].front ? G[j] : 0.0;
                    double dLda = Gq * T[q] - suffix / (1.0 - a[q]);
                    float oj = s->op[j];
                    double dado = 0.0;
                    if (oj > 0.0f && oj < ORC_OPACITY_MAX) dado = gam[q] * pow(1.0 - (double)oj, gam[q] - 1.0);
                    go[j] += dLda * dado;
                    suffix += gw[q];
                }
            }
            for (int64_t e = gptr[k]; e < gptr[k + 1]; ++e) G[gcol[e]] = 0.0;
        }
        free(G);
        free(buf);
        free(a);
        free(T);
        free(gw);
        free(gam);
    }
    for (int t = 0; t < nth; ++t)
        for (int64_t j = 0; j < s->n; ++j) grad_o[j] += part[(size_t)t * (size_t)s->n + j];
    free(part);
}

/* ------------------------------------------------------------------------
 * Centre-to-centre form factors (Sec. 8, Eq. radiosity-approx-1, in the
 * scalar Lambertian form of the transport): for each listed pair (i, j)
 *   F_ij = lambda_j A_j T_ij |n_i . v| |n_j . v| / (pi |v|^4),  v = p_j - p_i
 * (|n.w| / r^2 with the unit direction w = v / |v|), A_j the App. E
 * effective area (given), and T_ij = prod (1 - alpha_k) over every surfel
 * k != i, j whose support the open segment p_i + t v crosses at
 * t in (eps, 1 - eps), eps = t_eps / |v| (D_hit decisions, both faces
 * occlude; alpha from the FP64 intersection).
 * ---------------------------------------------------------------------- */
typedef struct {
    double t, u, w, gam, c;
    double h[3];
} orc_seg_hit;

/* FP64 intersection of the segment o + t d (FP32 o, d) with surfel k. */
static void seg_hit64(const orc_scene *s, const float o[3], const float d[3], int64_t k, orc_seg_hit *r) {
    double n[3] = {s->nx[k], s->ny[k], s->nz[k]};
    double q[3] = {(double)s->px[k] - o[0], (double)s->py[k] - o[1], (double)s->pz[k] - o[2]};
    double den = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    double t = (q[0] * n[0] + q[1] * n[1] + q[2] * n[2]) / den;
    for (int a = 0; a < 3; ++a) r->h[a] = t * d[a] - q[a];
    r->t = t;
    r->u = (r->h[0] * s->tux[k] + r->h[1] * s->tuy[k] + r->h[2] * s->tuz[k]) / (double)s->su[k];
    r->w = (r->h[0] * s->tvx[k] + r->h[1] * s->tvy[k] + r->h[2] * s->tvz[k]) / (double)s->sv[k];
    r->gam = exp(-1.7 * (r->u * r->u + r->w * r->w));
    r->c = -log1p(-(double)clamp_opacity(s->op[k]));
}

/* the segment's occluders (surfels k != i, j) and its transmittance */
static double segment(const orc_scene *s, int64_t i, int64_t j, float t_eps, orc_hit **buf, int64_t *cap,
                      int64_t *m_out, float o[3], float d[3], double *len2) {
    o[0] = s->px[i]; o[1] = s->py[i]; o[2] = s->pz[i];
    d[0] = s->px[j] - o[0]; d[1] = s->py[j] - o[1]; d[2] = s->pz[j] - o[2];
    float len = sqrtf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])));
    *len2 = (double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2];
    float t_lo = t_eps / len, t_hi = 1.0f - t_lo;
    int64_t m = collect_hits(s, o, d, i, t_lo, t_hi, 1, buf, cap);
    int64_t w = 0;
    for (int64_t q = 0; q < m; ++q)
        if ((*buf)[q].j != j) (*buf)[w++] = (*buf)[q];
    *m_out = w;
    double T = 1.0;
    for (int64_t q = 0; q < w; ++q) {
        orc_seg_hit h;
        seg_hit64(s, o, d, (*buf)[q].j, &h);
        T *= exp(-h.c * h.gam);
    }
    return T;
}

void orc_center_ff(const orc_scene *s, const int64_t *rows, const int32_t *cols, int64_t m, const double *lambda,
                   const double *area, float t_eps, double *F_out, double *T_out, int32_t n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
        orc_hit *buf = NULL;
        int64_t bcap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t e = 0; e < m; ++e) {
            int64_t i = rows[e], j = cols[e], nh;
            float o[3], d[3];
            double len2;
            double T = segment(s, i, j, t_eps, &buf, &bcap, &nh, o, d, &len2);
            double a = s->nx[i] * (double)d[0] + s->ny[i] * (double)d[1] + s->nz[i] * (double)d[2];
            double b = s->nx[j] * (double)d[0] + s->ny[j] * (double)d[1] + s->nz[j] * (double)d[2];
            F_out[e] = lambda[j] * area[j] * T * fabs(a) * fabs(b) / (ORC_PI * len2 * len2);
            if (T_out) T_out[e] = T;
        }
        free(buf);
    }
}

/* ------------------------------------------------------------------------
 * Gradients of L through the centre-to-centre form factors, given
 * G_e = dL/dF_e for the listed pairs (the decay term of Eq. dl-dgeo-0 with
 * the decay of Sec. 8): with F = kappa T Phi, kappa = lambda_j A_j / pi,
 * Phi = |a| |b| / r^4, a = n_i . v, b = n_j . v, v = p_j - p_i,
 *   dPhi/dp_j = (sgn(a)|b| n_i + |a| sgn(b) n_j) / r^4 - 4 |a||b| v / r^6 = -dPhi/dp_i
 *   dPhi/dn_i = sgn(a) |b| v / r^4,  dPhi/dn_j = |a| sgn(b) v / r^4
 *   dF/dlambda_j = A_j T Phi / pi,  dF/dA_j = lambda_j T Phi / pi
 *   (A_j -> s_u, s_v, o_j through dA/ds_u = A/s_u, dA/do given);
 * the transmittance, log T = -sum_k c_k gamma_k over the occluders k, with
 * the segment crossing k's plane at t_k = (q . n_k)/(v . n_k), q = p_k - p_i,
 * h = t_k v - q, u = h . t_u / s_u, w = h . t_v / s_v, gamma = e^(-1.7 (u^2+w^2)):
 *   W = G F;  g_h = W 3.4 c gamma (u t_u / s_u + w t_v / s_v);  beta = (g_h . v)/(v . n_k)
 *   g_q = beta n_k - g_h:  p_k += g_q,  p_i -= (1 - t_k) g_q,  p_j -= t_k g_q
 *   n_k -= beta h;  t_u,k += W 3.4 c gamma u h / s_u;  t_v,k likewise with w
 *   s_u,k -= W 3.4 c gamma u^2 / s_u;  s_v,k likewise;  o_k -= W gamma / (1 - o_k)
 * (opacity terms only where the clamp is inactive).  grads is [n][15]:
 * px py pz tux tuy tuz tvx tvy tvz nx ny nz su sv o, plus g_lambda [n].
 * ---------------------------------------------------------------------- */
void orc_center_backward(const orc_scene *s, const int64_t *rows, const int32_t *cols, int64_t m,
                         const double *lambda, const double *area, const double *dA_do, float t_eps, const double *G,
                         double *g_lambda, double *grads, int32_t n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    const int64_t n = s->n;
    double *part = (double *)calloc((size_t)nth * (size_t)n * 16, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = part + (size_t)tid * (size_t)n * 16;   /* [n][16]: 15 fields, lambda */
        orc_hit *buf = NULL;
        int64_t bcap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t e = 0; e < m; ++e) {
            int64_t i = rows[e], j = cols[e], nh;
            float o[3], d[3];
            double len2;
            double T = segment(s, i, j, t_eps, &buf, &bcap, &nh, o, d, &len2);
            double v[3] = {d[0], d[1], d[2]};
            double ni[3] = {s->nx[i], s->ny[i], s->nz[i]}, nj[3] = {s->nx[j], s->ny[j], s->nz[j]};
            double a = ni[0] * v[0] + ni[1] * v[1] + ni[2] * v[2];
            double b = nj[0] * v[0] + nj[1] * v[1] + nj[2] * v[2];
            double r4 = len2 * len2, r6 = r4 * len2;
            double Phi = fabs(a) * fabs(b) / r4;
            double kappa = lambda[j] * area[j] / ORC_PI;
            double F = kappa * T * Phi;
            double Ge = G[e];
            double sa = a > 0 ? 1.0 : (a < 0 ? -1.0 : 0.0), sb = b > 0 ? 1.0 : (b < 0 ? -1.0 : 0.0);
            double kT = Ge * kappa * T;
            for (int c = 0; c < 3; ++c) {
                double dpj = (sa * fabs(b) * ni[c] + fabs(a) * sb * nj[c]) / r4 - 4.0 * fabs(a) * fabs(b) * v[c] / r6;
                acc[j * 16 + c] += kT * dpj;
                acc[i * 16 + c] -= kT * dpj;
                acc[i * 16 + 9 + c] += kT * sa * fabs(b) * v[c] / r4;
                acc[j * 16 + 9 + c] += kT * fabs(a) * sb * v[c] / r4;
            }
            acc[j * 16 + 15] += Ge * area[j] * T * Phi / ORC_PI;
            double gA = Ge * lambda[j] * T * Phi / ORC_PI;
            acc[j * 16 + 12] += gA * area[j] / s->su[j];
            acc[j * 16 + 13] += gA * area[j] / s->sv[j];
            acc[j * 16 + 14] += gA * dA_do[j];
            double W = Ge * F;
            for (int64_t q = 0; q < nh; ++q) {
                int64_t k = buf[q].j;
                orc_seg_hit h;
                seg_hit64(s, o, d, k, &h);
                double tu[3] = {s->tux[k], s->tuy[k], s->tuz[k]}, tv[3] = {s->tvx[k], s->tvy[k], s->tvz[k]};
                double nk[3] = {s->nx[k], s->ny[k], s->nz[k]};
                double su = s->su[k], sv = s->sv[k];
                double f = W * 3.4 * h.c * h.gam;
                double gh[3], gq[3];
                for (int c = 0; c < 3; ++c) gh[c] = f * (h.u * tu[c] / su + h.w * tv[c] / sv);
                double den = v[0] * nk[0] + v[1] * nk[1] + v[2] * nk[2];
                double beta = (gh[0] * v[0] + gh[1] * v[1] + gh[2] * v[2]) / den;
                for (int c = 0; c < 3; ++c) {
                    gq[c] = beta * nk[c] - gh[c];
                    acc[k * 16 + c] += gq[c];
                    acc[i * 16 + c] -= (1.0 - h.t) * gq[c];
                    acc[j * 16 + c] -= h.t * gq[c];
                    acc[k * 16 + 9 + c] -= beta * h.h[c];
                    acc[k * 16 + 3 + c] += f * h.u * h.h[c] / su;
                    acc[k * 16 + 6 + c] += f * h.w * h.h[c] / sv;
                }
                acc[k * 16 + 12] -= f * h.u * h.u / su;
                acc[k * 16 + 13] -= f * h.w * h.w / sv;
                float ok = s->op[k];
                if (ok > 0.0f && ok < ORC_OPACITY_MAX) acc[k * 16 + 14] -= W * h.gam / (1.0 - (double)ok);
            }
        }
        free(buf);
    }
    for (int t = 0; t < nth; ++t)
        for (int64_t k = 0; k < n; ++k) {
            const double *p = part + ((size_t)t * (size_t)n + (size_t)k) * 16;
            for (int f = 0; f < 15; ++f) grads[k * 15 + f] += p[f];
            g_lambda[k] += p[15];
        }
    free(part);
}

/* ------------------------------------------------------------------------
 * Geometry gradients through the ray-cast form factors (Eq. dl-dgeo-0, the
 * decay term with the recorded pairs, for every surfel field).  For
 * receiver i and ray r (origin p_i, direction d = x t_u,i + y t_v,i + z n_i
 * from the ray's disc sample) with composited hits q on surfels k_q, the
 * F-part of the loss is sum_q G_q alpha_q T_q (G_q = gF[i, k_q] / R on front
 * hits kept in F), so with the compositing backward's dL/dalpha_q:
 *   alpha = 1 - e^(-c gamma):  dL/dgamma = dL/dalpha c (1 - alpha),
 *   dL/dc = dL/dalpha gamma (1 - alpha) -> o_k: / (1 - o_k) inside the clamp
 *   gamma = e^(-1.7 (u^2 + w^2)), u = h . t_u / s_u, w = h . t_v / s_v,
 *   h = t d - q, q = p_k - p_i, t = (q . n_k)/(d . n_k):
 *   g_h = dL/dgamma (-3.4 gamma) (u t_u / s_u + w t_v / s_v),
 *   beta = (g_h . d)/(d . n_k), g_q = beta n_k - g_h:
 *     p_k += g_q, p_i -= g_q, n_k -= beta h,
 *     d += -t g_q  ->  t_u,i += x (-t g_q), t_v,i += y (-t g_q), n_i += z (-t g_q)
 *     t_u,k += dL/du h / s_u, s_u,k -= dL/du u / s_u (likewise v).
 * The hit set, its order and the cut are those of the forward pass.
 * grads [n][15]: px py pz tux tuy tuz tvx tvy tvz nx ny nz su sv o.
 * ---------------------------------------------------------------------- */
static void ray_sample(const orc_scene *s, int64_t i, uint64_t r, uint64_t seed, float xyz[3]) {
    for (uint64_t a = 0; a < ORC_RAY_MAX_ATTEMPTS; ++a) {
        uint64_t ctr[4] = {r, (uint64_t)i, a, 0}, key[2] = {seed, 0}, w[4];
        orc_philox4x64_10(ctr, key, w);
        for (int p = 0; p < 2; ++p) {
            float x = (float)(uint32_t)(w[2 * p] >> 40) * 0x1p-23f - 1.0f;
            float y = (float)(uint32_t)(w[2 * p + 1] >> 40) * 0x1p-23f - 1.0f;
            float s2 = x * x + y * y;
            if (s2 < 1.0f) {
                xyz[0] = x; xyz[1] = y; xyz[2] = sqrtf(1.0f - s2);
                return;
            }
        }
    }
    xyz[0] = 0.0f; xyz[1] = 0.0f; xyz[2] = 1.0f;
}

void orc_geometry_backward(const orc_scene *s, const int64_t *recv, int64_t n_recv, const int64_t *gptr,
                           const int32_t *gcol, const double *gval, int32_t R, uint64_t seed, float t_eps,
                           float t_min, double *grads, int32_t n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    const int64_t n = s->n;
    double *part = (double *)calloc((size_t)nth * (size_t)n * 15, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = part + (size_t)tid * (size_t)n * 15;
        double *G = (double *)calloc((size_t)n, sizeof(double));
        orc_hit *buf = NULL;
        int64_t bcap = 0;
        double *a = NULL, *T = NULL, *gw = NULL;
        int64_t acap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t kr = 0; kr < n_recv; ++kr) {
            int64_t i = recv[kr];
            for (int64_t e = gptr[kr]; e < gptr[kr + 1]; ++e) G[gcol[e]] = gval[e] / (double)R;
            float o[3] = {s->px[i], s->py[i], s->pz[i]};
            for (int32_t r = 0; r < R; ++r) {
                float d[3], xyz[3];
                orc_ray_direction(s, i, (uint64_t)r, seed, 0, d);
                ray_sample(s, i, (uint64_t)r, seed, xyz);
                int64_t m = collect_hits(s, o, d, i, t_eps, 0.0f, 0, &buf, &bcap);
                if (m > acap) {
                    acap = m;
                    a = (double *)realloc(a, (size_t)acap * sizeof(double));
                    T = (double *)realloc(T, (size_t)acap * sizeof(double));
                    gw = (double *)realloc(gw, (size_t)acap * sizeof(double));
                }
                double Tc = 1.0;
                float T32 = 1.0f;
                int64_t mc = 0;
                for (int64_t q = 0; q < m; ++q) {
                    int64_t k = buf[q].j;
                    orc_seg_hit h;
                    seg_hit64(s, o, d, k, &h);
                    a[q] = -expm1(-h.c * h.gam);
                    T[q] = Tc;
                    gw[q] = buf[q].front ? G[k] * a[q] * Tc : 0.0;
                    Tc *= exp(-h.c * h.gam);
                    T32 = T32 * stop_factor(s, o, d, &buf[q]);
                    mc = q + 1;
                    if (T32 < t_min) break;
                }
                double suffix = 0.0;
                for (int64_t q = mc - 1; q >= 0; --q) {
                    int64_t k = buf[q].j;
                    double Gq = buf[q].front ? G[k] : 0.0;
                    double dLda = Gq * T[q] - suffix / (1.0 - a[q]);
                    suffix += gw[q];
                    orc_seg_hit h;
                    seg_hit64(s, o, d, k, &h);
                    double dLdg = dLda * h.c * (1.0 - a[q]);
                    float ok = s->op[k];
                    if (ok > 0.0f && ok < ORC_OPACITY_MAX)
                        acc[k * 15 + 14] += dLda * h.gam * (1.0 - a[q]) / (1.0 - (double)ok);
                    double su = s->su[k], sv = s->sv[k];
                    double du = dLdg * (-3.4 * h.gam) * h.u, dw = dLdg * (-3.4 * h.gam) * h.w;
                    double tu[3] = {s->tux[k], s->tuy[k], s->tuz[k]}, tv[3] = {s->tvx[k], s->tvy[k], s->tvz[k]};
                    double nk[3] = {s->nx[k], s->ny[k], s->nz[k]};
                    double gh[3], gq[3];
                    for (int c = 0; c < 3; ++c) gh[c] = du * tu[c] / su + dw * tv[c] / sv;
                    double den = d[0] * nk[0] + d[1] * nk[1] + d[2] * nk[2];
                    double beta = (gh[0] * d[0] + gh[1] * d[1] + gh[2] * d[2]) / den;
                    for (int c = 0; c < 3; ++c) {
                        gq[c] = beta * nk[c] - gh[c];
                        acc[k * 15 + c] += gq[c];
                        acc[i * 15 + c] -= gq[c];
                        acc[k * 15 + 9 + c] -= beta * h.h[c];
                        acc[k * 15 + 3 + c] += du * h.h[c] / su;
                        acc[k * 15 + 6 + c] += dw * h.h[c] / sv;
                        double gd = -h.t * gq[c];
                        acc[i * 15 + 3 + c] += xyz[0] * gd;
                        acc[i * 15 + 6 + c] += xyz[1] * gd;
                        acc[i * 15 + 9 + c] += xyz[2] * gd;
                    }
                    acc[k * 15 + 12] -= du * h.u / su;
                    acc[k * 15 + 13] -= dw * h.w / sv;
                }
            }
            for (int64_t e = gptr[kr]; e < gptr[kr + 1]; ++e) G[gcol[e]] = 0.0;
        }
        free(G);
        free(buf);
        free(a);
        free(T);
        free(gw);
    }
    for (int t = 0; t < nth; ++t)
        for (size_t k = 0; k < (size_t)n * 15; ++k) grads[k] += part[(size_t)t * (size_t)n * 15 + k];
    free(part);
}

/* ------------------------------------------------------------------------
 * Gradients of the direct light (Eq. forward rendering equation, direct
 * illumination) with respect to the lights' positions and intensities, the
 * albedo, and the surfel fields of the receivers and of the occluders on the
 * shadow segments (Sec. 9's light-position optimisation): with v = x_l - p_i,
 * r = |v|, ndot = n_i . v > 0,
 *   E_i,l,00,c = o_i a_i,c kappa I_l ndot T_il / r^3,  kappa = 2/sqrt(pi),
 *   S = sum_c dL/dE_i,l,00,c a_i,c,  Q = S o_i kappa I_l T_il:
 *   dL/dI_l += S o_i kappa ndot T / r^3,  dL/da_i,c += dL/dE_c o_i kappa I ndot T / r^3,
 *   dL/do_i += S kappa I ndot T / r^3 (inside the clamp),
 *   g_v = Q (n_i / r^3 - 3 ndot v / r^5):  x_l += g_v,  p_i -= g_v,  n_i += Q v / r^3,
 * and the transmittance as for a centre-to-centre segment with W = S o kappa I ndot T / r^3
 * (the light in the role of the far end).  grads [n][15] as in
 * orc_geometry_backward, g_lpos [Lt][3], g_lI [Lt], g_alb [n][3].
 * ---------------------------------------------------------------------- */
void orc_direct_light_backward(const orc_scene *s, const float *albedo, const float *lpos, const float *lI,
                               int32_t Lt, int32_t K, float t_eps, const double *gE, double *g_lpos, double *g_lI,
                               double *g_alb, double *grads, int32_t n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    const int64_t n = s->n;
    const size_t per = (size_t)n * 15 + (size_t)Lt * 4;
    double *part = (double *)calloc((size_t)nth * per, sizeof(double));
    const double kappa = 2.0 / sqrt(ORC_PI);
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = part + (size_t)tid * per;
        double *accl = acc + (size_t)n * 15;
        orc_hit *buf = NULL;
        int64_t bcap = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            float o[3] = {s->px[i], s->py[i], s->pz[i]};
            double oc = (double)clamp_opacity(s->op[i]);
            float oraw = s->op[i];
            for (int32_t l = 0; l < Lt; ++l) {
                float d[3] = {lpos[3 * l + 0] - o[0], lpos[3 * l + 1] - o[1], lpos[3 * l + 2] - o[2]};
                double v[3] = {d[0], d[1], d[2]};
                double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                double ni[3] = {s->nx[i], s->ny[i], s->nz[i]};
                double ndot = ni[0] * v[0] + ni[1] * v[1] + ni[2] * v[2];
                if (!(ndot > 0.0) || !(r2 > 0.0)) continue;
                double r = sqrt(r2), r3 = r2 * r, r5 = r3 * r2;
                float len = sqrtf(fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0])));
                float t_lo = t_eps / len;
                int64_t m = collect_hits(s, o, d, i, t_lo, 1.0f, 1, &buf, &bcap);
                double T = 1.0;
                for (int64_t q = 0; q < m; ++q) {
                    orc_seg_hit h;
                    seg_hit64(s, o, d, buf[q].j, &h);
                    T *= exp(-h.c * h.gam);
                }
                const double *ge = gE + (((size_t)i * Lt + l) * K) * 3;
                double S = 0.0;
                for (int c = 0; c < 3; ++c) S += ge[c] * (double)albedo[3 * i + c];
                double base = kappa * (double)lI[l] * ndot * T / r3;
                accl[(size_t)Lt * 3 + l] += S * oc * kappa * ndot * T / r3;
                for (int c = 0; c < 3; ++c) g_alb[3 * i + c] += ge[c] * oc * base;   /* row i is this thread's */
                if (oraw > 0.0f && oraw < ORC_OPACITY_MAX) acc[i * 15 + 14] += S * base;
                double Q = S * oc * kappa * (double)lI[l] * T;
                for (int c = 0; c < 3; ++c) {
                    double gv = Q * (ni[c] / r3 - 3.0 * ndot * v[c] / r5);
                    accl[3 * l + c] += gv;
                    acc[i * 15 + c] -= gv;
                    acc[i * 15 + 9 + c] += Q * v[c] / r3;
                }
                double W = S * oc * base;
                for (int64_t q = 0; q < m; ++q) {
                    int64_t k = buf[q].j;
                    orc_seg_hit h;
                    seg_hit64(s, o, d, k, &h);
                    double tu[3] = {s->tux[k], s->tuy[k], s->tuz[k]}, tv[3] = {s->tvx[k], s->tvy[k], s->tvz[k]};
                    double nk[3] = {s->nx[k], s->ny[k], s->nz[k]};
                    double su = s->su[k], sv = s->sv[k];
                    double f = W * 3.4 * h.c * h.gam;
                    double gh[3], gq[3];
                    for (int c = 0; c < 3; ++c) gh[c] = f * (h.u * tu[c] / su + h.w * tv[c] / sv);
                    double den = v[0] * nk[0] + v[1] * nk[1] + v[2] * nk[2];
                    double beta = (gh[0] * v[0] + gh[1] * v[1] + gh[2] * v[2]) / den;
                    for (int c = 0; c < 3; ++c) {
                        gq[c] = beta * nk[c] - gh[c];
                        acc[k * 15 + c] += gq[c];
                        acc[i * 15 + c] -= (1.0 - h.t) * gq[c];
                        accl[3 * l + c] -= h.t * gq[c];
                        acc[k * 15 + 9 + c] -= beta * h.h[c];
                        acc[k * 15 + 3 + c] += f * h.u * h.h[c] / su;
                        acc[k * 15 + 6 + c] += f * h.w * h.h[c] / sv;
                    }
                    acc[k * 15 + 12] -= f * h.u * h.u / su;
                    acc[k * 15 + 13] -= f * h.w * h.w / sv;
                    float ok = s->op[k];
                    if (ok > 0.0f && ok < ORC_OPACITY_MAX) acc[k * 15 + 14] -= W * h.gam / (1.0 - (double)ok);
                }
            }
        }
        free(buf);
    }
    for (int t = 0; t < nth; ++t) {
        const double *p = part + (size_t)t * per;
        for (size_t k = 0; k < (size_t)n * 15; ++k) grads[k] += p[k];
        for (int32_t l = 0; l < Lt; ++l) {
            for (int c = 0; c < 3; ++c) g_lpos[3 * l + c] += p[(size_t)n * 15 + 3 * l + c];
            g_lI[l] += p[(size_t)n * 15 + (size_t)Lt * 3 + l];
        }
    }
    free(part);
}
