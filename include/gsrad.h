/*
 * gsrad.h -- C ABI of libgsrad: surfel-to-surfel light transport with
 * alpha-composited visibility, its bounce iterations and their adjoint, on
 * one AMD Instinct MI355X (gfx950).
 *
 * Paper: "Differentiable Light Transport with Gaussian Surfels via Adapted
 * Radiosity for Efficient Relighting and Geometry Reconstruction" (Jiang et
 * al., ACM TOG 2025, DOI 10.1145/3763305).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are DEVICE pointers unless stated otherwise, FP32,
 *   C-contiguous, owned by the caller.  The library never frees them.
 * - Opaque handles (gsrad_bvh, gsrad_ff, gsrad_tape) are owned by the
 *   library and freed by the matching *_destroy.  Passing a pointer to a
 *   NULL handle creates one; passing an existing handle re-uses (and if
 *   needed grows) its device memory, so a steady-state loop allocates
 *   nothing.
 * - `stream` is a hipStream_t (NULL = the default stream).  Work is queued
 *   on it; arguments are validated synchronously before anything is queued.
 *   gsrad_form_factors additionally waits for its own kernels once (it reads
 *   the number of non-zeros and the overflow flags back to the host).
 * - Errors: every call returns GSRAD_OK (0) or a negative code; the message
 *   of the last error of the calling thread is gsrad_last_error().  No
 *   exception crosses the ABI.  A failed call leaves the handles it only
 *   reads as they were; a handle that a failed call was rebuilding or
 *   refilling in place is left unusable, and every later use of it returns
 *   GSRAD_ESTATE until a call rebuilds or refills it successfully.
 * - Layouts: E, B and their gradients are [N][Lt][K][3] (surfel, light,
 *   spherical-harmonic coefficient in the order Y00, Y1-1, Y10, Y11, ...,
 *   RGB), i.e. N rows of C = Lt*K*3 columns; colour = column % 3.  rho and
 *   albedo are [N][3].  K must be 1, 4, 9 or 16 (SH degree 0..3).
 */
#ifndef GSRAD_H
#define GSRAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gsrad_status;
#define GSRAD_OK 0
#define GSRAD_EINVAL (-1)    /* bad argument (null pointer, size, mismatch)   */
#define GSRAD_ENOMEM (-2)    /* device allocation failed                       */
#define GSRAD_EHIP (-3)      /* a HIP runtime call or kernel launch failed     */
#define GSRAD_ENAN (-4)      /* non-finite value found by a check              */
#define GSRAD_EOVERFLOW (-5) /* a fixed-capacity buffer overflowed             */
#define GSRAD_ESTATE (-6)    /* handle used in the wrong state                 */

#define GSRAD_FP32 0         /* precision argument of gsrad_transport_solve    */
#define GSRAD_BF16 1         /* dense BF16 matrix-core bounces (gsrad_ff_dense) */

/*
 * Gaussian surfels, structure of arrays, device FP32, length n
 * (Sec. 3.1, Eq. G): centre p, unit tangents t_u, t_v, unit normal
 * n = t_u x t_v, scales s_u, s_v > 0, and peak opacity o = alpha(0,0) of the
 * App. E opacity profile alpha(u,v) = 1 - exp(-c exp(-1.7 (u^2+v^2))),
 * c = -ln(1 - o).  o is clamped to [0, 0.9999].  The support is cut at
 * u^2 + v^2 <= 9.
 */
typedef struct gsrad_surfels {
    const float *px, *py, *pz;
    const float *tux, *tuy, *tuz;
    const float *tvx, *tvy, *tvz;
    const float *nx, *ny, *nz;
    const float *su, *sv;
    const float *opacity;
    int64_t n;
} gsrad_surfels;

/*
 * Ray-cast form-factor estimation parameters.
 *   rays_per_surfel  R >= 1: cosine-weighted hemisphere rays per receiver,
 *                    drawn with Philox4x64-10, counter (ray, receiver,
 *                    attempt, 0), key (seed, 0).
 *   seed             Philox key.
 *   t_min            compositing stops after the first hit that leaves the
 *                    transmittance below t_min (0 = never).
 *   t_eps            hits need t > t_eps; a value <= 0 selects
 *                    1e-5 * diagonal of the bounding box of the centres.
 *   topk             keep the topk largest entries per row (value desc,
 *                    index asc), 0 = keep all.
 *   flags            GSRAD_FF_NO_RECORDS: do not keep the per-ray hit
 *                    records (the opacity backward then recomputes every
 *                    ray by traversal instead of reading them).
 *                    GSRAD_FF_COMPACT: free the ray cast's scratch (hit
 *                    records not kept for the backward, row staging) before
 *                    returning, for many handles alive at once (batches of
 *                    scenes); the next cast on the handle allocates again.
 */
#define GSRAD_FF_NO_RECORDS 1
#define GSRAD_FF_COMPACT 2
typedef struct gsrad_ff_params {
    int32_t rays_per_surfel;
    int32_t topk;
    uint64_t seed;
    float t_min;
    float t_eps;
    int32_t flags;
    int32_t reserved;
} gsrad_ff_params;

typedef struct gsrad_bvh gsrad_bvh;   /* prepared surfels + LBVH            */
typedef struct gsrad_ff gsrad_ff;     /* sparse transport matrix F (CSR)    */
typedef struct gsrad_tape gsrad_tape;   /* forward iterates for the backward  */
typedef struct gsrad_batch gsrad_batch; /* scenes sharing one block-diagonal F */
typedef struct gsrad_mc gsrad_mc;       /* Monte-Carlo solver state and surfel groups */

/* Library version string (static storage). */
const char *gsrad_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *gsrad_last_error(void);

/*
 * Prepare the surfels and build a linear BVH over their 3-sigma bounds
 * (Karras 2012: 30-bit Morton codes of the centres, stable radix sort,
 * binary radix tree, bottom-up refit).  The surfel arrays are copied into
 * the handle, so they may change or be freed afterwards; a change of any
 * surfel (including its opacity) needs a new gsrad_build_bvh.
 * EINVAL: s or bvh NULL, a field pointer NULL, n < 1.
 */
gsrad_status gsrad_build_bvh(const gsrad_surfels *s, gsrad_bvh **bvh, void *stream);

/* Host query: number of surfels and the default t_eps (waits for the
 * stream the BVH was built on). */
gsrad_status gsrad_bvh_info(const gsrad_bvh *bvh, int64_t *n, float *t_eps_default);

/* Host query: height of the BVH (waits for the build stream). */
gsrad_status gsrad_bvh_height(const gsrad_bvh *bvh, int32_t *height);

/*
 * Effective area of every surfel, App. E closed form
 * int_P alpha dA = (2 pi / 3.4) s_u s_v Ein(c), in FP64: area_out is a device
 * double[n].  Used by the energy and reciprocity checks.
 */
gsrad_status gsrad_effective_area(const gsrad_bvh *bvh, double *area_out, void *stream);

/*
 * Lambertian reflectance per colour, rho_i = alpha_i(p_i) a_i = o_i a_i
 * (Sec. 5.3: the receiver opacity absorbed into the BRDF; App. A: the DC
 * coefficient c_00 = 4 a of the diffuse BRDF turns into the scalar a).
 * albedo [n][3] -> rho_out [n][3].
 */
gsrad_status gsrad_reflectance(const gsrad_bvh *bvh, const float *albedo, float *rho_out, void *stream);

/*
 * Form factors by ray casting (Eq. final-radiosity with the receiver kernel
 * a Dirac delta at p_i and a Lambertian receiver; App. B hemisphere form):
 *   F_ij = (1/R) sum_rays sum_{composited front-face hits q on surfel j}
 *          alpha_q prod_{k<q} (1 - alpha_k)
 * with hits ordered by (t, j) (Eq. L_I), self hits disabled, back faces
 * occluding but not reflecting (Sec. 5.1).  The result is a CSR matrix
 * with columns ascending in each row, values FP32, deterministic (bit
 * identical between runs).
 * EINVAL: null arguments, R < 1, topk < 0, t_min < 0.
 * Per-ray hit records (8 bytes per composited hit) grow automatically (the
 * call is then repeated) up to 2048 composited hits per ray; a row whose
 * distinct senders overflow the 4096-entry aggregation table is aggregated
 * again with 8192 entries within the same call, and a handle passed back in
 * starts from the capacities its previous call needed.
 * EOVERFLOW: more than 2048 composited hits on a ray, more than 8192
 * distinct senders in a row, or a traversal stack overflow.
 */
gsrad_status gsrad_form_factors(const gsrad_bvh *bvh, const gsrad_ff_params *p, gsrad_ff **ff, void *stream);

/* Host query: matrix size and number of stored entries. */
gsrad_status gsrad_ff_info(const gsrad_ff *ff, int64_t *n, int64_t *nnz);

/* Read-only device views of the CSR arrays: row_ptr int64[n+1],
 * col int32[nnz], val float[nnz].  Valid until the handle changes. */
gsrad_status gsrad_ff_view(const gsrad_ff *ff, const int64_t **row_ptr, const int32_t **col, const float **val);

/* Copy the CSR arrays into caller-owned device buffers of sizes n+1, nnz,
 * nnz (queued on stream). */
gsrad_status gsrad_ff_copy(const gsrad_ff *ff, int64_t *row_ptr, int32_t *col, float *val, void *stream);

/*
 * Wrap a caller-supplied CSR matrix (device arrays: row_ptr int64[n+1],
 * col int32[nnz] ascending within rows, val float[nnz]) as a transport
 * operator.  The arrays are copied.  For operator-level use of the solver
 * with an F that did not come from gsrad_form_factors.
 */
gsrad_status gsrad_ff_from_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                               const float *val, gsrad_ff **ff, void *stream);

/*
 * Dense BF16 copies of F for gsrad_transport_solve with GSRAD_BF16 (the
 * same operator B = E + rho F B of Eq. final-radiosity, evaluated as dense
 * matrix products on the matrix cores).  F and F^T are stored as
 * [Np][Np] BF16, Np = n rounded up to 256, each twice: the value rounded to
 * BF16 (hi) and the rounded remainder (lo), 4 * Np^2 * 2 bytes in all
 * (8.6 GB at n = 32768), owned by the handle.  Call again after F changes.
 * GSRAD_ENOMEM if the copies do not fit.
 */
gsrad_status gsrad_ff_dense(gsrad_ff *ff, void *stream);

/*
 * Direct light from isotropic point lights (Eq. forward rendering equation,
 * direct illumination; lights are infinitesimal emitters, Sec. 5.1):
 *   E_i,l,00,c = o_i a_i,c (2/sqrt(pi)) I_l max(0, n_i . w_il) / r_il^2 * T_il
 * with w_il the unit direction from p_i to the light, r_il its distance and
 * T_il the product of (1 - alpha) over every surfel crossed by the segment
 * (both faces occlude, t_eps as in the BVH's default).  Coefficients with
 * l >= 1 are written as 0.
 * light_pos [Lt][3] and light_I [Lt] are device arrays; E_out [n][Lt][K][3].
 */
gsrad_status gsrad_direct_light(const gsrad_bvh *bvh, const float *albedo, const float *light_pos,
                                const float *light_I, int32_t n_lights, int32_t K, float *E_out, void *stream);

/*
 * Bounce iterations (Eq. final-radiosity, scalar Lambertian transfer
 * applied to every SH coefficient and light):
 *   B^(0) = E,   B^(k+1) = E + rho * (F B^(k)),   k = 0 .. n_bounces-1
 * B_out = B^(n_bounces) (n_bounces = 0 copies E: direct light only).  If
 * tape is non-NULL the iterates B^(0..n-1) are kept in *tape (created or
 * re-used) for gsrad_transport_backward.  The accumulation order is fixed,
 * so results are bit identical between runs.
 *
 * precision GSRAD_FP32: sparse products on the CSR F in FP32.
 * precision GSRAD_BF16: dense products on the BF16 copies made by
 *   gsrad_ff_dense, FP32 accumulation: the first n_bounces - 1 bounces use
 *   F_hi and B rounded to BF16; the last one is the correction sweep
 *   F B ~ F_hi B_hi + F_hi B_lo + F_lo B_hi (16-bit operands, FP32
 *   accumulation), so that the result is B^(n) of the same recurrence with
 *   only the first n - 1 applications in BF16.  Error vs FP64 within 1e-3
 *   relative max-norm.  The tape then keeps F B^(k) (FP32) and B^(k)
 *   (BF16) for the backward.
 */
gsrad_status gsrad_transport_solve(const gsrad_ff *ff, const float *rho, const float *E, int32_t n_lights,
                                   int32_t K, int32_t n_bounces, int32_t precision, float *B_out,
                                   gsrad_tape **tape, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP32
 * bounces of gsrad_transport_solve without a tape, B_out = B^(n_bounces),
 * bit-identical to it.  The two ping-pong iterates live in a fixed 64 MiB
 * device array of the library, one per GPU, held until the process ends, so
 * the call allocates nothing: it needs 2 * n * n_lights * K * 3 * 4 <= 2^26
 * bytes when n_bounces >= 2 and returns GSRAD_EINVAL for larger operators.
 * The array belongs to the device current on the calling thread (which must
 * be the device of stream and of every buffer).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race and must be serialised by the caller.  FP32 only.
 */
gsrad_status gsrad_transport_solve_noalloc(const gsrad_ff *ff, const float *rho, const float *E, int32_t n_lights,
                                           int32_t K, int32_t n_bounces, float *B_out, void *stream);

/*
 * Exact adjoint of gsrad_transport_solve for dL/dB^(n) = grad_B (Eq.
 * final_dL_dE in division-free form, truncated like the forward):
 *   lambda^(n) = grad_B,  lambda^(k) = F^T (rho * lambda^(k+1))
 *   grad_E     = sum_{k=0..n} lambda^(k)
 *   grad_rho   = sum_{k<n} sum_{light, coef} lambda^(k+1) * (F B^(k))
 *                (per colour; Eq. final-dl-dbrdf before its fixed-point limit)
 *   grad_F[e]  = sum_{k<n} < rho_i * lambda_i^(k+1), B_j^(k) >  for the
 *                stored entry e = (i, j) (decay term of Eq. dl-dgeo-0)
 * grad_E [n][Lt][K][3], grad_rho [n][3], grad_F [nnz] in F's CSR order
 * (may be NULL).  rho must be the rho of the forward call.
 * A tape made with GSRAD_BF16 runs the adjoint of that forward (its first
 * step the correction sweep on F^T, the others BF16 on F^T) and forms
 * grad_F as the dense product sum_k (rho lambda^(k+1)) (B^(k))^T on the
 * matrix cores (both operands split into BF16 hi + lo, the three leading
 * products accumulated in FP32: the sum cancels, so plain BF16 operands
 * would leave errors near 4e-3) into an [n][n] FP32
 * array held by the tape (gsrad_tape_grad_F_dense copies it out), from
 * which the stored entries are copied to grad_F.
 */
gsrad_status gsrad_transport_backward(const gsrad_ff *ff, const gsrad_tape *tape, const float *rho,
                                      const float *grad_B, float *grad_E, float *grad_rho, float *grad_F,
                                      void *stream);

/*
 * Copy of the dense dL/dF [n][n] FP32 (row-major, caller-owned device
 * buffer) computed by the last gsrad_transport_backward with grad_F != NULL
 * on a GSRAD_BF16 tape; GSRAD_ESTATE if there is none.
 */
gsrad_status gsrad_tape_grad_F_dense(const gsrad_tape *tape, float *grad_F_out, void *stream);

/*
 * Batches of scenes of uneven size (many scenes, each lit by its own set of
 * point lights, propagated together; the batch-size paragraph of the
 * ablation study in Sec. 9 propagates once and renders many images from one
 * propagation).  gsrad_batch_create joins the scenes' transport operators
 * (each from gsrad_form_factors or gsrad_ff_from_csr, n_s rows) into one
 * block-diagonal F with global indices: scene s owns rows
 * [row_off_s, row_off_s + n_s) in the order given.  Scene s has
 * lights[s] >= 1 point lights and C_s = lights[s] * K * 3 columns, so rho
 * is [sum n_s][3] and E, B and their gradients are ragged: scene s's rows
 * are one [n_s][lights[s]][K][3] block, blocks concatenated in scene order
 * (val_off_s = sum_{t<s} n_t C_t values before it).  lights is a host
 * array of n_scenes entries; the scenes' handles may be destroyed after
 * the call.  *batch == NULL creates a batch; an existing batch with the
 * same scene sizes, lights and K is refilled with the new operators and
 * keeps its tuned shapes and captured loop.
 *
 * gsrad_batch_transport_solve runs the bounces of Eq. final-radiosity on
 * every scene at once: each bounce is one persistent launch in which
 * groups of lanes take rows from a work counter, largest cost (entries x
 * columns) first.  The lanes-per-row shape (16, 32 or 64) is chosen by
 * timing each candidate on the batch's own rows at the first solve (every
 * candidate adds each output in the same order, so the choice never
 * changes a result).  The bounce loop and the adjoint loop are each
 * captured once into a HIP graph and replayed while their arguments stay
 * the same.  The iterates are kept
 * in the batch for gsrad_batch_transport_backward, the exact adjoint
 * (same formulas as gsrad_transport_backward; grad_F in the block-diagonal
 * F's CSR order, see gsrad_batch_ff).  Calls on one batch must not overlap.
 */
gsrad_status gsrad_batch_create(const gsrad_ff *const *ffs, int32_t n_scenes, const int32_t *lights, int32_t K,
                                gsrad_batch **batch, void *stream);
/* total rows, total values of the ragged arrays, and the lanes per row
 * chosen for the bounce and the adjoint (0 before the first solve) */
gsrad_status gsrad_batch_info(const gsrad_batch *batch, int64_t *rows, int64_t *vals, int32_t *lanes_bounce,
                              int32_t *lanes_adjoint);
/* the block-diagonal F (read-only; valid while the batch lives) */
gsrad_status gsrad_batch_ff(const gsrad_batch *batch, const gsrad_ff **ff);
gsrad_status gsrad_batch_transport_solve(gsrad_batch *batch, const float *rho, const float *E, int32_t n_bounces,
                                         float *B_out, void *stream);
gsrad_status gsrad_batch_transport_backward(gsrad_batch *batch, const float *rho, const float *grad_B,
                                            float *grad_E, float *grad_rho, float *grad_F, void *stream);
/*
 * Force the lanes per row of the batch's bounce and adjoint launches (16, 32
 * or 64; 0 returns to the timed choice).  Every shape adds each output in
 * the same order, so results are bit-identical whatever is chosen; for
 * tests and tuning experiments.  The timed choice is remembered per batch
 * shape (rows, stored entries, values) for the rest of the process.
 */
gsrad_status gsrad_batch_set_lanes(gsrad_batch *batch, int32_t lanes_bounce, int32_t lanes_adjoint);
/*
 * Precision of the batch's transport (GSRAD_FP32, the default, or
 * GSRAD_BF16; the batch-size paragraph of Sec. 9's ablation: many images
 * from one propagation, here with half the bytes per gathered row).  With
 * GSRAD_BF16 the first n_bounces - 1 bounces gather the sender rows B^(k)
 * rounded to BF16 (round to nearest even) and sum in FP32; the last bounce
 * gathers the FP32 B^(n-1), as the dense BF16 path's correction sweep does.
 * The backward is the adjoint of that map with the rounding taken as the
 * identity: its first step gathers the FP32 lambda^(n), the others
 * lambda^(k+1) rounded to BF16; grad_F and grad_rho are formed from the
 * FP32 iterates (their sums cancel).  Error vs FP64 within 1e-3 relative
 * max-norm; deterministic.  A change of precision needs a new forward
 * solve before the backward (GSRAD_ESTATE otherwise).
 */
gsrad_status gsrad_batch_set_precision(gsrad_batch *batch, int32_t precision);
void gsrad_batch_destroy(gsrad_batch *batch);
/*
 * Monte-Carlo solver (Sec. 7, Alg. Monte-Carlo Solver, App. D) of the
 * scalar Lambertian transport B = E + rho (F B) with the centre-to-centre
 * decay of Sec. 8 (F_ij = lambda_j A_j T_ij |n_i.w||n_j.w| / (pi r^2), its
 * transmittance from one segment per drawn pair).  With E the direct light
 * (the lights' radiance already shot to every surfel) this is the paper's
 * hybrid scheme: the Monte-Carlo steps solve the remaining transport.
 *
 * gsrad_mc_create groups the surfels by K-Means on their centres (groups
 * <= 0: round(sqrt(n)); kmeans_iters Lloyd iterations from every
 * (n/groups)-th surfel in Morton order), each group keeping its mean centre
 * and normal.  The handle follows the BVH: a rebuild needs a new handle
 * (calls on the old one return GSRAD_ESTATE), and the BVH must not be
 * destroyed while the handle is used.
 *
 * gsrad_mc_estimate: one next event for every receiver a given the current
 * radiance B [n][Lt][K][3]: a group g drawn with probability proportional
 * to L_g (|n_a.w_g| + 0.05)(|nbar_g.w_g| + 0.05) / max(r_g^2, (0.01 diag)^2)
 * (L_g the summed luminance of its members' DC radiance), a member j != a
 * proportional to lum(B_j) |n_a.v||n_j.v| / |v|^4 (Eq. importance-sampling),
 * both by the inverse of their running sums (the same distribution as the
 * streaming weighted reservoir), and the one-point estimate (Eq.
 * one-point-estimator) delta_a = E_a + rho_a F_aj B_j / Pr[j] (E_a alone if
 * nothing can be drawn), written to delta_out [n][Lt][K][3].  Its
 * expectation is E + rho (F B) over the pairs with Pr > 0.  Draws:
 * Philox4x64-10 counter (receiver, step, 0, 2), key (seed, 0).
 *
 * gsrad_mc_solve: steps rounds of the TD(0) update (Eq. update) from zero:
 * the receivers are every surfel for the first 8 rounds, then n draws with
 * replacement in proportion to each surfel's tracked variance (summed over
 * the columns; stratified inverse CDF of 2^24-level integer weights,
 * counter (slot, step, 1, 1)); each receiver averages its estimates
 * (S_a += delta, S2_a += delta^2, D_a += 1, B_a = S_a / D_a).  B_out
 * [n][Lt][K][3]; visits_out [n] (uint32, may be NULL) the D_a.  Bit
 * identical between runs with the same seed.
 */
gsrad_status gsrad_mc_create(const gsrad_bvh *bvh, int32_t groups, int32_t kmeans_iters, gsrad_mc **mc,
                             void *stream);
gsrad_status gsrad_mc_estimate(gsrad_mc *mc, const float *lambda, const float *rho, const float *E, const float *B,
                               int32_t n_lights, int32_t K, uint64_t seed, int32_t step, float *delta_out,
                               void *stream);
gsrad_status gsrad_mc_solve(gsrad_mc *mc, const float *lambda, const float *rho, const float *E, int32_t n_lights,
                            int32_t K, int32_t steps, uint64_t seed, float *B_out, uint32_t *visits_out,
                            void *stream);
void gsrad_mc_destroy(gsrad_mc *mc);


/*
 * Directional transfer with the diffuse + Phong BRDF (Eq. final-radiosity
 * with f_i(w) = f^c_i x Ybar(w), Sec. 3.2; Eq. brdf, Sec. 5.1; App. A).
 * Coefficient vectors of surfel i (E_i, B_i, f^c_i, the rows of R) are taken
 * in its tangent frame (t_u, t_v, n) as (x, y, z): there App. A's
 * c_lm = (-1)^m c_l0 is the Phong lobe about the mirror direction.  Per
 * stored entry (i, j) of F the directional factors use the unit direction
 * d_ij from p_i to p_j (the BRDF and radiance factors taken as constant over
 * the pair, as Sec. 8 does); F_ij carries the decay:
 *   (T X)_i[l][a][c] = sum_j F_ij Y_a(d_ij in i's frame) sum_b Y_b(-d_ij in j's frame) X_j[l][b][c]
 *   B^(0) = E,  B^(k+1) = E + R (.) (T B^(k))
 * with R_i[a][c] = pi o_i f^c_i[a][c] (receiver opacity absorbed into the
 * BRDF; pi from the cosine-weighted hemisphere estimator of F).  For
 * k = 1 (Lambertian) and DC-only radiance this is exactly
 * gsrad_transport_solve.  Real SH in the order Y00, Y1-1, Y10, Y11, ...
 *
 * gsrad_brdf_reflectance: R [n][K][3] from the BRDF parameters per surfel:
 *   blend k [n] (diffuse weight), diffuse albedo a^d [n][3], specular
 *   albedo a^s [n][3], shininess s [n] (>= 0):
 *   f^c_00 = 4 k a^d + (1 - k) a^s,
 *   f^c_lm = (-1)^m (1 - k) g_l(s) a^s, g_1 = (s+1)/(s+2), g_2 = s/(s+3),
 *   g_3 = (s+1)(s-1)/((s+2)(s+4)).
 * gsrad_brdf_backward: the gradients of sum(grad_R * R) with respect to the
 *   opacity (0 where the clamp is active), k, a^d, a^s and s (each output
 *   may be NULL; written, not accumulated).
 */
gsrad_status gsrad_brdf_reflectance(const gsrad_bvh *bvh, const float *k, const float *albedo_d,
                                    const float *albedo_s, const float *shininess, int32_t K, float *R_out,
                                    void *stream);
gsrad_status gsrad_brdf_backward(const gsrad_bvh *bvh, const float *k, const float *albedo_d, const float *albedo_s,
                                 const float *shininess, int32_t K, const float *grad_R, float *grad_opacity,
                                 float *grad_k, float *grad_albedo_d, float *grad_albedo_s, float *grad_shininess,
                                 void *stream);

/*
 * Direct light with the BRDF (Eq. forward rendering equation, direct
 * illumination): E_i,l = (R_i / pi) (.) Y(w_il in i's frame)
 * I_l max(0, n_i . w_il) / r_il^2 T_il, w_il the unit direction to light l,
 * T_il the shadow transmittance as in gsrad_direct_light.  R [n][K][3],
 * E_out [n][n_lights][K][3].
 */
gsrad_status gsrad_direct_light_sh(const gsrad_bvh *bvh, const float *R, int32_t K, const float *light_pos,
                                   const float *light_I, int32_t n_lights, float *E_out, void *stream);

/*
 * Bounces of the directional transfer above on F (any gsrad_ff of n rows:
 * ray-cast or imported) with the geometry of bvh (same n surfels).  R
 * [n][K][3], E and B_out [n][n_lights][K][3].  The tape keeps B^(k) and
 * T B^(k) for gsrad_transport_backward_sh.  Deterministic.
 */
gsrad_status gsrad_transport_solve_sh(const gsrad_ff *ff, const gsrad_bvh *bvh, const float *R, const float *E,
                                      int32_t n_lights, int32_t K, int32_t n_bounces, float *B_out,
                                      gsrad_tape **tape, void *stream);

/*
 * Exact adjoint of gsrad_transport_solve_sh for dL/dB^(n) = grad_B (Eq.
 * final_dL_dE in division-free form; the backward runs the same transfer
 * on F^T with the pair directions reversed, App. C):
 *   lambda^(n) = grad_B,  lambda^(k) = T^T (R (.) lambda^(k+1)),  grad_E = sum_k lambda^(k)
 *   grad_R[i][a][c] = sum_{k<n} sum_l lambda^(k+1)_i[l][a][c] (T B^(k))_i[l][a][c]
 *   grad_F[e = (i, j)] = sum_{k<n} sum_{l, c} (Y(d_ij)^T (R (.) lambda^(k+1))_i[l][:, c])
 *                                             (Y(-d_ij)^T B^(k)_j[l][:, c])
 * (Eq. final-dl-dbrdf and the decay term of Eq. dl-dgeo-0 before their
 * fixed-point limits).  grad_R [n][K][3] and grad_F [nnz] may be NULL.
 */
gsrad_status gsrad_transport_backward_sh(const gsrad_ff *ff, const gsrad_bvh *bvh, const gsrad_tape *tape,
                                         const float *R, const float *grad_B, float *grad_E, float *grad_R,
                                         float *grad_F, void *stream);

/*
 * Centre-to-centre form factors with a learnable scale (Sec. 8, Eq.
 * radiosity-approx-1 and the approximated forward rendering equation; the
 * effective area of App. E), on the pattern of an existing operator
 * (typically the pairs a ray cast recorded as visible, Sec. 6): for every
 * stored entry (i, j) of pattern,
 *   F_ij = lambda_j A_j T_ij |n_i . w| |n_j . w| / (pi r^2),
 *   w = (p_j - p_i) / r,  r = |p_j - p_i|,
 * i.e. the scalar Lambertian form V_ji / pi of the paper's decay, with A_j
 * the App. E area, lambda_j > 0 the per-surfel scale (device float [n]) and
 * T_ij the product of (1 - alpha) over the surfels other than i and j whose
 * support the segment between the centres crosses (both faces occlude; the
 * segment's ends trimmed by the BVH's t_eps; one segment per entry).  The
 * result is a new F handle (*ff created or refilled; it must differ from
 * pattern) with pattern's sparsity, usable by every transport call.
 * Deterministic.  EOVERFLOW: traversal stack overflow.
 */
gsrad_status gsrad_ff_center(const gsrad_bvh *bvh, const gsrad_ff *pattern, const float *lambda, gsrad_ff **ff,
                             void *stream);

/*
 * Gradients of sum_e grad_F[e] F_e through gsrad_ff_center (the decay term
 * of Eq. dl-dgeo-0 with the decay of Sec. 8, for every recorded pair), with
 * respect to lambda and to the surfel fields of the pairs' ends and of every
 * occluder on their segments: centres, tangent frames (t_u, t_v, n as given,
 * not renormalised), scales and opacities (0 where the opacity clamp is
 * active).  Each output is a device float [n], written (not accumulated);
 * any may be NULL.  The sums are 64-bit fixed point with a per-field
 * power-of-two scale from the largest contribution (two passes over the
 * segments), bit-identical between runs.  ff must come from
 * gsrad_ff_center on this bvh as it is now (EINVAL otherwise).
 */
typedef struct gsrad_surfel_grads {
    float *px, *py, *pz;
    float *tux, *tuy, *tuz;
    float *tvx, *tvy, *tvz;
    float *nx, *ny, *nz;
    float *su, *sv;
    float *opacity;
} gsrad_surfel_grads;

gsrad_status gsrad_ff_center_backward(const gsrad_bvh *bvh, const gsrad_ff *ff, const float *lambda,
                                      const float *grad_F, float *grad_lambda, const gsrad_surfel_grads *grads,
                                      void *stream);

/*
 * Geometry gradients through the ray-cast form factors (Eq. dl-dgeo-0, the
 * decay term over the recorded pairs, Sec. 6): for grad_F = dL/dF [nnz] in
 * F's CSR order, the gradient of sum_e grad_F[e] F_e with respect to every
 * surfel field of the hit surfels (the hit point u, v on each through its
 * centre, frame and scales; its opacity through c) and of the receivers
 * (ray origin p_i, ray direction x t_u + y t_v + z n_i from the ray's disc
 * sample), with the compositing backward's dL/dalpha per recorded hit; the
 * hit sets, their order and the cut are those of the forward pass.  The
 * opacity output is the F part of gsrad_opacity_backward's (without the
 * receiver term).  Outputs device float [n] each (written; NULL skipped).
 * Needs the per-ray hit records (GSRAD_ESTATE without them).  64-bit fixed
 * point sums with per-field scales from a first pass: bit-identical between
 * runs.
 */
gsrad_status gsrad_geometry_backward(const gsrad_bvh *bvh, const gsrad_ff *ff, const float *grad_F,
                                     const gsrad_surfel_grads *grads, void *stream);

/*
 * Gradients through gsrad_direct_light (Eq. forward rendering equation,
 * direct illumination; the light-position optimisation of Sec. 9) for
 * grad_E = dL/dE [n][Lt][K][3] (only its DC coefficients matter): with
 * v = x_l - p_i, r = |v|, E_c = o_i a_c (2/sqrt(pi)) I_l max(0, n_i . v) T_il / r^3,
 * the gradients with respect to the light positions grad_light_pos
 * [Lt][3], intensities grad_light_I [Lt], the albedo grad_albedo [n][3],
 * and the surfel fields of the receivers (centre, normal, opacity) and of
 * every occluder on the shadow segments (as in gsrad_ff_center_backward),
 * in grads.  Every output is written (NULL skipped).  Fixed-point sums with
 * per-field scales from a first pass: bit-identical between runs.
 */
gsrad_status gsrad_direct_light_backward(const gsrad_bvh *bvh, const float *albedo, const float *light_pos,
                                         const float *light_I, int32_t n_lights, int32_t K, const float *grad_E,
                                         float *grad_light_pos, float *grad_light_I, float *grad_albedo,
                                         const gsrad_surfel_grads *grads, void *stream);

/*
 * Opacity and albedo gradients (Eq. dl-dgeo-0, decay term, restricted to
 * opacity; and rho = o a).  For every ray of every receiver i the hits of
 * the forward pass are recomputed and, with G_q = grad_F[i, j_q] / R on
 * front hits kept in F (0 otherwise) and w_q = alpha_q T_q,
 *   dL/dalpha_q = G_q T_q - (sum_{p>q} G_p w_p) / (1 - alpha_q)
 *   dL/do_j    += dL/dalpha_q * gamma_q (1 - o_j)^(gamma_q - 1),
 *                 gamma_q = exp(-1.7 (u_q^2 + v_q^2))
 * plus the receiver term dL/do_i += sum_c grad_rho_ic a_ic, and
 * dL/da = grad_rho * o (both zero where the opacity clamp is active).
 * The hits are read from the per-ray records gsrad_form_factors kept (it
 * keeps them when the record slab of all receivers, n R rcap slots of
 * 8 B (rcap >= 256 per ray), fits in half of the device memory free at the
 * cast, and GSRAD_FF_NO_RECORDS is not set); otherwise every ray is
 * recomputed by traversal, with identical decisions.
 * grad_F is [nnz] in F's CSR order; grad_rho and albedo [n][3];
 * grad_opacity [n], grad_albedo [n][3] (either may be NULL).  The hit
 * recomputation needs the ff handle made from this bvh.
 */
gsrad_status gsrad_opacity_backward(const gsrad_bvh *bvh, const gsrad_ff *ff, const float *grad_F,
                                    const float *grad_rho, const float *albedo, float *grad_opacity,
                                    float *grad_albedo, void *stream);

/*
 * Recorded hits (Sec. 6: the pairs found visible in the forward pass), for
 * diagnostics and tests: for every ray r of each listed receiver k (device
 * int64 receivers[n_receivers], original indices) the ray direction
 * dirs[(k*R + r)*3 + 0..2], the number of composited hits count[k*R + r] and
 * the first max_hits of them in depth order: surfel hit_j, depth hit_t,
 * front face hit_front, transmittance in front of it hit_T (arrays
 * [n_receivers*R*max_hits]).  Same rays, decisions and compositing as
 * gsrad_form_factors with the same parameters (t_eps <= 0: default).
 */
gsrad_status gsrad_ray_hits(const gsrad_bvh *bvh, const gsrad_ff_params *p, const int64_t *receivers,
                            int64_t n_receivers, int32_t max_hits, float *dirs, int32_t *count, int32_t *hit_j,
                            float *hit_t, int8_t *hit_front, float *hit_T, void *stream);

/*
 * FP64 checks on the GPU.  out_host[0] = || E + rho*(F B) - B ||_2 / ||B||_2
 * (the fixed-point residual of B), out_host[1] = max_i sum_j F_ij (energy
 * bound: <= 1 for ray-cast F), out_host[2] = 1 if any value of E, rho or
 * B is not finite.  Waits for the stream.  Returns GSRAD_ENAN if
 * out_host[2] != 0.
 */
gsrad_status gsrad_check(const gsrad_ff *ff, const float *rho, const float *E, const float *B, int32_t n_lights,
                         int32_t K, double *out_host, void *stream);

/*
 * Reciprocity of the estimated operator: A_i F_ij = A_j F_ji holds for
 * exact form factors (the reciprocity of classical radiosity, which the
 * paper does not state; an invariant of the estimator), with A the App. E
 * effective areas of gsrad_effective_area.  FP64 over the stored entries, the mirror entry
 * F_ji found in row j (0 when it is not stored, e.g. cut by top-k):
 *   out_host[0] = sum |A_i F_ij - A_j F_ji| / sum A_i F_ij
 *   out_host[1] = max |A_i F_ij - A_j F_ji| / max(A_i F_ij, A_j F_ji)
 * The ray-cast estimate is reciprocal only in expectation and up to the
 * receiver-centre approximation, so these measure noise plus that bias.
 * bvh and ff must describe the same n surfels.
 */
gsrad_status gsrad_check_reciprocity(const gsrad_bvh *bvh, const gsrad_ff *ff, double *out_host, void *stream);

/*
 * Timing of the library's phases with HIP events recorded on the caller's
 * stream around each kernel group (bvh_build, ff_trace, ff_aggregate,
 * ff_csr, direct_light, bounce, transpose, adjoint, sddmm, opacity_records,
 * opacity_pass1, opacity_pass2, opacity_finish).  gsrad_profile_enable(1) clears the record
 * and starts recording, 0 stops.  gsrad_profile_report waits for the events
 * and writes one line per phase into buf (host, len bytes):
 * "name<TAB>count<TAB>total_ms<TAB>min_ms<TAB>max_ms\n".  Not thread safe.
 */
gsrad_status gsrad_profile_enable(int32_t on);
gsrad_status gsrad_profile_report(char *buf, int64_t len);

void gsrad_bvh_destroy(gsrad_bvh *bvh);
void gsrad_ff_destroy(gsrad_ff *ff);
void gsrad_tape_destroy(gsrad_tape *tape);

#ifdef __cplusplus
}
#endif

#endif /* GSRAD_H */
