// C ABI of libgsrad: argument validation, handle lifetime, buffer reuse and
// the order of kernel launches for each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "bvh_build.h"
#include "gsrad_internal.h"
#include "trace_api.h"
#include "dense_api.h"
#include "batch_api.h"
#include "sh_api.h"

namespace gsrad {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

gsrad_status check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return GSRAD_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return GSRAD_EHIP;
}

// A growable device allocation.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    gsrad_status ensure(size_t want, const char *what) {
        if (want <= bytes && p) return GSRAD_OK;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            bytes = 0;
        }
        if (want == 0) want = 256;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            set_error("out of device memory allocating %zu bytes for %s", want, what);
            return GSRAD_ENOMEM;
        }
        bytes = want;
        return GSRAD_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T *as() const {
        return static_cast<T *>(p);
    }
};

constexpr int kTapeSH = 2;          // tape precision tag of gsrad_transport_solve_sh
constexpr int kLog2Table = 12;      // 4096-entry aggregation table per receiver
constexpr int kLog2TableMax = 13;   // 8192 entries: rows with more distinct senders
constexpr int kRecCap = 256;        // recorded hits per ray to start with (composited: ~27 mean here)
constexpr size_t kChunkRecordBudget = size_t(4) << 30;   // records of one chunk otherwise

// ---------------------------------------------------------------------------
// optional per-phase timing with HIP events on the caller's stream
// ---------------------------------------------------------------------------
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
static bool g_prof = false;
static std::vector<ProfRec> g_recs;
static std::vector<hipEvent_t> g_pool;

static hipEvent_t prof_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

struct ProfScope {
    ProfRec r{nullptr, nullptr, nullptr};
    hipStream_t st;
    ProfScope(const char *name, hipStream_t s) : st(s) {
        if (!g_prof) return;
        r.name = name;
        r.a = prof_event();
        if (r.a) (void)hipEventRecord(r.a, st);
    }
    ~ProfScope() {
        if (!g_prof || !r.a) return;
        r.b = prof_event();
        if (!r.b) return;
        (void)hipEventRecord(r.b, st);
        g_recs.push_back(r);
    }
};

static void prof_clear() {
    for (ProfRec &r : g_recs) {
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
}

}  // namespace gsrad

using namespace gsrad;

struct gsrad_bvh {
    int64_t n = 0;               // 0 after a failed (re)build: unusable
    uint64_t gen = 0;            // unique per successful build
    hipStream_t stream = nullptr;
    DevBuf rec, nodes, leafbox, leaf_parent, inv, cst, opc, opraw, area, dado, bounds, height, temp, lacc;
    BvhBuffers B;
    BvhDev dev() const {
        BvhDev d;
        d.n = n;
        d.rec = B.rec;
        d.nodes = B.nodes;
        d.inv = B.inv;
        d.c = B.cst;
        d.op = B.opc;
        d.raw_op = B.opraw;
        d.bounds = B.bounds;
        d.area = B.area;
        d.dado = B.dado;
        d.leaf_box_r = 0.0f;
        return d;
    }
    ~gsrad_bvh() {
        for (DevBuf *b : {&rec, &nodes, &leafbox, &leaf_parent, &inv, &cst, &opc, &opraw, &area, &dado, &bounds, &height,
                          &temp, &lacc})
            b->release();
    }
};

struct gsrad_ff {
    int64_t n = 0, nnz = 0;      // n = 0 after a failed (re)fill: unusable
    int max_row = 0;
    DevBuf row_ptr, col, val;
    // transpose, built on first use by the backward
    bool has_t = false;
    // receivers in Morton order (ray-cast F): the order the row kernels take
    bool has_order = false;
    DevBuf row_order;
    DevBuf t_row_ptr, t_col, t_val, t_temp;
    // unique per successful fill of the values (0: unusable); tapes record it
    uint64_t fill_gen = 0;
    // provenance for the opacity backward
    const gsrad_bvh *bvh = nullptr;
    uint64_t bvh_gen = 0;
    // centre-to-centre values (gsrad_ff_center): the BVH they were made from
    const gsrad_bvh *center_bvh = nullptr;
    uint64_t center_gen = 0;
    int R = 0, topk = 0;
    uint64_t seed = 0;
    float t_eps = 0.0f, t_min = 0.0f;
    // recorded hits (j, +-gamma) per ray for the backward, if they fit
    bool has_records = false;
    int rec_cap = 0;
    DevBuf recs, rcnt;
    // capacities the last ray cast needed (starting points of the next)
    int deep_stack = 0, agg_log2h = 0;
    // scratch of the ray-cast path
    DevBuf slab, ell_col, ell_val, row_len, err, scan_temp, redo, pools;
    // opacity backward: per-XCD fixed-point accumulators and scale
    DevBuf opac, cacc;
    // dense BF16 copies (gsrad_ff_dense): F and F^T, hi and lo parts
    bool has_dense = false;
    int64_t Np = 0;
    DevBuf d_hi, d_lo, dt_hi, dt_lo;
    DevBuf xa, xb, xl;   // transposed BF16 operands of the dense products
    Csr csr() const {
        Csr c;
        c.n = n;
        c.nnz = nnz;
        c.row_ptr = row_ptr.as<int64_t>();
        c.col = col.as<int32_t>();
        c.val = val.as<float>();
        c.order = has_order ? row_order.as<int32_t>() : nullptr;
        return c;
    }
    Csr csr_t() const {
        Csr c;
        c.n = n;
        c.nnz = nnz;
        c.row_ptr = t_row_ptr.as<int64_t>();
        c.col = t_col.as<int32_t>();
        c.val = t_val.as<float>();
        c.order = has_order ? row_order.as<int32_t>() : nullptr;
        return c;
    }
    ~gsrad_ff() {
        for (DevBuf *b : {&row_ptr, &col, &val, &t_row_ptr, &t_col, &t_val, &t_temp, &slab, &ell_col, &redo, &row_order,
                          &ell_val, &row_len, &err, &scan_temp, &pools, &recs, &rcnt, &d_hi, &d_lo, &dt_hi, &dt_lo, &xa, &xb, &xl, &opac,
                          &cacc})
            b->release();
    }
};

struct gsrad_tape {
    int64_t n = 0;
    int C = 0, nb = 0, Lt = 0, K = 0;
    int precision = GSRAD_FP32;
    const gsrad_ff *ff = nullptr;     // null: unusable (no solve yet, or the last one failed)
    uint64_t ff_gen = 0;              // the fill of ff the tape was recorded on
    const gsrad_bvh *bvh = nullptr;   // directional transfer: the geometry it used
    uint64_t bvh_gen = 0;
    DevBuf B, L, lam0, pp;
    // GSRAD_BF16: Q^(k) = F B^(k) (FP32 [nb][n][C]), B^(k) in BF16 as
    // [Np][Kp] rows (k-major columns), the adjoint's BF16 rows
    // rho lambda^(k+1), its FP32 iterates, and the dense dL/dF [n][n]
    int64_t Kp = 0;
    bool has_G = false;
    DevBuf Q, bb, bb_lo, pb, pb_lo, lam_a, lam_b, G;
    ~gsrad_tape() {
        for (DevBuf *b : {&B, &L, &lam0, &pp, &Q, &bb, &bb_lo, &pb, &pb_lo, &lam_a, &lam_b, &G}) b->release();
    }
};

struct gsrad_batch {
    int32_t S = 0;
    int K = 0;
    int64_t rows = 0, vals = 0;
    gsrad_ff *F = nullptr;   // block-diagonal, owned
    DevBuf row_off, val_off, scene_C, row_scene, order, counter, temp;
    std::vector<int64_t> scene_rows;   // row offsets (host copy)
    std::vector<int32_t> scene_cols;   // C_s (host copy)
    // forward iterates B^(0..nb-1) and adjoint iterates lambda^(1..nb)
    int nb = -1;
    DevBuf Bt, Lt, lam0;
    // GSRAD_BF16: the gathered rows of all but the last bounce (and of all but
    // the first adjoint step) in BF16, two ping-pong slots each
    int precision = GSRAD_FP32;
    DevBuf Bh, Lh;
    // lanes per row chosen by timing (0: not yet)
    int lpr_fwd = 0, lpr_adj = 0;
    // captured bounce loop and the arguments it was captured with
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_rho = nullptr, *g_E = nullptr, *g_B = nullptr, *g_tape = nullptr, *g_h = nullptr;
    int g_nb = -1, g_lpr = 0, g_prec = GSRAD_FP32;
    // captured adjoint loop and its arguments
    hipGraph_t agraph = nullptr;
    hipGraphExec_t aexec = nullptr;
    const void *a_rho = nullptr, *a_gE = nullptr, *a_L = nullptr, *a_lam0 = nullptr, *a_ft[3] = {}, *a_h = nullptr;
    int a_nb = -1, a_lpr = 0, a_prec = GSRAD_FP32;
    // lanes per row forced by gsrad_batch_set_lanes (0: tuned)
    int force_fwd = 0, force_adj = 0;
    gsrad::BatchDev dev() const {
        gsrad::BatchDev d;
        d.rows = rows;
        d.scenes = S;
        d.row_off = row_off.as<int64_t>();
        d.val_off = val_off.as<int64_t>();
        d.scene_C = scene_C.as<int32_t>();
        d.row_scene = row_scene.as<int32_t>();
        d.order = order.as<int64_t>();
        return d;
    }
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        g_nb = -1;
        if (aexec) (void)hipGraphExecDestroy(aexec);
        if (agraph) (void)hipGraphDestroy(agraph);
        aexec = nullptr;
        agraph = nullptr;
        a_nb = -1;
    }
    ~gsrad_batch() {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
        delete F;
        for (DevBuf *b : {&row_off, &val_off, &scene_C, &row_scene, &order, &counter, &temp, &Bt, &Lt, &lam0, &Bh, &Lh})
            b->release();
    }
};

struct gsrad_mc {
    const gsrad_bvh *bvh = nullptr;
    uint64_t gen = 0;
    int64_t n = 0;
    int G = 0;
    float rmin2 = 0.0f;
    DevBuf cent, gnrm, L, key, ids, skey, members, count, goff, rtemp, stemp;
    DevBuf S, S2, B, delta, var, D, q, maxbits, recv, cdf, err;
    gsrad::McBuffers mb() const {
        gsrad::McBuffers m;
        m.cent = cent.as<float>();
        m.gnrm = gnrm.as<float>();
        m.L = L.as<float>();
        m.key = key.as<uint32_t>();
        m.ids = ids.as<uint32_t>();
        m.skey = skey.as<uint32_t>();
        m.members = members.as<uint32_t>();
        m.count = count.as<uint32_t>();
        m.goff = goff.as<int64_t>();
        m.rtemp = rtemp.p;
        m.rtemp_bytes = rtemp.bytes;
        m.stemp = stemp.p;
        m.stemp_bytes = stemp.bytes;
        m.S = S.as<float>();
        m.S2 = S2.as<float>();
        m.B = B.as<float>();
        m.delta = delta.as<float>();
        m.var = var.as<float>();
        m.D = D.as<uint32_t>();
        m.q = q.as<uint32_t>();
        m.maxbits = maxbits.as<uint32_t>();
        m.recv = recv.as<int32_t>();
        m.cdf = cdf.as<int64_t>();
        return m;
    }
    ~gsrad_mc() {
        for (DevBuf *b : {&cent, &gnrm, &L, &key, &ids, &skey, &members, &count, &goff, &rtemp, &stemp, &S, &S2, &B,
                          &delta, &var, &D, &q, &maxbits, &recv, &cdf, &err})
            b->release();
    }
};

namespace {

#define GS_TRY(expr)                          \
    do {                                      \
        gsrad_status _s = (expr);             \
        if (_s != GSRAD_OK) return _s;        \
    } while (0)

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline gsrad_status einval(const char *msg) {
    set_error("%s", msg);
    return GSRAD_EINVAL;
}

bool valid_K(int K) { return K == 1 || K == 4 || K == 9 || K == 16; }

std::atomic<uint64_t> g_build_gen{0};
std::atomic<uint64_t> g_fill_gen{0};

// A handle whose last (re)build or (re)fill failed part-way is left with
// n = 0 and refuses every later use until it is rebuilt.
gsrad_status usable(const gsrad_bvh *b, const char *fn) {
    if (b->n >= 1) return GSRAD_OK;
    set_error("%s: the BVH handle is unusable after a failed gsrad_build_bvh", fn);
    return GSRAD_ESTATE;
}

gsrad_status usable(const gsrad_ff *f, const char *fn) {
    if (f->n >= 1) return GSRAD_OK;
    set_error("%s: the F handle is unusable after a failed call that refilled it", fn);
    return GSRAD_ESTATE;
}

void invalidate(gsrad_ff *f) {
    f->fill_gen = 0;
    f->n = 0;
    f->nnz = 0;
    f->max_row = 0;
    f->has_t = false;
    f->has_order = false;
    f->has_records = false;
    f->has_dense = false;
    f->bvh = nullptr;
    f->bvh_gen = 0;
    f->center_bvh = nullptr;
    f->center_gen = 0;
}

__global__ void k_max_u32(const uint32_t *__restrict__ v, int64_t n, int *out) {
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (int)v[i]);
    atomicMax(out, m);
}

__global__ void k_row_len_from_ptr(const int64_t *__restrict__ rp, int64_t n, int *out) {
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (int)(rp[i + 1] - rp[i]));
    atomicMax(out, m);
}

gsrad_status ensure_transpose(gsrad_ff *ff, hipStream_t st) {
    if (ff->has_t) return GSRAD_OK;
    GS_TRY(ff->t_row_ptr.ensure((size_t)(ff->n + 1) * 8, "F^T row_ptr"));
    GS_TRY(ff->t_col.ensure((size_t)std::max<int64_t>(ff->nnz, 1) * 4, "F^T col"));
    GS_TRY(ff->t_val.ensure((size_t)std::max<int64_t>(ff->nnz, 1) * 4, "F^T val"));
    const size_t tb = transpose_temp_bytes(ff->n, ff->nnz);
    GS_TRY(ff->t_temp.ensure(tb, "transpose temp"));
    GS_TRY(csr_transpose(ff->csr(), ff->t_row_ptr.as<int64_t>(), ff->t_col.as<int32_t>(), ff->t_val.as<float>(),
                         ff->t_temp.p, tb, st));
    ff->has_t = true;
    // a large sort scratch (batches of many scenes) is not kept
    if (tb > (size_t(2) << 30)) {
        GS_TRY(check_hip(hipStreamSynchronize(st), "transpose sync"));
        ff->t_temp.release();
    }
    return GSRAD_OK;
}

}  // namespace

extern "C" {

const char *gsrad_version(void) { return "gsrad 0.1 (gfx950)"; }

const char *gsrad_last_error(void) { return g_err; }

gsrad_status gsrad_build_bvh(const gsrad_surfels *s, gsrad_bvh **bvh, void *stream) {
    if (!s || !bvh) return einval("gsrad_build_bvh: null argument");
    if (s->n < 1) return einval("gsrad_build_bvh: n must be >= 1");
    if (s->n >= (int64_t)1 << 31) return einval("gsrad_build_bvh: n must be < 2^31");
    const float *f[] = {s->px, s->py, s->pz, s->tux, s->tuy, s->tuz, s->tvx, s->tvy, s->tvz, s->nx, s->ny, s->nz,
                        s->su, s->sv, s->opacity};
    for (const float *p : f)
        if (!p) return einval("gsrad_build_bvh: a surfel field pointer is null");
    const bool created = *bvh == nullptr;
    gsrad_bvh *h = created ? new gsrad_bvh() : *bvh;
    const int64_t n = s->n;
    hipStream_t st = S(stream);
    h->n = 0;   // unusable until this build succeeds
    h->gen = 0;
    auto fail = [&](gsrad_status e) {
        if (created) delete h;
        return e;
    };
    gsrad_status e;
#define ENS(buf, bytes, what)                                  \
    if ((e = h->buf.ensure((size_t)(bytes), what)) != GSRAD_OK) return fail(e);
    ENS(rec, n * sizeof(SurfRec), "surfel records");
    ENS(nodes, std::max<int64_t>(n - 1, 1) * sizeof(Node), "bvh nodes");
    ENS(leafbox, n * 6 * sizeof(float), "leaf boxes");
    ENS(leaf_parent, n * 4, "leaf parents");
    ENS(inv, n * 4, "inverse order");
    ENS(cst, n * 4, "opacity constants");
    ENS(opc, n * 4, "clamped opacity");
    ENS(opraw, n * 4, "opacity");
    ENS(area, n * 8, "areas");
    ENS(dado, n * 4, "area derivatives");
    ENS(bounds, 64, "bounds");
    ENS(height, 64, "height");
    ENS(temp, bvh_temp_bytes(n), "bvh temp");
#undef ENS
    h->stream = st;
    BvhBuffers &B = h->B;
    B.rec = h->rec.as<SurfRec>();
    B.nodes = h->nodes.as<Node>();
    B.leafbox = h->leafbox.as<float>();
    B.leaf_parent = h->leaf_parent.as<int32_t>();
    B.inv = h->inv.as<int32_t>();
    B.cst = h->cst.as<float>();
    B.opc = h->opc.as<float>();
    B.opraw = h->opraw.as<float>();
    B.area = h->area.as<double>();
    B.dado = h->dado.as<float>();
    B.bounds = h->bounds.as<float>();
    B.height = h->height.as<int>();
    B.temp = h->temp.p;
    B.temp_bytes = h->temp.bytes;
    if ((e = check_hip(hipMemsetAsync(B.height, 0, sizeof(int), st), "bvh height")) != GSRAD_OK) return fail(e);
    {
        ProfScope ps("bvh_build", st);
        if ((e = bvh_build(*s, B, st)) != GSRAD_OK) return fail(e);
    }
    h->n = n;
    h->gen = ++g_build_gen;
    *bvh = h;
    return GSRAD_OK;
}

gsrad_status gsrad_bvh_info(const gsrad_bvh *bvh, int64_t *n, float *t_eps_default) {
    if (!bvh) return einval("gsrad_bvh_info: null handle");
    if (n) *n = bvh->n;
    if (t_eps_default) {
        float b[8];
        GS_TRY(check_hip(hipStreamSynchronize(bvh->stream), "bvh info sync"));
        GS_TRY(check_hip(hipMemcpy(b, bvh->B.bounds, sizeof(b), hipMemcpyDeviceToHost), "bvh info copy"));
        *t_eps_default = b[6];
    }
    return GSRAD_OK;
}

gsrad_status gsrad_bvh_height(const gsrad_bvh *bvh, int32_t *height) {
    if (!bvh || !height) return einval("gsrad_bvh_height: null argument");
    GS_TRY(usable(bvh, "gsrad_bvh_height"));
    GS_TRY(check_hip(hipStreamSynchronize(bvh->stream), "bvh height sync"));
    return check_hip(hipMemcpy(height, bvh->B.height, sizeof(int32_t), hipMemcpyDeviceToHost), "bvh height copy");
}

gsrad_status gsrad_effective_area(const gsrad_bvh *bvh, double *area_out, void *stream) {
    if (!bvh || !area_out) return einval("gsrad_effective_area: null argument");
    GS_TRY(usable(bvh, "gsrad_effective_area"));
    return check_hip(hipMemcpyAsync(area_out, bvh->B.area, (size_t)bvh->n * 8, hipMemcpyDeviceToDevice, S(stream)),
                     "effective area copy");
}

gsrad_status gsrad_reflectance(const gsrad_bvh *bvh, const float *albedo, float *rho_out, void *stream) {
    if (!bvh || !albedo || !rho_out) return einval("gsrad_reflectance: null argument");
    GS_TRY(usable(bvh, "gsrad_reflectance"));
    return launch_reflectance(bvh->dev(), albedo, rho_out, S(stream));
}

gsrad_status gsrad_form_factors(const gsrad_bvh *bvh, const gsrad_ff_params *p, gsrad_ff **ff, void *stream) {
    if (!bvh || !p || !ff) return einval("gsrad_form_factors: null argument");
    if (p->rays_per_surfel < 1 || p->rays_per_surfel > (1 << 20))
        return einval("gsrad_form_factors: rays_per_surfel must be in [1, 2^20]");
    if (p->topk < 0 || p->topk > (1 << kLog2Table)) return einval("gsrad_form_factors: topk must be in [0, 4096]");
    if (!(p->t_min >= 0.0f) || !(p->t_min <= 1.0f)) return einval("gsrad_form_factors: t_min must be in [0, 1]");
    if (!std::isfinite(p->t_eps)) return einval("gsrad_form_factors: t_eps must be finite");
    GS_TRY(usable(bvh, "gsrad_form_factors"));
    const bool created = *ff == nullptr;
    gsrad_ff *h = created ? new gsrad_ff() : *ff;
    // a reused handle is unusable until this call succeeds (its buffers are
    // overwritten or reallocated on the way)
    const int prev_rec_cap = h->rec_cap, prev_log2h = h->agg_log2h, prev_deep = h->deep_stack;
    invalidate(h);
    auto fail = [&](gsrad_status e) {
        if (created) delete h;
        return e;
    };
    hipStream_t st = S(stream);
    const int64_t n = bvh->n;
    const int R = p->rays_per_surfel;
    // a handle traced before starts from the record slots, stack and
    // aggregation table its last call needed (the rows do not depend on them)
    int rcap = created ? kRecCap : std::max(kRecCap, prev_rec_cap);
    const int log2h = created ? kLog2Table : std::max(kLog2Table, prev_log2h);
    int deep = created ? 0 : prev_deep;
    const int64_t cap_row = p->topk > 0 ? p->topk : (1 << kLog2TableMax);
    gsrad_status e;
    float t_eps = p->t_eps;
    if (!(t_eps > 0.0f)) {
        float b[8];
        if ((e = check_hip(hipStreamSynchronize(st), "ff sync")) != GSRAD_OK) return fail(e);
        if ((e = check_hip(hipMemcpy(b, bvh->B.bounds, sizeof(b), hipMemcpyDeviceToHost), "ff t_eps")) != GSRAD_OK)
            return fail(e);
        t_eps = b[6];
    }
    int flags[4];
    int64_t nnz = 0;
    bool keep = false;
    // Records are kept for the backward when the slab fits in half of the
    // device memory that is free now (counting the slab this handle holds).
    size_t mem_free = 0, mem_total = 0;
    if ((e = check_hip(hipMemGetInfo(&mem_free, &mem_total), "ff memory info")) != GSRAD_OK) return fail(e);
    const size_t record_budget = (mem_free + h->recs.bytes) / 2;
    for (int attempt = 0;; ++attempt) {
        // Records of every receiver are kept for the backward when they fit;
        // otherwise receivers are traced in chunks whose records are only
        // used to build F (the backward then recomputes the rays).
        const size_t per_recv = (size_t)R * rcap * sizeof(uint2);
        keep = (size_t)n * per_recv <= record_budget && !(p->flags & GSRAD_FF_NO_RECORDS);
        const int64_t chunk =
            keep ? n : std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(kChunkRecordBudget / per_recv)));
#define ENS(buf, bytes, what) \
    if ((e = h->buf.ensure((size_t)(bytes), what)) != GSRAD_OK) return fail(e);
        ENS(recs, (size_t)chunk * per_recv, "hit records");
        ENS(rcnt, (size_t)chunk * R * 4, "hit record counts");
        ENS(ell_col, n * cap_row * 4, "row staging");
        ENS(ell_val, n * cap_row * 4, "row staging");
        ENS(row_len, n * 4, "row lengths");
        ENS(redo, ((size_t)chunk + 2) * 4, "aggregation redo list");
        ENS(err, 128, "error flags");
        ENS(row_ptr, (n + 1) * 8, "row_ptr");
        ENS(scan_temp, scan_temp_bytes(n), "scan temp");
        ENS(pools, ff_pool_list_bytes(chunk, R), "ray pools");
#undef ENS
        int *err = h->err.as<int>();
        if ((e = check_hip(hipMemsetAsync(err, 0, 64, st), "ff flags")) != GSRAD_OK) return fail(e);
        const BvhDev bv = bvh->dev();
        for (int64_t s0 = 0; s0 < n; s0 += chunk) {
            const int64_t cnt = std::min(chunk, n - s0);
            {
                ProfScope ps("ray_pools", st);
                if ((e = launch_ray_pools(bv, R, p->seed, s0, cnt, keep ? 1 : 0, h->rcnt.as<uint32_t>(), h->pools.p,
                                          st)) != GSRAD_OK)
                    return fail(e);
            }
            {
                ProfScope ps("ff_trace", st);
                if ((e = launch_ff_trace(bv, R, t_eps, p->t_min, s0, cnt, keep ? 1 : 0, h->recs.as<uint2>(),
                                         h->rcnt.as<uint32_t>(), rcap, deep, h->pools.p, err, st)) != GSRAD_OK)
                    return fail(e);
            }
            ProfScope ps("ff_aggregate", st);
            if ((e = launch_ff_aggregate(bv, h->recs.as<uint2>(), h->rcnt.as<uint32_t>(), rcap, s0, cnt, keep ? 1 : 0,
                                         R, p->topk, log2h, kLog2TableMax, h->redo.as<int32_t>() + 2,
                                         h->redo.as<uint32_t>(), cap_row, h->ell_col.as<int32_t>(),
                                         h->ell_val.as<float>(), h->row_len.as<uint32_t>(), err, st)) != GSRAD_OK)
                return fail(e);
        }
        hipLaunchKernelGGL(k_max_u32, dim3(64), dim3(256), 0, st, h->row_len.as<uint32_t>(), n, err + 1);
        if ((e = exclusive_scan_u32_i64(h->row_len.as<uint32_t>(), h->row_ptr.as<int64_t>(), n, h->scan_temp.p,
                                        h->scan_temp.bytes, st)) != GSRAD_OK)
            return fail(e);
        if ((e = check_hip(hipMemcpyAsync(flags, err, sizeof(flags), hipMemcpyDeviceToHost, st), "ff flags copy")) !=
            GSRAD_OK)
            return fail(e);
        if ((e = check_hip(hipMemcpyAsync(&nnz, h->row_ptr.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, st),
                           "ff nnz copy")) != GSRAD_OK)
            return fail(e);
        if ((e = check_hip(hipStreamSynchronize(st), "ff sync")) != GSRAD_OK) return fail(e);
        // a tree deeper than the shallow traversal stack: trace again with
        // the deep one
        if ((flags[0] & kErrStack) && !deep) {
            deep = 1;
            continue;
        }
        // a ray composited more hits than its record slots: the rows are
        // incomplete, so run again with twice the slots
        if ((flags[0] & kErrRecords) && attempt < 4) {
            while (rcap < flags[3]) rcap *= 2;
            continue;
        }
        break;
    }
    if (flags[0] != 0) {
        set_error("gsrad_form_factors: overflow flags 0x%x (1 traversal stack, 4 aggregation table of %d, 8 row, "
                  "16 hit records of %d per ray)", flags[0], 1 << kLog2TableMax, rcap);
        if (created) delete h;
        return GSRAD_EOVERFLOW;
    }
    if ((e = h->col.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "F col")) != GSRAD_OK) return fail(e);
    if ((e = h->val.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "F val")) != GSRAD_OK) return fail(e);
    ProfScope ps_csr("ff_csr", st);
    if ((e = launch_ell_to_csr(h->ell_col.as<int32_t>(), h->ell_val.as<float>(), cap_row, h->row_ptr.as<int64_t>(), n,
                               h->col.as<int32_t>(), h->val.as<float>(), st)) != GSRAD_OK)
        return fail(e);
    if ((e = h->row_order.ensure((size_t)n * 4, "row order")) != GSRAD_OK) return fail(e);
    if ((e = launch_sorted_order(bvh->dev(), h->row_order.as<int32_t>(), st)) != GSRAD_OK) return fail(e);
    h->n = n;
    h->nnz = nnz;
    h->fill_gen = ++g_fill_gen;
    h->max_row = flags[1];
    h->has_t = false;
    h->has_order = true;
    h->has_dense = false;
    h->bvh = bvh;
    h->bvh_gen = bvh->gen;
    h->R = R;
    h->topk = p->topk;
    h->seed = p->seed;
    h->t_eps = t_eps;
    h->t_min = p->t_min;
    h->has_records = keep;
    h->rec_cap = rcap;
    h->deep_stack = deep;
    // most rows needed the largest table: start there next time
    h->agg_log2h = flags[2] > n / 4 ? kLog2TableMax : log2h;
    if (p->flags & GSRAD_FF_COMPACT) {
        // the stream must be done with the scratch before it is freed
        if ((e = check_hip(hipStreamSynchronize(st), "ff compact sync")) != GSRAD_OK) return fail(e);
        if (!keep) {
            h->recs.release();
            h->rcnt.release();
        }
        for (DevBuf *b : {&h->ell_col, &h->ell_val, &h->row_len, &h->redo, &h->scan_temp}) b->release();
    }
    *ff = h;
    return GSRAD_OK;
}

gsrad_status gsrad_ff_info(const gsrad_ff *ff, int64_t *n, int64_t *nnz) {
    if (!ff) return einval("gsrad_ff_info: null handle");
    if (n) *n = ff->n;
    if (nnz) *nnz = ff->nnz;
    return GSRAD_OK;
}

gsrad_status gsrad_ff_view(const gsrad_ff *ff, const int64_t **row_ptr, const int32_t **col, const float **val) {
    if (!ff) return einval("gsrad_ff_view: null handle");
    if (row_ptr) *row_ptr = ff->row_ptr.as<int64_t>();
    if (col) *col = ff->col.as<int32_t>();
    if (val) *val = ff->val.as<float>();
    return GSRAD_OK;
}

gsrad_status gsrad_ff_copy(const gsrad_ff *ff, int64_t *row_ptr, int32_t *col, float *val, void *stream) {
    if (!ff || !row_ptr || (ff->nnz > 0 && (!col || !val))) return einval("gsrad_ff_copy: null argument");
    GS_TRY(usable(ff, "gsrad_ff_copy"));
    hipStream_t st = S(stream);
    GS_TRY(check_hip(hipMemcpyAsync(row_ptr, ff->row_ptr.p, (size_t)(ff->n + 1) * 8, hipMemcpyDeviceToDevice, st),
                     "ff copy row_ptr"));
    if (ff->nnz > 0) {
        GS_TRY(check_hip(hipMemcpyAsync(col, ff->col.p, (size_t)ff->nnz * 4, hipMemcpyDeviceToDevice, st), "ff copy col"));
        GS_TRY(check_hip(hipMemcpyAsync(val, ff->val.p, (size_t)ff->nnz * 4, hipMemcpyDeviceToDevice, st), "ff copy val"));
    }
    return GSRAD_OK;
}

gsrad_status gsrad_ff_from_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const float *val,
                               gsrad_ff **ff, void *stream) {
    if (!ff || !row_ptr || (nnz > 0 && (!col || !val))) return einval("gsrad_ff_from_csr: null argument");
    if (n < 1 || nnz < 0 || nnz >= ((int64_t)1 << 32)) return einval("gsrad_ff_from_csr: bad size");
    const bool created = *ff == nullptr;
    gsrad_ff *h = created ? new gsrad_ff() : *ff;
    invalidate(h);
    auto fail = [&](gsrad_status e) {
        if (created) delete h;
        return e;
    };
    hipStream_t st = S(stream);
    gsrad_status e;
    if ((e = h->row_ptr.ensure((size_t)(n + 1) * 8, "row_ptr")) != GSRAD_OK) return fail(e);
    if ((e = h->col.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "col")) != GSRAD_OK) return fail(e);
    if ((e = h->val.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "val")) != GSRAD_OK) return fail(e);
    if ((e = h->err.ensure(128, "flags")) != GSRAD_OK) return fail(e);
    if ((e = check_hip(hipMemcpyAsync(h->row_ptr.p, row_ptr, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, st),
                       "copy row_ptr")) != GSRAD_OK)
        return fail(e);
    if (nnz > 0) {
        if ((e = check_hip(hipMemcpyAsync(h->col.p, col, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st), "copy col")) !=
            GSRAD_OK)
            return fail(e);
        if ((e = check_hip(hipMemcpyAsync(h->val.p, val, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st), "copy val")) !=
            GSRAD_OK)
            return fail(e);
    }
    int mx = 0;
    if ((e = check_hip(hipMemsetAsync(h->err.p, 0, 64, st), "flags")) != GSRAD_OK) return fail(e);
    hipLaunchKernelGGL(k_row_len_from_ptr, dim3(64), dim3(256), 0, st, h->row_ptr.as<int64_t>(), n, h->err.as<int>());
    if ((e = check_hip(hipMemcpyAsync(&mx, h->err.p, 4, hipMemcpyDeviceToHost, st), "max row")) != GSRAD_OK)
        return fail(e);
    if ((e = check_hip(hipStreamSynchronize(st), "ff_from_csr sync")) != GSRAD_OK) return fail(e);
    h->n = n;
    h->nnz = nnz;
    h->fill_gen = ++g_fill_gen;
    h->max_row = mx;
    h->has_t = false;
    h->has_order = false;
    h->has_dense = false;
    h->bvh = nullptr;
    *ff = h;
    return GSRAD_OK;
}

gsrad_status gsrad_ff_dense(gsrad_ff *ff, void *stream) {
    if (!ff) return einval("gsrad_ff_dense: null handle");
    GS_TRY(usable(ff, "gsrad_ff_dense"));
    if (ff->n < 1) return einval("gsrad_ff_dense: empty operator");
    hipStream_t st = S(stream);
    const int64_t Np = dense_pad(ff->n);
    const size_t bytes = (size_t)Np * (size_t)Np * sizeof(__bf16);
    ff->has_dense = false;
    for (DevBuf *b : {&ff->d_hi, &ff->d_lo, &ff->dt_hi, &ff->dt_lo}) {
        GS_TRY(b->ensure(bytes, "dense BF16 operator"));
        GS_TRY(check_hip(hipMemsetAsync(b->p, 0, bytes, st), "dense operator zero"));
    }
    ProfScope ps("dense_scatter", st);
    GS_TRY(launch_dense_scatter(ff->csr(), Np, ff->d_hi.as<__bf16>(), ff->d_lo.as<__bf16>(), ff->dt_hi.as<__bf16>(),
                                ff->dt_lo.as<__bf16>(), st));
    ff->Np = Np;
    ff->has_dense = true;
    return GSRAD_OK;
}

gsrad_status gsrad_direct_light(const gsrad_bvh *bvh, const float *albedo, const float *light_pos,
                                const float *light_I, int32_t n_lights, int32_t K, float *E_out, void *stream) {
    if (!bvh || !albedo || !light_pos || !light_I || !E_out) return einval("gsrad_direct_light: null argument");
    GS_TRY(usable(bvh, "gsrad_direct_light"));
    if (n_lights < 1) return einval("gsrad_direct_light: n_lights must be >= 1");
    if (!valid_K(K)) return einval("gsrad_direct_light: K must be 1, 4, 9 or 16");
    hipStream_t st = S(stream);
    gsrad_bvh *h = const_cast<gsrad_bvh *>(bvh);
    GS_TRY(h->height.ensure(64, "flags"));
    ProfScope ps("direct_light", st);
    return launch_direct(bvh->dev(), albedo, light_pos, light_I, n_lights, K, E_out, h->height.as<int>() + 4, st);
}

namespace {

// Forward bounces on the dense BF16 copies: n_bounces - 1 BF16 products,
// then the correction sweep (split operands).  The transposed BF16 operand
// of B^(k) alternates between two buffers; the low part is made only for
// the input of the correction sweep.
gsrad_status dense_solve(const gsrad_ff *ff, const float *rho, const float *E, int C, int nb, float *B_out,
                         gsrad_tape *tp, hipStream_t st) {
    const int64_t n = ff->n, Np = ff->Np, Cp = dense_pad(C);
    const size_t xbytes = (size_t)Cp * Np * sizeof(__bf16);
    gsrad_ff *m = const_cast<gsrad_ff *>(ff);
    // the operand buffers are scratch of the handle (like the FP32 ping-pong)
    DevBuf &xa = m->xa, &xb = m->xb, &xl = m->xl;
    for (DevBuf *b : {&xa, &xb, &xl}) {
        GS_TRY(b->ensure(xbytes, "BF16 bounce operand"));
        GS_TRY(check_hip(hipMemsetAsync(b->p, 0, xbytes, st), "operand zero"));
    }
    int64_t Kp = 0;
    if (tp) {
        Kp = ((int64_t)nb * C + 63) / 64 * 64;
        GS_TRY(tp->Q.ensure((size_t)nb * n * C * sizeof(float), "F B tape"));
        for (DevBuf *b : {&tp->bb, &tp->bb_lo}) {
            GS_TRY(b->ensure((size_t)Np * Kp * sizeof(__bf16), "BF16 B tape"));
            GS_TRY(check_hip(hipMemsetAsync(b->p, 0, (size_t)Np * Kp * sizeof(__bf16), st), "B tape zero"));
        }
        GS_TRY(launch_to_bf16_rows(E, nullptr, n, C, tp->bb.as<__bf16>(), tp->bb_lo.as<__bf16>(), Kp, 0, st));
        tp->Kp = Kp;
    }
    GS_TRY(launch_to_bf16_t(E, nullptr, n, C, xa.as<__bf16>(), nb == 1 ? xl.as<__bf16>() : nullptr, Np, st));
    for (int k = 0; k < nb; ++k) {
        DenseBounce a;
        a.f_hi = ff->d_hi.as<__bf16>();
        a.f_lo = ff->d_lo.as<__bf16>();
        a.ld = Np;
        a.x_hi = (k & 1 ? xb : xa).as<__bf16>();
        a.x_lo = xl.as<__bf16>();
        a.ldx = Np;
        a.split = k == nb - 1;
        a.E = E;
        a.rho = rho;
        a.n = n;
        a.C = C;
        a.Bout = k == nb - 1 ? B_out : nullptr;
        a.Q = tp ? tp->Q.as<float>() + (size_t)k * n * C : nullptr;
        a.xt_hi = k < nb - 1 ? (k & 1 ? xa : xb).as<__bf16>() : nullptr;
        a.xt_lo = k == nb - 2 ? xl.as<__bf16>() : nullptr;
        a.bb = tp && k + 1 < nb ? tp->bb.as<__bf16>() : nullptr;
        a.bb_lo = tp && k + 1 < nb ? tp->bb_lo.as<__bf16>() : nullptr;
        a.ldbb = Kp;
        a.boff = (int64_t)(k + 1) * C;
        ProfScope ps(a.split ? "dense_bounce_fix" : "dense_bounce", st);
        GS_TRY(launch_dense_bounce(a, st));
    }
    return GSRAD_OK;
}

// Adjoint of dense_solve: the first step (k = nb-1) on the split F^T, the
// others BF16; dL/drho from the tape's F B^(k); the dense dL/dF product
// when grad_F is wanted.
gsrad_status dense_backward(const gsrad_ff *ff, gsrad_tape *tp, const float *rho, const float *grad_B,
                            float *grad_E, float *grad_rho, float *grad_F, hipStream_t st) {
    const int64_t n = ff->n, Np = ff->Np;
    const int C = tp->C, nb = tp->nb;
    const int64_t Cp = dense_pad(C), Kp = tp->Kp;
    const size_t xbytes = (size_t)Cp * Np * sizeof(__bf16);
    const size_t row_bytes = (size_t)n * C * sizeof(float);
    gsrad_ff *m = const_cast<gsrad_ff *>(ff);
    for (DevBuf *b : {&m->xa, &m->xb, &m->xl}) {
        GS_TRY(b->ensure(xbytes, "BF16 adjoint operand"));
        GS_TRY(check_hip(hipMemsetAsync(b->p, 0, xbytes, st), "operand zero"));
    }
    GS_TRY(tp->lam_a.ensure(row_bytes, "adjoint iterate"));
    GS_TRY(tp->lam_b.ensure(row_bytes, "adjoint iterate"));
    const bool want_F = grad_F != nullptr;
    if (want_F) {
        for (DevBuf *b : {&tp->pb, &tp->pb_lo}) {
            GS_TRY(b->ensure((size_t)Np * Kp * sizeof(__bf16), "BF16 adjoint tape"));
            GS_TRY(check_hip(hipMemsetAsync(b->p, 0, (size_t)Np * Kp * sizeof(__bf16), st), "adjoint tape zero"));
        }
        GS_TRY(launch_to_bf16_rows(grad_B, rho, n, C, tp->pb.as<__bf16>(), tp->pb_lo.as<__bf16>(), Kp,
                                   (int64_t)(nb - 1) * C, st));
    }
    float *gr = grad_rho;
    if (gr) {
        GS_TRY(check_hip(hipMemsetAsync(gr, 0, (size_t)n * 12, st), "grad_rho zero"));
        GS_TRY(launch_grad_rho_acc(grad_B, tp->Q.as<float>() + (size_t)(nb - 1) * n * C, n, C, gr, st));
    }
    GS_TRY(launch_to_bf16_t(grad_B, rho, n, C, m->xa.as<__bf16>(), m->xl.as<__bf16>(), Np, st));
    for (int k = nb - 1, s = 0; k >= 0; --k, ++s) {
        DenseAdjoint a;
        a.ft_hi = ff->dt_hi.as<__bf16>();
        a.ft_lo = ff->dt_lo.as<__bf16>();
        a.ld = Np;
        a.y_hi = (s & 1 ? m->xb : m->xa).as<__bf16>();
        a.y_lo = m->xl.as<__bf16>();
        a.ldx = Np;
        a.split = k == nb - 1;
        a.rho = rho;
        a.n = n;
        a.C = C;
        a.lam = (s & 1 ? tp->lam_b : tp->lam_a).as<float>();
        a.gE = grad_E;
        a.yt_hi = k >= 1 ? (s & 1 ? m->xa : m->xb).as<__bf16>() : nullptr;
        a.p = want_F && k >= 1 ? tp->pb.as<__bf16>() : nullptr;
        a.p_lo = want_F && k >= 1 ? tp->pb_lo.as<__bf16>() : nullptr;
        a.ldp = Kp;
        a.poff = (int64_t)(k - 1) * C;
        {
            ProfScope ps(a.split ? "dense_adjoint_fix" : "dense_adjoint", st);
            GS_TRY(launch_dense_adjoint(a, st));
        }
        if (gr && k >= 1) GS_TRY(launch_grad_rho_acc(a.lam, tp->Q.as<float>() + (size_t)(k - 1) * n * C, n, C, gr, st));
    }
    tp->has_G = false;
    if (want_F) {
        GS_TRY(tp->G.ensure((size_t)n * n * sizeof(float), "dense dL/dF"));
        {
            ProfScope ps("dense_grad_F", st);
            GS_TRY(launch_dense_grad_F(tp->pb.as<__bf16>(), tp->pb_lo.as<__bf16>(), tp->bb.as<__bf16>(),
                                       tp->bb_lo.as<__bf16>(), Kp, Kp, n, Np, tp->G.as<float>(), n, st));
        }
        GS_TRY(launch_gather_csr(ff->csr(), tp->G.as<float>(), n, grad_F, st));
        tp->has_G = true;
    }
    return GSRAD_OK;
}

}  // namespace

gsrad_status gsrad_tape_grad_F_dense(const gsrad_tape *tape, float *grad_F_out, void *stream) {
    if (!tape || !grad_F_out) return einval("gsrad_tape_grad_F_dense: null argument");
    if (!tape->has_G) {
        set_error("gsrad_tape_grad_F_dense: no dense dL/dF on this tape");
        return GSRAD_ESTATE;
    }
    return check_hip(hipMemcpyAsync(grad_F_out, tape->G.p, (size_t)tape->n * tape->n * sizeof(float),
                                    hipMemcpyDeviceToDevice, S(stream)),
                     "dense dL/dF copy");
}

gsrad_status gsrad_transport_solve(const gsrad_ff *ff, const float *rho, const float *E, int32_t n_lights, int32_t K,
                                   int32_t n_bounces, int32_t precision, float *B_out, gsrad_tape **tape,
                                   void *stream) {
    if (!ff || !rho || !E || !B_out) return einval("gsrad_transport_solve: null argument");
    GS_TRY(usable(ff, "gsrad_transport_solve"));
    if (n_lights < 1) return einval("gsrad_transport_solve: n_lights must be >= 1");
    if (!valid_K(K)) return einval("gsrad_transport_solve: K must be 1, 4, 9 or 16");
    if (n_bounces < 0 || n_bounces > 4096) return einval("gsrad_transport_solve: n_bounces must be in [0, 4096]");
    if (precision != GSRAD_FP32 && precision != GSRAD_BF16)
        return einval("gsrad_transport_solve: precision must be GSRAD_FP32 or GSRAD_BF16");
    if (precision == GSRAD_BF16 && !ff->has_dense)
        return einval("gsrad_transport_solve: GSRAD_BF16 needs the dense copies of gsrad_ff_dense");
    hipStream_t st = S(stream);
    const int C = n_lights * K * 3;
    const int64_t n = ff->n;
    const size_t row_bytes = (size_t)n * C * sizeof(float);
    gsrad_tape *tp = nullptr;
    bool created = false;
    if (tape) {
        created = *tape == nullptr;
        tp = created ? new gsrad_tape() : *tape;
        tp->ff = nullptr;   // unusable unless this solve succeeds
        tp->has_G = false;
    }
    auto fail = [&](gsrad_status e) {
        if (created) delete tp;
        return e;
    };
    gsrad_status e;
    const Csr F = ff->csr();
    if (precision == GSRAD_BF16 && n_bounces > 0) {
        if ((e = dense_solve(ff, rho, E, C, n_bounces, B_out, tp, st)) != GSRAD_OK) return fail(e);
    } else if (n_bounces == 0) {
        if ((e = check_hip(hipMemcpyAsync(B_out, E, row_bytes, hipMemcpyDeviceToDevice, st), "solve copy")) !=
            GSRAD_OK)
            return fail(e);
    } else {
        float *slots = nullptr;
        if (tp) {
            if ((e = tp->B.ensure(row_bytes * n_bounces, "forward tape")) != GSRAD_OK) return fail(e);
            slots = tp->B.as<float>();
            if ((e = check_hip(hipMemcpyAsync(slots, E, row_bytes, hipMemcpyDeviceToDevice, st), "tape copy")) !=
                GSRAD_OK)
                return fail(e);
        } else if (n_bounces > 1) {
            gsrad_ff *m = const_cast<gsrad_ff *>(ff);
            if ((e = m->slab.ensure(std::max(m->slab.bytes, row_bytes * 2), "ping-pong")) != GSRAD_OK) return fail(e);
        }
        const float *src = E;
        for (int k = 0; k < n_bounces; ++k) {
            float *dst;
            if (k == n_bounces - 1) dst = B_out;
            else if (tp) dst = slots + (size_t)(k + 1) * n * C;
            else dst = const_cast<gsrad_ff *>(ff)->slab.as<float>() + (size_t)(k & 1) * n * C;
            ProfScope ps("bounce", st);
            if ((e = launch_bounce(F, C, src, E, rho, dst, st)) != GSRAD_OK) return fail(e);
            src = dst;
        }
    }
    if (tp) {
        tp->n = n;
        tp->C = C;
        tp->nb = n_bounces;
        tp->Lt = n_lights;
        tp->K = K;
        tp->precision = precision;
        tp->has_G = false;
        tp->ff = ff;
        tp->ff_gen = ff->fill_gen;
        tp->bvh = nullptr;
        tp->bvh_gen = 0;
        *tape = tp;
    }
    return GSRAD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free bounce iterations: the ping-pong iterates live in a
// fixed device array of this translation unit (one per GPU, held until the
// process ends).  Its device address is looked up once per device; host
// code only ever passes that address, never the array's name.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchMaxDevices] = {};

gsrad_status scratch_of_current_device(void **out) {
    int dev = -1;
    GS_TRY(check_hip(hipGetDevice(&dev), "scratch: current device"));
    if (dev < 0 || dev >= kScratchMaxDevices) {
        set_error("scratch: device %d out of range", dev);
        return GSRAD_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        GS_TRY(check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch: symbol address"));
        if (!p) {
            set_error("scratch: null symbol address on device %d", dev);
            return GSRAD_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GSRAD_OK;
}

}  // namespace

extern "C" {

gsrad_status gsrad_transport_solve_noalloc(const gsrad_ff *ff, const float *rho, const float *E, int32_t n_lights,
                                           int32_t K, int32_t n_bounces, float *B_out, void *stream) {
    if (!ff || !rho || !E || !B_out) return einval("gsrad_transport_solve_noalloc: null argument");
    GS_TRY(usable(ff, "gsrad_transport_solve_noalloc"));
    if (n_lights < 1) return einval("gsrad_transport_solve_noalloc: n_lights must be >= 1");
    if (!valid_K(K)) return einval("gsrad_transport_solve_noalloc: K must be 1, 4, 9 or 16");
    if (n_bounces < 0 || n_bounces > 4096)
        return einval("gsrad_transport_solve_noalloc: n_bounces must be in [0, 4096]");
    hipStream_t st = S(stream);
    const int C = n_lights * K * 3;
    const int64_t n = ff->n;
    const size_t row_bytes = (size_t)n * C * sizeof(float);
    if (n_bounces == 0)
        return check_hip(hipMemcpyAsync(B_out, E, row_bytes, hipMemcpyDeviceToDevice, st), "noalloc solve copy");
    float *slots = nullptr;
    if (n_bounces > 1) {
        if (2 * row_bytes > kScratchBytes) {
            set_error("gsrad_transport_solve_noalloc: two iterates of %lld x %d values need %zu bytes, more than the "
                      "%zu-byte scratch array", (long long)n, C, 2 * row_bytes, kScratchBytes);
            return GSRAD_EINVAL;
        }
        void *p = nullptr;
        GS_TRY(scratch_of_current_device(&p));
        slots = static_cast<float *>(p);
    }
    const Csr F = ff->csr();
    const float *src = E;
    for (int k = 0; k < n_bounces; ++k) {
        float *dst = k == n_bounces - 1 ? B_out : slots + (size_t)(k & 1) * n * C;
        GS_TRY(launch_bounce(F, C, src, E, rho, dst, st));
        src = dst;
    }
    return GSRAD_OK;
}

gsrad_status gsrad_transport_backward(const gsrad_ff *ff, const gsrad_tape *tape, const float *rho,
                                      const float *grad_B, float *grad_E, float *grad_rho, float *grad_F,
                                      void *stream) {
    if (!ff || !tape || !rho || !grad_B || !grad_E) return einval("gsrad_transport_backward: null argument");
    GS_TRY(usable(ff, "gsrad_transport_backward"));
    if (tape->ff != ff || tape->ff_gen != ff->fill_gen || tape->n != ff->n)
        return einval("gsrad_transport_backward: tape does not belong to this F as it is now");
    if (tape->precision == kTapeSH)
        return einval("gsrad_transport_backward: the tape is from gsrad_transport_solve_sh (use gsrad_transport_backward_sh)");
    hipStream_t st = S(stream);
    gsrad_ff *f = const_cast<gsrad_ff *>(ff);
    gsrad_tape *tp = const_cast<gsrad_tape *>(tape);
    const int64_t n = ff->n;
    const int C = tape->C, nb = tape->nb;
    const size_t row_bytes = (size_t)n * C * sizeof(float);
    GS_TRY(check_hip(hipMemcpyAsync(grad_E, grad_B, row_bytes, hipMemcpyDeviceToDevice, st), "grad_E init"));
    if (nb == 0) {
        if (grad_rho) GS_TRY(check_hip(hipMemsetAsync(grad_rho, 0, (size_t)n * 12, st), "grad_rho zero"));
        if (grad_F && ff->nnz > 0)
            GS_TRY(check_hip(hipMemsetAsync(grad_F, 0, (size_t)ff->nnz * 4, st), "grad_F zero"));
        return GSRAD_OK;
    }
    if (tape->precision == GSRAD_BF16) {
        if (!ff->has_dense) return einval("gsrad_transport_backward: the dense copies of F are gone");
        return dense_backward(ff, tp, rho, grad_B, grad_E, grad_rho, grad_F, st);
    }
    {
        ProfScope ps("transpose", st);
        GS_TRY(ensure_transpose(f, st));
    }
    GS_TRY(tp->L.ensure(row_bytes * nb, "adjoint tape"));
    GS_TRY(tp->lam0.ensure(row_bytes, "adjoint scratch"));
    float *L = tp->L.as<float>();
    GS_TRY(check_hip(hipMemcpyAsync(L + (size_t)(nb - 1) * n * C, grad_B, row_bytes, hipMemcpyDeviceToDevice, st),
                     "adjoint seed"));
    const Csr FT = f->csr_t();
    for (int k = nb - 1; k >= 0; --k) {
        const float *lam_in = L + (size_t)k * n * C;   // lambda^(k+1)
        float *lam_out = k >= 1 ? L + (size_t)(k - 1) * n * C : tp->lam0.as<float>();
        ProfScope ps("adjoint", st);
        GS_TRY(launch_adjoint(FT, C, lam_in, rho, lam_out, grad_E, st));
    }
    ProfScope ps("sddmm", st);
    if (grad_F || grad_rho) GS_TRY(launch_sddmm(ff->csr(), C, nb, tp->B.as<float>(), L, rho, grad_F, grad_rho, st));
    return GSRAD_OK;
}

// ---------------------------------------------------------------------------
// directional (spherical-harmonic) transfer with the diffuse + Phong BRDF
// ---------------------------------------------------------------------------
gsrad_status gsrad_brdf_reflectance(const gsrad_bvh *bvh, const float *k, const float *albedo_d,
                                    const float *albedo_s, const float *shininess, int32_t K, float *R_out,
                                    void *stream) {
    if (!bvh || !k || !albedo_d || !albedo_s || !shininess || !R_out)
        return einval("gsrad_brdf_reflectance: null argument");
    GS_TRY(usable(bvh, "gsrad_brdf_reflectance"));
    if (!valid_K(K)) return einval("gsrad_brdf_reflectance: K must be 1, 4, 9 or 16");
    return launch_brdf_reflectance(bvh->dev(), k, albedo_d, albedo_s, shininess, K, R_out, S(stream));
}

gsrad_status gsrad_brdf_backward(const gsrad_bvh *bvh, const float *k, const float *albedo_d, const float *albedo_s,
                                 const float *shininess, int32_t K, const float *grad_R, float *grad_opacity,
                                 float *grad_k, float *grad_albedo_d, float *grad_albedo_s, float *grad_shininess,
                                 void *stream) {
    if (!bvh || !k || !albedo_d || !albedo_s || !shininess || !grad_R)
        return einval("gsrad_brdf_backward: null argument");
    GS_TRY(usable(bvh, "gsrad_brdf_backward"));
    if (!valid_K(K)) return einval("gsrad_brdf_backward: K must be 1, 4, 9 or 16");
    return launch_brdf_backward(bvh->dev(), k, albedo_d, albedo_s, shininess, K, grad_R, grad_opacity, grad_k,
                                grad_albedo_d, grad_albedo_s, grad_shininess, S(stream));
}

gsrad_status gsrad_direct_light_sh(const gsrad_bvh *bvh, const float *R, int32_t K, const float *light_pos,
                                   const float *light_I, int32_t n_lights, float *E_out, void *stream) {
    if (!bvh || !R || !light_pos || !light_I || !E_out) return einval("gsrad_direct_light_sh: null argument");
    GS_TRY(usable(bvh, "gsrad_direct_light_sh"));
    if (n_lights < 1) return einval("gsrad_direct_light_sh: n_lights must be >= 1");
    if (!valid_K(K)) return einval("gsrad_direct_light_sh: K must be 1, 4, 9 or 16");
    gsrad_bvh *h = const_cast<gsrad_bvh *>(bvh);
    GS_TRY(h->height.ensure(64, "flags"));
    ProfScope ps("direct_light_sh", S(stream));
    return launch_direct_sh(bvh->dev(), R, light_pos, light_I, n_lights, K, E_out, h->height.as<int>() + 4, S(stream));
}

gsrad_status gsrad_transport_solve_sh(const gsrad_ff *ff, const gsrad_bvh *bvh, const float *R, const float *E,
                                      int32_t n_lights, int32_t K, int32_t n_bounces, float *B_out,
                                      gsrad_tape **tape, void *stream) {
    if (!ff || !bvh || !R || !E || !B_out) return einval("gsrad_transport_solve_sh: null argument");
    GS_TRY(usable(ff, "gsrad_transport_solve_sh"));
    GS_TRY(usable(bvh, "gsrad_transport_solve_sh"));
    if (bvh->n != ff->n) return einval("gsrad_transport_solve_sh: the BVH and F have different sizes");
    if (n_lights < 1) return einval("gsrad_transport_solve_sh: n_lights must be >= 1");
    if (!valid_K(K)) return einval("gsrad_transport_solve_sh: K must be 1, 4, 9 or 16");
    if (n_bounces < 0 || n_bounces > 4096) return einval("gsrad_transport_solve_sh: n_bounces must be in [0, 4096]");
    hipStream_t st = S(stream);
    const int C = n_lights * K * 3;
    const int64_t n = ff->n;
    const size_t row_bytes = (size_t)n * C * sizeof(float);
    gsrad_tape *tp = nullptr;
    bool created = false;
    if (tape) {
        created = *tape == nullptr;
        tp = created ? new gsrad_tape() : *tape;
        tp->ff = nullptr;   // unusable unless this solve succeeds
        tp->has_G = false;
    }
    auto fail = [&](gsrad_status e) {
        if (created) delete tp;
        return e;
    };
    gsrad_status e;
    const BvhDev bv = bvh->dev();
    const Csr F = ff->csr();
    if (n_bounces == 0) {
        if ((e = check_hip(hipMemcpyAsync(B_out, E, row_bytes, hipMemcpyDeviceToDevice, st), "solve copy")) != GSRAD_OK)
            return fail(e);
    } else {
        float *slots = nullptr, *qs = nullptr;
        if (tp) {
            if ((e = tp->B.ensure(row_bytes * n_bounces, "forward tape")) != GSRAD_OK) return fail(e);
            if ((e = tp->Q.ensure(row_bytes * n_bounces, "transfer tape")) != GSRAD_OK) return fail(e);
            slots = tp->B.as<float>();
            qs = tp->Q.as<float>();
            if ((e = check_hip(hipMemcpyAsync(slots, E, row_bytes, hipMemcpyDeviceToDevice, st), "tape copy")) !=
                GSRAD_OK)
                return fail(e);
        } else if (n_bounces > 1) {
            gsrad_ff *m = const_cast<gsrad_ff *>(ff);
            if ((e = m->slab.ensure(std::max(m->slab.bytes, row_bytes * 2), "ping-pong")) != GSRAD_OK) return fail(e);
        }
        const float *src = E;
        for (int k = 0; k < n_bounces; ++k) {
            float *dst;
            if (k == n_bounces - 1) dst = B_out;
            else if (tp) dst = slots + (size_t)(k + 1) * n * C;
            else dst = const_cast<gsrad_ff *>(ff)->slab.as<float>() + (size_t)(k & 1) * n * C;
            ProfScope ps("bounce_sh", st);
            if ((e = launch_transfer_sh(bv, F, n_lights, K, src, E, R, qs ? qs + (size_t)k * n * C : nullptr, dst, 0,
                                        st)) != GSRAD_OK)
                return fail(e);
            src = dst;
        }
    }
    if (tp) {
        tp->n = n;
        tp->C = C;
        tp->nb = n_bounces;
        tp->Lt = n_lights;
        tp->K = K;
        tp->precision = kTapeSH;
        tp->has_G = false;
        tp->ff = ff;
        tp->ff_gen = ff->fill_gen;
        tp->bvh = bvh;
        tp->bvh_gen = bvh->gen;
        *tape = tp;
    }
    return GSRAD_OK;
}

gsrad_status gsrad_transport_backward_sh(const gsrad_ff *ff, const gsrad_bvh *bvh, const gsrad_tape *tape,
                                         const float *R, const float *grad_B, float *grad_E, float *grad_R,
                                         float *grad_F, void *stream) {
    if (!ff || !bvh || !tape || !R || !grad_B || !grad_E) return einval("gsrad_transport_backward_sh: null argument");
    GS_TRY(usable(ff, "gsrad_transport_backward_sh"));
    GS_TRY(usable(bvh, "gsrad_transport_backward_sh"));
    if (tape->ff != ff || tape->ff_gen != ff->fill_gen || tape->n != ff->n || bvh->n != ff->n ||
        tape->bvh != bvh || tape->bvh_gen != bvh->gen)
        return einval("gsrad_transport_backward_sh: tape, F and BVH do not belong together as they are now");
    if (tape->precision != kTapeSH)
        return einval("gsrad_transport_backward_sh: the tape is not from gsrad_transport_solve_sh");
    hipStream_t st = S(stream);
    gsrad_ff *f = const_cast<gsrad_ff *>(ff);
    gsrad_tape *tp = const_cast<gsrad_tape *>(tape);
    const int64_t n = ff->n;
    const int C = tape->C, nb = tape->nb, Lt = tape->Lt, K = tape->K;
    const size_t row_bytes = (size_t)n * C * sizeof(float);
    GS_TRY(check_hip(hipMemcpyAsync(grad_E, grad_B, row_bytes, hipMemcpyDeviceToDevice, st), "grad_E init"));
    if (nb == 0) {
        if (grad_R) GS_TRY(check_hip(hipMemsetAsync(grad_R, 0, (size_t)n * K * 12, st), "grad_R zero"));
        if (grad_F && ff->nnz > 0)
            GS_TRY(check_hip(hipMemsetAsync(grad_F, 0, (size_t)ff->nnz * 4, st), "grad_F zero"));
        return GSRAD_OK;
    }
    {
        ProfScope ps("transpose", st);
        GS_TRY(ensure_transpose(f, st));
    }
    GS_TRY(tp->L.ensure(row_bytes * nb, "adjoint tape"));
    GS_TRY(tp->lam0.ensure(row_bytes, "adjoint scratch"));
    GS_TRY(tp->pp.ensure(row_bytes, "adjoint scaled rows"));
    float *L = tp->L.as<float>();
    float *u = tp->pp.as<float>();
    GS_TRY(check_hip(hipMemcpyAsync(L + (size_t)(nb - 1) * n * C, grad_B, row_bytes, hipMemcpyDeviceToDevice, st),
                     "adjoint seed"));
    const BvhDev bv = bvh->dev();
    const Csr FT = f->csr_t();
    for (int k = nb - 1; k >= 0; --k) {
        const float *lam_in = L + (size_t)k * n * C;   // lambda^(k+1)
        float *lam_out = k >= 1 ? L + (size_t)(k - 1) * n * C : tp->lam0.as<float>();
        ProfScope ps("adjoint_sh", st);
        GS_TRY(launch_scale_rows(lam_in, R, n, Lt, K, u, st));
        GS_TRY(launch_transfer_sh(bv, FT, Lt, K, u, nullptr, nullptr, lam_out, grad_E, 1, st));
    }
    ProfScope ps("sddmm_sh", st);
    if (grad_R) GS_TRY(launch_grad_R(L, tp->Q.as<float>(), n, Lt, K, nb, grad_R, st));
    if (grad_F) GS_TRY(launch_sddmm_sh(bv, ff->csr(), Lt, K, nb, tp->B.as<float>(), L, R, grad_F, st));
    return GSRAD_OK;
}

// ---------------------------------------------------------------------------
// centre-to-centre form factors with a learnable scale (Sec. 8)
// ---------------------------------------------------------------------------
gsrad_status gsrad_ff_center(const gsrad_bvh *bvh, const gsrad_ff *pattern, const float *lambda, gsrad_ff **ff,
                             void *stream) {
    if (!bvh || !pattern || !lambda || !ff) return einval("gsrad_ff_center: null argument");
    GS_TRY(usable(bvh, "gsrad_ff_center"));
    GS_TRY(usable(pattern, "gsrad_ff_center"));
    if (*ff == pattern) return einval("gsrad_ff_center: the output handle must differ from the pattern");
    if (pattern->n != bvh->n) return einval("gsrad_ff_center: the BVH and the pattern have different sizes");
    const bool created = *ff == nullptr;
    gsrad_ff *h = created ? new gsrad_ff() : *ff;
    invalidate(h);
    auto fail = [&](gsrad_status e) {
        if (created) delete h;
        return e;
    };
    hipStream_t st = S(stream);
    const int64_t n = pattern->n, nnz = pattern->nnz;
    gsrad_status e;
    if ((e = h->row_ptr.ensure((size_t)(n + 1) * 8, "row_ptr")) != GSRAD_OK) return fail(e);
    if ((e = h->col.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "col")) != GSRAD_OK) return fail(e);
    if ((e = h->val.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "val")) != GSRAD_OK) return fail(e);
    if ((e = h->err.ensure(128, "flags")) != GSRAD_OK) return fail(e);
    if ((e = check_hip(hipMemcpyAsync(h->row_ptr.p, pattern->row_ptr.p, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice,
                                      st), "copy row_ptr")) != GSRAD_OK)
        return fail(e);
    if (nnz > 0 && (e = check_hip(hipMemcpyAsync(h->col.p, pattern->col.p, (size_t)nnz * 4, hipMemcpyDeviceToDevice,
                                                 st), "copy col")) != GSRAD_OK)
        return fail(e);
    if (pattern->has_order) {
        if ((e = h->row_order.ensure((size_t)n * 4, "row order")) != GSRAD_OK) return fail(e);
        if ((e = check_hip(hipMemcpyAsync(h->row_order.p, pattern->row_order.p, (size_t)n * 4,
                                          hipMemcpyDeviceToDevice, st), "copy row order")) != GSRAD_OK)
            return fail(e);
    }
    if ((e = check_hip(hipMemsetAsync(h->err.p, 0, 64, st), "flags")) != GSRAD_OK) return fail(e);
    h->n = n;
    h->nnz = nnz;
    h->fill_gen = ++g_fill_gen;
    h->has_order = pattern->has_order;
    Csr P = h->csr();
    {
        ProfScope ps("ff_center", st);
        if ((e = launch_ff_center(bvh->dev(), P, lambda, h->val.as<float>(), h->err.as<int>(), st)) != GSRAD_OK)
            return fail(e);
    }
    int flag = 0;
    if ((e = check_hip(hipMemcpyAsync(&flag, h->err.p, 4, hipMemcpyDeviceToHost, st), "flags copy")) != GSRAD_OK)
        return fail(e);
    if ((e = check_hip(hipStreamSynchronize(st), "ff_center sync")) != GSRAD_OK) return fail(e);
    if (flag) {
        invalidate(h);
        set_error("gsrad_ff_center: traversal stack overflow");
        if (created) delete h;
        return GSRAD_EOVERFLOW;
    }
    h->max_row = pattern->max_row;
    h->center_bvh = bvh;
    h->center_gen = bvh->gen;
    *ff = h;
    return GSRAD_OK;
}

gsrad_status gsrad_ff_center_backward(const gsrad_bvh *bvh, const gsrad_ff *ff, const float *lambda,
                                      const float *grad_F, float *grad_lambda, const gsrad_surfel_grads *grads,
                                      void *stream) {
    if (!bvh || !ff || !lambda || !grad_F) return einval("gsrad_ff_center_backward: null argument");
    GS_TRY(usable(bvh, "gsrad_ff_center_backward"));
    GS_TRY(usable(ff, "gsrad_ff_center_backward"));
    if (ff->center_bvh != bvh || ff->center_gen != bvh->gen)
        return einval("gsrad_ff_center_backward: F was not made by gsrad_ff_center from this BVH as it is now");
    hipStream_t st = S(stream);
    gsrad_ff *f = const_cast<gsrad_ff *>(ff);
    const size_t bytes = center_acc_bytes(ff->n);
    GS_TRY(f->cacc.ensure(bytes, "centre-to-centre gradient accumulators"));
    GS_TRY(check_hip(hipMemsetAsync(f->cacc.p, 0, bytes, st), "accumulators zero"));
    GS_TRY(f->err.ensure(128, "flags"));
    CenterOutputs out;
    const gsrad_surfel_grads z{};
    const gsrad_surfel_grads &g = grads ? *grads : z;
    float *fields[16] = {g.px, g.py, g.pz, g.tux, g.tuy, g.tuz, g.tvx, g.tvy, g.tvz, g.nx, g.ny, g.nz, g.su, g.sv,
                         g.opacity, grad_lambda};
    for (int k = 0; k < 16; ++k) out.p[k] = fields[k];
    ProfScope ps("ff_center_backward", st);
    return launch_center_backward(bvh->dev(), ff->csr(), lambda, grad_F, f->cacc.p, out, f->err.as<int>() + 8, st);
}

gsrad_status gsrad_direct_light_backward(const gsrad_bvh *bvh, const float *albedo, const float *light_pos,
                                         const float *light_I, int32_t n_lights, int32_t K, const float *grad_E,
                                         float *grad_light_pos, float *grad_light_I, float *grad_albedo,
                                         const gsrad_surfel_grads *grads, void *stream) {
    if (!bvh || !albedo || !light_pos || !light_I || !grad_E) return einval("gsrad_direct_light_backward: null argument");
    GS_TRY(usable(bvh, "gsrad_direct_light_backward"));
    if (n_lights < 1) return einval("gsrad_direct_light_backward: n_lights must be >= 1");
    if (!valid_K(K)) return einval("gsrad_direct_light_backward: K must be 1, 4, 9 or 16");
    hipStream_t st = S(stream);
    gsrad_bvh *h = const_cast<gsrad_bvh *>(bvh);
    const size_t bytes = light_acc_bytes(bvh->n, n_lights);
    GS_TRY(h->lacc.ensure(bytes, "direct light gradient accumulators"));
    GS_TRY(check_hip(hipMemsetAsync(h->lacc.p, 0, bytes, st), "accumulators zero"));
    GS_TRY(h->height.ensure(64, "flags"));
    const gsrad_surfel_grads z{};
    const gsrad_surfel_grads &g = grads ? *grads : z;
    CenterOutputs out;
    float *fields[16] = {g.px, g.py, g.pz, g.tux, g.tuy, g.tuz, g.tvx, g.tvy, g.tvz, g.nx, g.ny, g.nz, g.su, g.sv,
                         g.opacity, nullptr};
    for (int k = 0; k < 16; ++k) out.p[k] = fields[k];
    ProfScope ps("direct_light_backward", st);
    return launch_direct_backward(bvh->dev(), albedo, light_pos, light_I, n_lights, K, grad_E, h->lacc.p,
                                  grad_light_pos, grad_light_I, grad_albedo, out, h->height.as<int>() + 12, st);
}

gsrad_status gsrad_geometry_backward(const gsrad_bvh *bvh, const gsrad_ff *ff, const float *grad_F,
                                     const gsrad_surfel_grads *grads, void *stream) {
    if (!bvh || !ff || !grad_F || !grads) return einval("gsrad_geometry_backward: null argument");
    GS_TRY(usable(bvh, "gsrad_geometry_backward"));
    GS_TRY(usable(ff, "gsrad_geometry_backward"));
    if (ff->bvh != bvh || ff->bvh_gen != bvh->gen || ff->n != bvh->n)
        return einval("gsrad_geometry_backward: the F handle was not made by gsrad_form_factors from this BVH as it "
                      "is now");
    if (!ff->has_records) {
        set_error("gsrad_geometry_backward: needs the per-ray hit records (cast F without GSRAD_FF_NO_RECORDS "
                  "and within the record budget)");
        return GSRAD_ESTATE;
    }
    hipStream_t st = S(stream);
    gsrad_ff *f = const_cast<gsrad_ff *>(ff);
    const size_t bytes = center_acc_bytes(ff->n);
    GS_TRY(f->cacc.ensure(bytes, "geometry gradient accumulators"));
    GS_TRY(check_hip(hipMemsetAsync(f->cacc.p, 0, bytes, st), "accumulators zero"));
    const gsrad_surfel_grads &g = *grads;
    CenterOutputs out;
    float *fields[16] = {g.px, g.py, g.pz, g.tux, g.tuy, g.tuz, g.tvx, g.tvy, g.tvz, g.nx, g.ny, g.nz, g.su, g.sv,
                         g.opacity, nullptr};
    for (int k = 0; k < 16; ++k) out.p[k] = fields[k];
    if (f->nnz == 0) {
        for (int k = 0; k < 15; ++k)
            if (fields[k]) GS_TRY(check_hip(hipMemsetAsync(fields[k], 0, (size_t)ff->n * 4, st), "zero gradient"));
        return GSRAD_OK;
    }
    ProfScope ps("geometry_backward", st);
    return launch_geometry_rec(bvh->dev(), f->R, f->seed, f->recs.as<uint2>(), f->rcnt.as<uint32_t>(), f->rec_cap,
                               f->row_ptr.as<int64_t>(), f->col.as<int32_t>(), grad_F, std::max(f->max_row, 1),
                               f->cacc.p, out, st);
}

gsrad_status gsrad_opacity_backward(const gsrad_bvh *bvh, const gsrad_ff *ff, const float *grad_F,
                                    const float *grad_rho, const float *albedo, float *grad_opacity,
                                    float *grad_albedo, void *stream) {
    if (!bvh || !ff) return einval("gsrad_opacity_backward: null handle");
    GS_TRY(usable(bvh, "gsrad_opacity_backward"));
    if (grad_F) {
        GS_TRY(usable(ff, "gsrad_opacity_backward"));
        if (ff->bvh != bvh || ff->bvh_gen != bvh->gen || ff->n != bvh->n)
            return einval("gsrad_opacity_backward: the F handle was not made by gsrad_form_factors from this BVH "
                          "as it is now (it was rebuilt since)");
    }
    if (grad_rho && !albedo) return einval("gsrad_opacity_backward: grad_rho needs albedo");
    hipStream_t st = S(stream);
    gsrad_ff *f = const_cast<gsrad_ff *>(ff);
    const int64_t n = bvh->n;
    const size_t acc_bytes = opacity_acc_bytes(n);
    GS_TRY(f->opac.ensure(acc_bytes, "opacity accumulators"));
    void *acc = f->opac.p;
    GS_TRY(check_hip(hipMemsetAsync(acc, 0, acc_bytes, st), "opacity zero"));
    const bool with_F = grad_F && f->nnz > 0;
    GS_TRY(launch_opacity_scale(with_F ? grad_F : nullptr, f->nnz, n, acc, st));
    if (with_F) {
        if ((size_t)f->max_row * 8 + ff_stack_bytes(256) > 150 * 1024)
            return einval("gsrad_opacity_backward: row too long for the LDS row cache");
        if (f->has_records) {
            ProfScope ps("opacity_records", st);
            GS_TRY(launch_opacity_rec(bvh->dev(), f->R, f->recs.as<uint2>(), f->rcnt.as<uint32_t>(), f->rec_cap,
                                      f->row_ptr.as<int64_t>(), f->col.as<int32_t>(), grad_F, std::max(f->max_row, 1),
                                      acc, st));
        } else {
            // recompute the rays without (complete) records by traversal
            GS_TRY(f->slab.ensure(std::max(f->slab.bytes, (size_t)n * f->R * sizeof(float2)), "ray sums"));
            GS_TRY(f->err.ensure(128, "flags"));
            for (int pass = 0; pass < 2; ++pass) {
                ProfScope ps(pass == 0 ? "opacity_pass1" : "opacity_pass2", st);
                GS_TRY(launch_opacity_bwd(bvh->dev(), f->R, f->seed, f->t_eps, f->t_min, f->row_ptr.as<int64_t>(),
                                          f->col.as<int32_t>(), grad_F, std::max(f->max_row, 1), f->slab.as<float2>(),
                                          acc, pass, nullptr, 0, f->err.as<int>() + 8, st));
            }
        }
    }
    ProfScope ps("opacity_finish", st);
    return launch_opacity_finish(bvh->dev(), acc, grad_rho, albedo, grad_opacity, grad_albedo, st);
}

gsrad_status gsrad_ray_hits(const gsrad_bvh *bvh, const gsrad_ff_params *p, const int64_t *receivers,
                            int64_t n_receivers, int32_t max_hits, float *dirs, int32_t *count, int32_t *hit_j,
                            float *hit_t, int8_t *hit_front, float *hit_T, void *stream) {
    if (!bvh || !p || !receivers || !dirs || !count) return einval("gsrad_ray_hits: null argument");
    GS_TRY(usable(bvh, "gsrad_ray_hits"));
    if (max_hits < 0 || (max_hits > 0 && (!hit_j || !hit_t || !hit_front || !hit_T)))
        return einval("gsrad_ray_hits: bad hit buffers");
    if (p->rays_per_surfel < 1 || n_receivers < 1) return einval("gsrad_ray_hits: bad sizes");
    gsrad_bvh *h = const_cast<gsrad_bvh *>(bvh);
    GS_TRY(h->height.ensure(64, "flags"));
    return launch_ray_hits(bvh->dev(), p->rays_per_surfel, p->seed, p->t_eps, p->t_min, receivers, n_receivers,
                           max_hits, dirs, count, hit_j, hit_t, hit_front, hit_T, h->height.as<int>() + 8, S(stream));
}

gsrad_status gsrad_check(const gsrad_ff *ff, const float *rho, const float *E, const float *B, int32_t n_lights,
                         int32_t K, double *out_host, void *stream) {
    if (!ff || !rho || !E || !B || !out_host) return einval("gsrad_check: null argument");
    GS_TRY(usable(ff, "gsrad_check"));
    if (n_lights < 1 || !valid_K(K)) return einval("gsrad_check: bad n_lights or K");
    hipStream_t st = S(stream);
    gsrad_ff *f = const_cast<gsrad_ff *>(ff);
    GS_TRY(f->err.ensure(128, "check accumulators"));
    double *acc = reinterpret_cast<double *>(f->err.as<char>() + 64);
    GS_TRY(check_hip(hipMemsetAsync(acc, 0, 32, st), "check zero"));
    GS_TRY(launch_check(ff->csr(), n_lights * K * 3, rho, E, B, acc, st));
    double a[4];
    GS_TRY(check_hip(hipMemcpyAsync(a, acc, sizeof(a), hipMemcpyDeviceToHost, st), "check copy"));
    GS_TRY(check_hip(hipStreamSynchronize(st), "check sync"));
    out_host[0] = a[1] > 0 ? std::sqrt(a[0] / a[1]) : std::sqrt(a[0]);
    out_host[1] = a[2];
    out_host[2] = a[3] > 0 ? 1.0 : 0.0;
    if (a[3] > 0) {
        set_error("gsrad_check: %g non-finite values", a[3]);
        return GSRAD_ENAN;
    }
    return GSRAD_OK;
}

gsrad_status gsrad_check_reciprocity(const gsrad_bvh *bvh, const gsrad_ff *ff, double *out_host, void *stream) {
    if (!bvh || !ff || !out_host) return einval("gsrad_check_reciprocity: null argument");
    GS_TRY(usable(bvh, "gsrad_check_reciprocity"));
    GS_TRY(usable(ff, "gsrad_check_reciprocity"));
    if (bvh->n != ff->n) return einval("gsrad_check_reciprocity: the BVH and F have different sizes");
    hipStream_t st = S(stream);
    gsrad_ff *f = const_cast<gsrad_ff *>(ff);
    GS_TRY(f->err.ensure(128, "check accumulators"));
    double *acc = reinterpret_cast<double *>(f->err.as<char>() + 64);
    GS_TRY(check_hip(hipMemsetAsync(acc, 0, 24, st), "reciprocity zero"));
    GS_TRY(launch_reciprocity(ff->csr(), bvh->B.area, acc, st));
    double a[3];
    GS_TRY(check_hip(hipMemcpyAsync(a, acc, sizeof(a), hipMemcpyDeviceToHost, st), "reciprocity copy"));
    GS_TRY(check_hip(hipStreamSynchronize(st), "reciprocity sync"));
    out_host[0] = a[1] > 0 ? a[0] / a[1] : 0.0;
    out_host[1] = a[2];
    return GSRAD_OK;
}

gsrad_status gsrad_profile_enable(int32_t on) {
    prof_clear();
    g_prof = on != 0;
    return GSRAD_OK;
}

gsrad_status gsrad_profile_report(char *buf, int64_t len) {
    if (!buf || len < 1) return einval("gsrad_profile_report: null buffer");
    struct Acc {
        int64_t count = 0;
        double total = 0.0, mn = 1e300, mx = 0.0;
    };
    std::map<std::string, Acc> acc;
    for (ProfRec &r : g_recs) {
        GS_TRY(check_hip(hipEventSynchronize(r.b), "profile sync"));
        float ms = 0.0f;
        GS_TRY(check_hip(hipEventElapsedTime(&ms, r.a, r.b), "profile elapsed"));
        Acc &a = acc[r.name];
        a.count += 1;
        a.total += ms;
        a.mn = std::min(a.mn, (double)ms);
        a.mx = std::max(a.mx, (double)ms);
    }
    std::string out;
    char line[256];
    for (auto &kv : acc) {
        snprintf(line, sizeof(line), "%s\t%lld\t%.6f\t%.6f\t%.6f\n", kv.first.c_str(), (long long)kv.second.count,
                 kv.second.total, kv.second.mn, kv.second.mx);
        out += line;
    }
    if ((int64_t)out.size() + 1 > len) return einval("gsrad_profile_report: buffer too small");
    memcpy(buf, out.c_str(), out.size() + 1);
    return GSRAD_OK;
}

void gsrad_bvh_destroy(gsrad_bvh *bvh) { delete bvh; }
void gsrad_ff_destroy(gsrad_ff *ff) { delete ff; }
void gsrad_tape_destroy(gsrad_tape *tape) { delete tape; }

gsrad_status gsrad_batch_create(const gsrad_ff *const *ffs, int32_t n_scenes, const int32_t *lights, int32_t K,
                                gsrad_batch **batch, void *stream) {
    if (!ffs || !lights || !batch) return einval("gsrad_batch_create: null argument");
    if (n_scenes < 1) return einval("gsrad_batch_create: n_scenes must be >= 1");
    if (!valid_K(K)) return einval("gsrad_batch_create: K must be 1, 4, 9 or 16");
    std::vector<int64_t> roff(n_scenes + 1, 0), voff(n_scenes + 1, 0), eoff(n_scenes + 1, 0);
    std::vector<int32_t> Cs(n_scenes);
    int max_row = 0;
    for (int s = 0; s < n_scenes; ++s) {
        if (!ffs[s] || ffs[s]->n < 1) {
            set_error("gsrad_batch_create: scene %d has no (usable) operator", s);
            return GSRAD_EINVAL;
        }
        if (lights[s] < 1) {
            set_error("gsrad_batch_create: scene %d needs at least one light", s);
            return GSRAD_EINVAL;
        }
        Cs[s] = lights[s] * K * 3;
        roff[s + 1] = roff[s] + ffs[s]->n;
        voff[s + 1] = voff[s] + ffs[s]->n * (int64_t)Cs[s];
        eoff[s + 1] = eoff[s] + ffs[s]->nnz;
        max_row = std::max(max_row, ffs[s]->max_row);
    }
    if (roff[n_scenes] >= ((int64_t)1 << 31) || eoff[n_scenes] >= ((int64_t)1 << 32))
        return einval("gsrad_batch_create: batch too large (rows < 2^31, entries < 2^32)");
    hipStream_t st = S(stream);
    // an existing batch of the same scene layout is refilled in place: its
    // tuned lanes per row stay, and so does its captured bounce loop while
    // no buffer has to grow
    gsrad_batch *b = *batch;
    const bool reuse = b && b->S == n_scenes && b->K == K && b->rows == roff[n_scenes] && b->vals == voff[n_scenes] &&
                       b->scene_rows == std::vector<int64_t>(roff.begin(), roff.end()) && b->scene_cols == Cs;
    const bool created = !reuse;
    gsrad_batch *const old = created ? *batch : nullptr;   // replaced on success
    if (created) b = new gsrad_batch();
    auto fail = [&](gsrad_status e) {
        if (created) {
            delete b;
        } else {
            // a batch refilled part-way is unusable until refilled again
            b->drop_graph();
            b->nb = -1;
            if (b->F) invalidate(b->F);
        }
        return e;
    };
    gsrad_status e;
    b->S = n_scenes;
    b->K = K;
    b->rows = roff[n_scenes];
    b->vals = voff[n_scenes];
    b->scene_rows.assign(roff.begin(), roff.end());
    b->scene_cols = Cs;
    if (!b->F) b->F = new gsrad_ff();
    gsrad_ff *F = b->F;
    const void *old_ptrs[3] = {F->row_ptr.p, F->col.p, F->val.p};
    const int64_t rows = b->rows, nnz = eoff[n_scenes];
    if ((e = F->row_ptr.ensure((size_t)(rows + 1) * 8, "batch row_ptr")) != GSRAD_OK) return fail(e);
    if ((e = F->col.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "batch col")) != GSRAD_OK) return fail(e);
    if ((e = F->val.ensure((size_t)std::max<int64_t>(nnz, 1) * 4, "batch val")) != GSRAD_OK) return fail(e);
    for (int s = 0; s < n_scenes; ++s) {
        const gsrad_ff *f = ffs[s];
        if ((e = launch_offset_copy_i64(f->row_ptr.as<int64_t>(), f->n, eoff[s], F->row_ptr.as<int64_t>() + roff[s],
                                        st)) != GSRAD_OK)
            return fail(e);
        if ((e = launch_offset_copy_i32(f->col.as<int32_t>(), f->nnz, (int32_t)roff[s], F->col.as<int32_t>() + eoff[s],
                                        st)) != GSRAD_OK)
            return fail(e);
        if (f->nnz > 0 && (e = check_hip(hipMemcpyAsync(F->val.as<float>() + eoff[s], f->val.p, (size_t)f->nnz * 4,
                                                        hipMemcpyDeviceToDevice, st),
                                         "batch val copy")) != GSRAD_OK)
            return fail(e);
    }
    if ((e = check_hip(hipMemcpyAsync(F->row_ptr.as<int64_t>() + rows, &eoff[n_scenes], 8, hipMemcpyHostToDevice, st),
                       "batch row_ptr end")) != GSRAD_OK)
        return fail(e);
    F->n = rows;
    F->nnz = nnz;
    F->fill_gen = ++g_fill_gen;
    F->max_row = max_row;
    F->has_t = false;
    F->has_order = false;
    if (old_ptrs[0] != F->row_ptr.p || old_ptrs[1] != F->col.p || old_ptrs[2] != F->val.p) b->drop_graph();
    if ((e = b->row_off.ensure((size_t)(n_scenes + 1) * 8, "scene rows")) != GSRAD_OK) return fail(e);
    if ((e = b->val_off.ensure((size_t)(n_scenes + 1) * 8, "scene values")) != GSRAD_OK) return fail(e);
    if ((e = b->scene_C.ensure((size_t)n_scenes * 4, "scene columns")) != GSRAD_OK) return fail(e);
    if ((e = b->row_scene.ensure((size_t)rows * 4, "row scenes")) != GSRAD_OK) return fail(e);
    if ((e = b->order.ensure((size_t)rows * 8, "row order")) != GSRAD_OK) return fail(e);
    if ((e = b->counter.ensure(256, "work counter")) != GSRAD_OK) return fail(e);
    if ((e = b->temp.ensure(batch_order_temp_bytes(rows), "batch temp")) != GSRAD_OK) return fail(e);
    if ((e = check_hip(hipMemcpyAsync(b->row_off.p, roff.data(), (size_t)(n_scenes + 1) * 8, hipMemcpyHostToDevice, st),
                       "scene rows copy")) != GSRAD_OK)
        return fail(e);
    if ((e = check_hip(hipMemcpyAsync(b->val_off.p, voff.data(), (size_t)(n_scenes + 1) * 8, hipMemcpyHostToDevice, st),
                       "scene values copy")) != GSRAD_OK)
        return fail(e);
    if ((e = check_hip(hipMemcpyAsync(b->scene_C.p, Cs.data(), (size_t)n_scenes * 4, hipMemcpyHostToDevice, st),
                       "scene columns copy")) != GSRAD_OK)
        return fail(e);
    if ((e = batch_order_rows(b->dev(), F->row_ptr.as<int64_t>(), b->temp.p, b->temp.bytes, st)) != GSRAD_OK)
        return fail(e);
    // scenes that all come from a ray cast: their rows in the receivers'
    // Morton order, scene after scene, so the rows running together gather
    // from one scene's nearby columns (replaces the cost order)
    bool all_ordered = true;
    for (int s = 0; s < n_scenes; ++s) all_ordered = all_ordered && ffs[s]->has_order;
    if (all_ordered)
        for (int s = 0; s < n_scenes; ++s)
            if ((e = launch_offset_widen(ffs[s]->row_order.as<int32_t>(), ffs[s]->n, roff[s],
                                         b->order.as<int64_t>() + roff[s], st)) != GSRAD_OK)
                return fail(e);
    // the host vectors above are sources of asynchronous copies
    if ((e = check_hip(hipStreamSynchronize(st), "batch create sync")) != GSRAD_OK) return fail(e);
    b->nb = -1;
    *batch = b;
    if (old) delete old;
    return GSRAD_OK;
}

gsrad_status gsrad_batch_info(const gsrad_batch *b, int64_t *rows, int64_t *vals, int32_t *lanes_bounce,
                              int32_t *lanes_adjoint) {
    if (!b) return einval("gsrad_batch_info: null handle");
    if (rows) *rows = b->rows;
    if (vals) *vals = b->vals;
    if (lanes_bounce) *lanes_bounce = b->lpr_fwd;
    if (lanes_adjoint) *lanes_adjoint = b->lpr_adj;
    return GSRAD_OK;
}

gsrad_status gsrad_batch_ff(const gsrad_batch *b, const gsrad_ff **ff) {
    if (!b || !ff) return einval("gsrad_batch_ff: null argument");
    *ff = b->F;
    return GSRAD_OK;
}

namespace {

// Lanes per row for a ragged product: each candidate runs once on the
// batch's own rows (into scratch) and the fastest is kept.
gsrad_status autotune_lanes_timed(gsrad_batch *b, const Csr &F, bool adjoint, const float *in, const float *rho,
                                  float *scratch, float *scratch2, hipStream_t st, int *best) {
    hipEvent_t e0, e1;
    GS_TRY(check_hip(hipEventCreate(&e0), "tune event"));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return check_hip(hipErrorOutOfMemory, "tune event");
    }
    float best_ms = 0.0f;
    gsrad_status e = GSRAD_OK;
    for (int lpr : {64, 32, 16}) {
        for (int rep = 0; rep < 2 && e == GSRAD_OK; ++rep) {   // the first run warms the caches
            if ((e = check_hip(hipEventRecord(e0, st), "tune record")) != GSRAD_OK) break;
            e = launch_ragged_spmm(b->dev(), F, lpr, adjoint, in, false, in, rho, scratch, scratch2,
                                   b->counter.as<uint32_t>(), st);
            if (e == GSRAD_OK) e = check_hip(hipEventRecord(e1, st), "tune record");
        }
        if (e != GSRAD_OK) break;
        if ((e = check_hip(hipEventSynchronize(e1), "tune sync")) != GSRAD_OK) break;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (*best == 0 || ms < best_ms) {
            best_ms = ms;
            *best = lpr;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

// Lanes per row chosen by timing, remembered per batch shape (rows, stored
// entries, values of the ragged arrays, direction) for the process, so a
// new batch of a shape already seen skips the timing runs.
std::mutex g_tune_mu;
std::map<std::tuple<int64_t, int64_t, int64_t, bool>, int> g_tune_cache;

gsrad_status autotune_lanes(gsrad_batch *b, const Csr &F, bool adjoint, const float *in, const float *rho,
                            float *scratch, float *scratch2, hipStream_t st, int *best) {
    const auto key = std::make_tuple(b->rows, F.nnz, b->vals, adjoint);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = it->second;
            return GSRAD_OK;
        }
    }
    const gsrad_status r = autotune_lanes_timed(b, F, adjoint, in, rho, scratch, scratch2, st, best);
    if (r == GSRAD_OK && *best != 0) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = *best;
    }
    return r;
}

}  // namespace

gsrad_status gsrad_batch_transport_solve(gsrad_batch *b, const float *rho, const float *E, int32_t n_bounces,
                                         float *B_out, void *stream) {
    if (!b || !rho || !E || !B_out) return einval("gsrad_batch_transport_solve: null argument");
    if (!b->F || b->F->n < 1) {
        set_error("gsrad_batch_transport_solve: the batch is unusable after a failed refill");
        return GSRAD_ESTATE;
    }
    if (n_bounces < 0 || n_bounces > 4096) return einval("gsrad_batch_transport_solve: n_bounces must be in [0, 4096]");
    hipStream_t st = S(stream);
    const int64_t vals = b->vals;
    const Csr F = b->F->csr();
    b->nb = -1;
    if (n_bounces == 0) {
        GS_TRY(check_hip(hipMemcpyAsync(B_out, E, (size_t)vals * 4, hipMemcpyDeviceToDevice, st), "batch copy"));
        b->nb = 0;
        return GSRAD_OK;
    }
    const size_t tape_bytes = (size_t)n_bounces * vals * 4;
    if (b->Bt.bytes < tape_bytes) {
        b->drop_graph();   // the captured loop writes into the old tape
        GS_TRY(b->Bt.ensure(tape_bytes, "batch forward tape"));
    }
    if (b->force_fwd) b->lpr_fwd = b->force_fwd;
    if (b->lpr_fwd == 0) {
        ProfScope ps("batch_tune", st);
        GS_TRY(autotune_lanes(b, F, false, E, rho, B_out, nullptr, st, &b->lpr_fwd));
    }
    float *tape = b->Bt.as<float>();
    const bool bf = b->precision == GSRAD_BF16;
    if (bf && b->Bh.bytes < (size_t)vals * 4) {
        b->drop_graph();
        GS_TRY(b->Bh.ensure((size_t)vals * 4, "batch BF16 rows"));
    }
    char *bh = bf ? static_cast<char *>(b->Bh.p) : nullptr;   // two [vals] BF16 slots
    const bool hit = b->exec && b->g_rho == rho && b->g_E == E && b->g_B == B_out && b->g_tape == tape &&
                     b->g_nb == n_bounces && b->g_lpr == b->lpr_fwd && b->g_prec == b->precision && b->g_h == bh;
    if (!hit) {
        b->drop_graph();
        if (!b->cap) GS_TRY(check_hip(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream"));
        GS_TRY(check_hip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture"));
        gsrad_status e = launch_copy_f32(E, vals, tape, b->cap);
        // BF16: bounces 0 .. n-2 gather B^(k) rounded to BF16, the last one
        // gathers the FP32 B^(n-1)
        if (bf && n_bounces > 1 && e == GSRAD_OK) e = launch_round_bf16(E, vals, bh, b->cap);
        for (int k = 0; k < n_bounces && e == GSRAD_OK; ++k) {
            const bool last = k == n_bounces - 1;
            const bool in_bf = bf && !last;
            const void *in = in_bf ? static_cast<const void *>(bh + (size_t)(k & 1) * vals * 2)
                                   : static_cast<const void *>(tape + (size_t)k * vals);
            float *out = last ? B_out : tape + (size_t)(k + 1) * vals;
            e = launch_ragged_spmm(b->dev(), F, b->lpr_fwd, false, in, in_bf, E, rho, out, nullptr,
                                   b->counter.as<uint32_t>(), b->cap);
            if (e == GSRAD_OK && bf && k + 1 < n_bounces - 1)
                e = launch_round_bf16(out, vals, bh + (size_t)((k + 1) & 1) * vals * 2, b->cap);
        }
        hipGraph_t g = nullptr;
        const gsrad_status ec = check_hip(hipStreamEndCapture(b->cap, &g), "end capture");
        if (e != GSRAD_OK || ec != GSRAD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return e != GSRAD_OK ? e : ec;
        }
        b->graph = g;
        GS_TRY(check_hip(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate"));
        b->g_rho = rho;
        b->g_E = E;
        b->g_B = B_out;
        b->g_tape = tape;
        b->g_nb = n_bounces;
        b->g_lpr = b->lpr_fwd;
        b->g_prec = b->precision;
        b->g_h = bh;
    }
    {
        ProfScope ps("batch_bounces", st);
        GS_TRY(check_hip(hipGraphLaunch(b->exec, st), "graph launch"));
    }
    b->nb = n_bounces;
    return GSRAD_OK;
}

gsrad_status gsrad_batch_transport_backward(gsrad_batch *b, const float *rho, const float *grad_B, float *grad_E,
                                            float *grad_rho, float *grad_F, void *stream) {
    if (!b || !rho || !grad_B || !grad_E) return einval("gsrad_batch_transport_backward: null argument");
    if (b->nb < 0) {
        set_error("gsrad_batch_transport_backward: no forward solve on this batch");
        return GSRAD_ESTATE;
    }
    hipStream_t st = S(stream);
    const int64_t vals = b->vals, rows = b->rows;
    const int nb = b->nb;
    GS_TRY(check_hip(hipMemcpyAsync(grad_E, grad_B, (size_t)vals * 4, hipMemcpyDeviceToDevice, st), "grad_E init"));
    if (nb == 0) {
        if (grad_rho) GS_TRY(check_hip(hipMemsetAsync(grad_rho, 0, (size_t)rows * 12, st), "grad_rho zero"));
        if (grad_F && b->F->nnz > 0)
            GS_TRY(check_hip(hipMemsetAsync(grad_F, 0, (size_t)b->F->nnz * 4, st), "grad_F zero"));
        return GSRAD_OK;
    }
    {
        ProfScope ps("transpose", st);
        GS_TRY(ensure_transpose(b->F, st));
    }
    GS_TRY(b->Lt.ensure((size_t)(nb + 1) * vals * 4, "batch adjoint tape"));   // + one scratch slot
    GS_TRY(b->lam0.ensure((size_t)vals * 4, "batch adjoint scratch"));
    float *L = b->Lt.as<float>();
    GS_TRY(check_hip(hipMemcpyAsync(L + (size_t)(nb - 1) * vals, grad_B, (size_t)vals * 4, hipMemcpyDeviceToDevice, st),
                     "adjoint seed"));
    const Csr FT = b->F->csr_t();
    if (b->force_adj) b->lpr_adj = b->force_adj;
    if (b->lpr_adj == 0) {
        // timing runs write only into scratch: lam0 and the slot past the tape
        float *s2 = L + (size_t)nb * vals;
        ProfScope ps("batch_tune", st);
        GS_TRY(check_hip(hipMemsetAsync(s2, 0, (size_t)vals * 4, st), "tune scratch"));
        GS_TRY(autotune_lanes(b, FT, true, grad_B, rho, b->lam0.as<float>(), s2, st, &b->lpr_adj));
    }
    // the adjoint loop is captured once into a HIP graph and replayed while
    // its arguments stay the same
    float *lam0 = b->lam0.as<float>();
    const bool bf = b->precision == GSRAD_BF16;
    if (bf && b->Lh.bytes < (size_t)vals * 4) {
        if (b->aexec) (void)hipGraphExecDestroy(b->aexec);
        if (b->agraph) (void)hipGraphDestroy(b->agraph);
        b->aexec = nullptr;
        b->agraph = nullptr;
        b->a_nb = -1;
        GS_TRY(b->Lh.ensure((size_t)vals * 4, "batch BF16 adjoint rows"));
    }
    char *lh = bf ? static_cast<char *>(b->Lh.p) : nullptr;   // two [vals] BF16 slots
    const bool hit = b->aexec && b->a_rho == rho && b->a_gE == grad_E && b->a_L == L && b->a_lam0 == lam0 &&
                     b->a_nb == nb && b->a_lpr == b->lpr_adj && b->a_ft[0] == FT.row_ptr && b->a_ft[1] == FT.col &&
                     b->a_ft[2] == FT.val && b->a_prec == b->precision && b->a_h == lh;
    if (!hit) {
        if (b->aexec) (void)hipGraphExecDestroy(b->aexec);
        if (b->agraph) (void)hipGraphDestroy(b->agraph);
        b->aexec = nullptr;
        b->agraph = nullptr;
        b->a_nb = -1;
        if (!b->cap) GS_TRY(check_hip(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream"));
        GS_TRY(check_hip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture"));
        gsrad_status e = GSRAD_OK;
        // BF16: the adjoint of the forward above: its first step (the last
        // bounce's transpose) gathers the FP32 lambda^(n), the others
        // lambda^(k+1) rounded to BF16
        for (int k = nb - 1; k >= 0 && e == GSRAD_OK; --k) {
            const bool in_bf = bf && k < nb - 1;
            const void *in = in_bf ? static_cast<const void *>(lh + (size_t)(k & 1) * vals * 2)
                                   : static_cast<const void *>(L + (size_t)k * vals);   // lambda^(k+1)
            float *out = k >= 1 ? L + (size_t)(k - 1) * vals : lam0;
            e = launch_ragged_spmm(b->dev(), FT, b->lpr_adj, true, in, in_bf, nullptr, rho, out, grad_E,
                                   b->counter.as<uint32_t>(), b->cap);
            if (e == GSRAD_OK && bf && k >= 1) e = launch_round_bf16(out, vals, lh + (size_t)((k - 1) & 1) * vals * 2, b->cap);
        }
        hipGraph_t gr = nullptr;
        const gsrad_status ec = check_hip(hipStreamEndCapture(b->cap, &gr), "end capture");
        if (e != GSRAD_OK || ec != GSRAD_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return e != GSRAD_OK ? e : ec;
        }
        b->agraph = gr;
        GS_TRY(check_hip(hipGraphInstantiate(&b->aexec, gr, nullptr, nullptr, 0), "graph instantiate"));
        b->a_rho = rho;
        b->a_gE = grad_E;
        b->a_L = L;
        b->a_lam0 = lam0;
        b->a_nb = nb;
        b->a_lpr = b->lpr_adj;
        b->a_ft[0] = FT.row_ptr;
        b->a_ft[1] = FT.col;
        b->a_ft[2] = FT.val;
        b->a_prec = b->precision;
        b->a_h = lh;
    }
    {
        ProfScope ps("batch_adjoint", st);
        GS_TRY(check_hip(hipGraphLaunch(b->aexec, st), "graph launch"));
    }
    if (grad_F || grad_rho) {
        ProfScope ps("batch_sddmm", st);
        const int max_C = *std::max_element(b->scene_cols.begin(), b->scene_cols.end());
        GS_TRY(launch_ragged_sddmm(b->dev(), b->F->csr(), nb, vals, max_C, b->Bt.as<float>(), L, rho, grad_F, grad_rho,
                                   b->counter.as<uint32_t>(), st));
    }
    return GSRAD_OK;
}

gsrad_status gsrad_batch_set_precision(gsrad_batch *b, int32_t precision) {
    if (!b) return einval("gsrad_batch_set_precision: null batch");
    if (precision != GSRAD_FP32 && precision != GSRAD_BF16)
        return einval("gsrad_batch_set_precision: precision must be GSRAD_FP32 or GSRAD_BF16");
    if (precision != b->precision) {
        b->drop_graph();
        b->precision = precision;
        b->nb = -1;   // a forward solve of the new precision must come first
    }
    return GSRAD_OK;
}

gsrad_status gsrad_batch_set_lanes(gsrad_batch *b, int32_t lanes_bounce, int32_t lanes_adjoint) {
    if (!b) return einval("gsrad_batch_set_lanes: null batch");
    for (int v : {lanes_bounce, lanes_adjoint})
        if (v != 0 && v != 16 && v != 32 && v != 64)
            return einval("gsrad_batch_set_lanes: lanes per row must be 0 (tuned), 16, 32 or 64");
    b->force_fwd = lanes_bounce;
    b->force_adj = lanes_adjoint;
    // the next solve / backward takes the forced (or re-tuned) shape
    b->lpr_fwd = lanes_bounce;
    b->lpr_adj = lanes_adjoint;
    b->drop_graph();
    return GSRAD_OK;
}

// ---------------------------------------------------------------------------
// Monte-Carlo TD(0) solver (Sec. 7, App. D)
// ---------------------------------------------------------------------------
gsrad_status gsrad_mc_create(const gsrad_bvh *bvh, int32_t groups, int32_t kmeans_iters, gsrad_mc **mc,
                             void *stream) {
    if (!bvh || !mc) return einval("gsrad_mc_create: null argument");
    GS_TRY(usable(bvh, "gsrad_mc_create"));
    const int64_t n = bvh->n;
    int G = groups > 0 ? groups : (int)std::lround(std::sqrt((double)n));
    if (G < 1 || G > n || G > (1 << 20)) return einval("gsrad_mc_create: groups must be in [1, min(n, 2^20)]");
    if (kmeans_iters < 1 || kmeans_iters > 100) return einval("gsrad_mc_create: kmeans_iters must be in [1, 100]");
    hipStream_t st = S(stream);
    gsrad_mc *h = new gsrad_mc();
    auto fail = [&](gsrad_status e) {
        delete h;
        return e;
    };
    gsrad_status e;
#define ENS(buf, bytes, what) \
    if ((e = h->buf.ensure((size_t)(bytes), what)) != GSRAD_OK) return fail(e);
    ENS(cent, (size_t)G * 12, "group centres");
    ENS(gnrm, (size_t)G * 12, "group normals");
    ENS(L, (size_t)G * 4, "group luminance");
    ENS(key, n * 4, "k-means keys");
    ENS(ids, n * 4, "k-means ids");
    ENS(skey, n * 4, "k-means keys");
    ENS(members, n * 4, "group members");
    ENS(count, (size_t)G * 4, "group counts");
    ENS(goff, ((size_t)G + 1) * 8, "group offsets");
    ENS(rtemp, radix_temp_bytes(n), "k-means sort temp");
    ENS(stemp, scan_temp_bytes(std::max<int64_t>(n, G)), "scan temp");
    ENS(err, 64, "flags");
#undef ENS
    if ((e = check_hip(hipMemsetAsync(h->err.p, 0, 64, st), "flags")) != GSRAD_OK) return fail(e);
    if ((e = check_hip(hipMemsetAsync(h->gnrm.p, 0, (size_t)G * 12, st), "group normals")) != GSRAD_OK) return fail(e);
    gsrad::McBuffers m = h->mb();
    if ((e = mc_kmeans(bvh->dev(), G, kmeans_iters, m, st)) != GSRAD_OK) return fail(e);
    float b[8];
    if ((e = check_hip(hipStreamSynchronize(st), "mc sync")) != GSRAD_OK) return fail(e);
    if ((e = check_hip(hipStreamSynchronize(bvh->stream), "mc sync")) != GSRAD_OK) return fail(e);
    if ((e = check_hip(hipMemcpy(b, bvh->B.bounds, sizeof(b), hipMemcpyDeviceToHost), "bounds")) != GSRAD_OK)
        return fail(e);
    h->bvh = bvh;
    h->gen = bvh->gen;
    h->n = n;
    h->G = G;
    h->rmin2 = (0.01f * b[7]) * (0.01f * b[7]);
    if (*mc) delete *mc;
    *mc = h;
    return GSRAD_OK;
}

static gsrad_status mc_ready(gsrad_mc *mc, int Lt, int K, const char *fn) {
    if (!mc->bvh || mc->bvh->n != mc->n || mc->bvh->gen != mc->gen) {
        set_error("%s: the BVH changed since gsrad_mc_create", fn);
        return GSRAD_ESTATE;
    }
    if (Lt < 1 || !valid_K(K)) {
        set_error("%s: bad n_lights or K", fn);
        return GSRAD_EINVAL;
    }
    const size_t row = (size_t)mc->n * Lt * K * 3 * 4;
    for (DevBuf *b : {&mc->S, &mc->S2, &mc->B, &mc->delta}) GS_TRY(b->ensure(row, "mc state"));
    GS_TRY(mc->var.ensure((size_t)mc->n * 4, "mc variance"));
    GS_TRY(mc->D.ensure((size_t)mc->n * 4, "mc visits"));
    GS_TRY(mc->q.ensure((size_t)mc->n * 4, "mc weights"));
    GS_TRY(mc->maxbits.ensure(64, "mc max"));
    GS_TRY(mc->recv.ensure((size_t)mc->n * 4, "mc receivers"));
    GS_TRY(mc->cdf.ensure(((size_t)mc->n + 1) * 8, "mc cdf"));
    return GSRAD_OK;
}

gsrad_status gsrad_mc_estimate(gsrad_mc *mc, const float *lambda, const float *rho, const float *E, const float *B,
                               int32_t n_lights, int32_t K, uint64_t seed, int32_t step, float *delta_out,
                               void *stream) {
    if (!mc || !lambda || !rho || !E || !B || !delta_out) return einval("gsrad_mc_estimate: null argument");
    GS_TRY(mc_ready(mc, n_lights, K, "gsrad_mc_estimate"));
    gsrad::McBuffers m = mc->mb();
    return mc_step(mc->bvh->dev(), m, mc->G, mc->rmin2, lambda, rho, E, B, n_lights, K, seed, step, nullptr,
                   delta_out, mc->err.as<int>(), S(stream));
}

gsrad_status gsrad_mc_solve(gsrad_mc *mc, const float *lambda, const float *rho, const float *E, int32_t n_lights,
                            int32_t K, int32_t steps, uint64_t seed, float *B_out, uint32_t *visits_out,
                            void *stream) {
    if (!mc || !lambda || !rho || !E || !B_out) return einval("gsrad_mc_solve: null argument");
    if (steps < 1 || steps > (1 << 20)) return einval("gsrad_mc_solve: steps must be in [1, 2^20]");
    GS_TRY(mc_ready(mc, n_lights, K, "gsrad_mc_solve"));
    hipStream_t st = S(stream);
    gsrad::McBuffers m = mc->mb();
    {
        ProfScope ps("mc_solve", st);
        GS_TRY(mc_solve(mc->bvh->dev(), m, mc->G, mc->rmin2, lambda, rho, E, n_lights, K, steps, seed, B_out,
                        mc->err.as<int>(), st));
    }
    if (visits_out)
        GS_TRY(check_hip(hipMemcpyAsync(visits_out, mc->D.p, (size_t)mc->n * 4, hipMemcpyDeviceToDevice, st),
                         "visits copy"));
    return GSRAD_OK;
}

void gsrad_mc_destroy(gsrad_mc *mc) { delete mc; }

void gsrad_batch_destroy(gsrad_batch *batch) { delete batch; }

}  // extern "C"
