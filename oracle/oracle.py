"""FP64 CPU oracle for the surfel radiosity hot path.

TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the GPU path (the package ``paper_2509_18497_amd``) and never imports it.

Paper: "Differentiable Light Transport with Gaussian Surfels via Adapted
Radiosity" (Jiang et al., ACM TOG 2025).  Each function cites the passage it
follows.  The ray casting (visibility, form-factor rows, direct light,
compositing backward) lives in ``gsrad_oracle.c``; this module holds the
linear-algebra steps in FP64 NumPy/SciPy:

* ``bounce``   -- Eq. final-radiosity for a Lambertian scalar transport,
  B = E + diag(rho) F B, iterated from B^(0) = E (B^(k+1) = E + rho*(F B^(k)));
* ``adjoint``  -- the exact adjoint of that n-step map (Eq. final_dL_dE in
  its division-free form u = g + F^T (rho * u), truncated the same way),
  with the BRDF gradient (Eq. final-dl-dbrdf) and the per-entry gradient of
  the decay term (Eq. dl-dgeo-0) on F's sparsity pattern;
* ``effective_area`` -- App. E closed form (2 pi / 3.4) s_u s_v Ein(c).

Array layout: E and B are [N, Lt, K, 3] (surfel, light, SH coefficient,
RGB), handled as [N, C] with C = Lt*K*3 and colour = column % 3.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.special

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsrad_oracle.so")
OPACITY_MAX = np.float32(0.9999)
SOA = ("px", "py", "pz", "tux", "tuy", "tuz", "tvx", "tvy", "tvz", "nx", "ny", "nz", "su", "sv", "opacity")

_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "gsrad_oracle.c")
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
            from . import build as _b  # noqa: F401  (package-relative when imported as oracle.oracle)
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.orc_philox4x64_10.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint64), P(ctypes.c_uint64)]
        L.orc_ray_direction.argtypes = [P(_Scene), ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64, P(ctypes.c_float)]
        L.orc_ray_direction.restype = ctypes.c_int
        L.orc_default_t_eps.argtypes = [P(_Scene)]
        L.orc_default_t_eps.restype = ctypes.c_float
        L.orc_trace_ray.argtypes = [P(_Scene), ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_int64, P(ctypes.c_float), P(ctypes.c_int32),
                                    P(ctypes.c_int8), P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_float),
                                    P(ctypes.c_int64), P(ctypes.c_float)]
        L.orc_trace_ray.restype = ctypes.c_int64
        L.orc_exp_fx.argtypes = [ctypes.c_float]
        L.orc_exp_fx.restype = ctypes.c_float
        L.orc_ff_rows.argtypes = [P(_Scene), P(ctypes.c_int64), ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_int64, P(ctypes.c_int32),
                                  P(ctypes.c_double), P(ctypes.c_int64), P(ctypes.c_double), ctypes.c_int32]
        L.orc_ff_rows.restype = ctypes.c_int
        L.orc_direct_light.argtypes = [P(_Scene), P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float),
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P(ctypes.c_int64),
                                       ctypes.c_int64, P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int32]
        L.orc_opacity_backward.argtypes = [P(_Scene), P(ctypes.c_int64), ctypes.c_int64, P(ctypes.c_int64),
                                           P(ctypes.c_int32), P(ctypes.c_double), ctypes.c_int32, ctypes.c_uint64,
                                           ctypes.c_float, ctypes.c_float, P(ctypes.c_double), ctypes.c_int32]
        L.orc_geometry_backward.argtypes = L.orc_opacity_backward.argtypes
        L.orc_direct_light_backward.argtypes = [P(_Scene), P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float),
                                                ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P(ctypes.c_double),
                                                P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
                                                P(ctypes.c_double), ctypes.c_int32]
        _lib = L
    return _lib


class _Scene(ctypes.Structure):
    _fields_ = [(f, ctypes.POINTER(ctypes.c_float)) for f in
                ("px", "py", "pz", "tux", "tuy", "tuz", "tvx", "tvy", "tvz", "nx", "ny", "nz", "su", "sv", "op")] + \
               [("n", ctypes.c_int64)]


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class _SceneRef:
    """Keeps the FP32 arrays alive while C holds pointers to them."""

    def __init__(self, surfels):
        self.arrays = [np.ascontiguousarray(surfels[f], dtype=np.float32) for f in SOA]
        n = self.arrays[0].shape[0]
        for a in self.arrays:
            assert a.shape == (n,)
        self.s = _Scene(*[_ptr(a, ctypes.c_float) for a in self.arrays], n)
        self.n = n

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _nthreads(n_threads):
    if n_threads is not None:
        return int(n_threads)
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# random numbers and rays
# ---------------------------------------------------------------------------
def philox4x64_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    """One Philox4x64-10 block (Salmon et al., SC'11)."""
    c = np.asarray(ctr, np.uint64)
    k = np.asarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(c, ctypes.c_uint64), _ptr(k, ctypes.c_uint64), _ptr(out, ctypes.c_uint64))
    return out


def ray_direction(surfels, i: int, r: int, seed: int, tag: int = 0):
    """Cosine-weighted hemisphere direction of ray r of receiver i (App. B
    hemisphere integral; Malley's method); returns (d[3] float32, attempts)."""
    sc = _SceneRef(surfels)
    d = np.zeros(3, np.float32)
    a = lib().orc_ray_direction(sc.ref, int(i), int(r), int(seed), int(tag), _ptr(d, ctypes.c_float))
    return d, a


def default_t_eps(surfels) -> np.float32:
    sc = _SceneRef(surfels)
    return np.float32(lib().orc_default_t_eps(sc.ref))


def trace_ray(surfels, i: int, r: int, seed: int, t_eps: float, t_min: float, cap: int = 4096):
    """Every hit of one ray in (t, j) order with FP64 alpha and the
    transmittance in front of it (Eq. L_I), plus the FP32 transmittance of
    the compositing cut (D_stop); n_comp hits are composited."""
    sc = _SceneRef(surfels)
    t = np.zeros(cap, np.float32)
    j = np.zeros(cap, np.int32)
    fr = np.zeros(cap, np.int8)
    al = np.zeros(cap, np.float64)
    T = np.zeros(cap, np.float64)
    T32 = np.zeros(cap, np.float32)
    nc = ctypes.c_int64(0)
    d = np.zeros(3, np.float32)
    m = lib().orc_trace_ray(sc.ref, int(i), int(r), int(seed), float(t_eps), float(t_min), cap,
                            _ptr(t, ctypes.c_float), _ptr(j, ctypes.c_int32), _ptr(fr, ctypes.c_int8),
                            _ptr(al, ctypes.c_double), _ptr(T, ctypes.c_double), _ptr(T32, ctypes.c_float),
                            ctypes.byref(nc), _ptr(d, ctypes.c_float))
    if m < 0:
        return trace_ray(surfels, i, r, seed, t_eps, t_min, cap=-m)
    return {"t": t[:m], "j": j[:m], "front": fr[:m].astype(bool), "alpha": al[:m], "T": T[:m],
            "T32": T32[:m], "n_comp": int(nc.value), "d": d}


# ---------------------------------------------------------------------------
# form factors
# ---------------------------------------------------------------------------
def ff_rows(surfels, receivers, R: int, seed: int, t_eps: float, t_min: float = 1e-4, topk: int = 0,
            n_threads: Optional[int] = None, cap_row: Optional[int] = None):
    """Form-factor rows for the listed receivers (Eq. final-radiosity with a
    Lambertian receiver; F_ij = (1/R) sum of composited front-hit weights).
    Returns (row_ptr, cols, vals, diag) over the listed receivers, columns
    ascending, plus diag[k] = (front sum before truncation, back-face sum,
    (1/R) sum (1 - T_ray), max composited hits on one ray)."""
    sc = _SceneRef(surfels)
    recv = np.ascontiguousarray(np.asarray(receivers, np.int64))
    nr = recv.shape[0]
    cap = int(cap_row) if cap_row is not None else (topk if topk > 0 else 2048)
    while True:
        cols = np.zeros(max(nr * cap, 1), np.int32)
        vals = np.zeros(max(nr * cap, 1), np.float64)
        cnt = np.zeros(max(nr, 1), np.int64)
        diag = np.zeros(max(nr * 4, 1), np.float64)
        st = lib().orc_ff_rows(sc.ref, _ptr(recv, ctypes.c_int64), nr, int(R), int(seed), float(t_eps),
                               float(t_min), int(topk), cap, _ptr(cols, ctypes.c_int32), _ptr(vals, ctypes.c_double),
                               _ptr(cnt, ctypes.c_int64), _ptr(diag, ctypes.c_double), _nthreads(n_threads))
        if st == 0:
            break
        cap = int(cnt[:nr].max())
    cnt = cnt[:nr]
    row_ptr = np.zeros(nr + 1, np.int64)
    row_ptr[1:] = np.cumsum(cnt)
    sel = (np.arange(cap)[None, :] < cnt[:, None]).ravel()
    return row_ptr, cols[: nr * cap][sel], vals[: nr * cap][sel], diag[: nr * 4].reshape(nr, 4)


def ff_matrix(surfels, R: int, seed: int, t_eps: Optional[float] = None, t_min: float = 1e-4, topk: int = 0,
              n_threads: Optional[int] = None):
    """The full N x N form-factor matrix as FP64 scipy CSR (brute force)."""
    n = surfels["px"].shape[0]
    if t_eps is None:
        t_eps = default_t_eps(surfels)
    rp, c, v, diag = ff_rows(surfels, np.arange(n), R, seed, t_eps, t_min, topk, n_threads)
    F = sp.csr_matrix((v, c, rp), shape=(n, n))
    return F, diag


# ---------------------------------------------------------------------------
# surfel quantities
# ---------------------------------------------------------------------------
def clamp_opacity(o) -> np.ndarray:
    """Peak opacity clamped to [0, 0.9999] (FP32), so c = -ln(1-o) is finite."""
    o = np.asarray(o, np.float32)
    return np.minimum(np.maximum(o, np.float32(0.0)), OPACITY_MAX)


def opacity_constant(o) -> np.ndarray:
    """c = -ln(1 - o): App. E writes alpha = 1 - exp(-0.03279 (g G)^3.4);
    with G^3.4 = exp(-1.7 r^2) the peak alpha(0) = o fixes 0.03279 g^3.4."""
    return -np.log1p(-clamp_opacity(o).astype(np.float64))


def ein(c) -> np.ndarray:
    """Entire exponential integral Ein(c) = int_0^c (1 - e^-y)/y dy
    = E1(c) + ln c + Euler gamma (App. E)."""
    c = np.asarray(c, np.float64)
    out = np.zeros_like(c)
    small = c < 1e-3
    cs = c[small]
    out[small] = cs - cs ** 2 / 4 + cs ** 3 / 18 - cs ** 4 / 96
    cl = c[~small]
    out[~small] = scipy.special.exp1(cl) + np.log(cl) + np.euler_gamma
    return out


def effective_area(su, sv, opacity) -> np.ndarray:
    """int_P alpha dA = (2 pi / 3.4) s_u s_v Ein(c)  (App. E closed form)."""
    return (2.0 * np.pi / 3.4) * np.asarray(su, np.float64) * np.asarray(sv, np.float64) * ein(opacity_constant(opacity))


def rho(opacity, albedo) -> np.ndarray:
    """rho_i = alpha_i(p_i) a_i: the receiver opacity absorbed into the BRDF
    (Sec. 5.3, text after Eq. before-final-radiosity); with a Lambertian BRDF
    (App. A, c_00 = 4 a) the scalar transfer per colour is o_i a_i."""
    return clamp_opacity(opacity).astype(np.float64)[:, None] * np.asarray(albedo, np.float64)


def direct_light(surfels, albedo, light_pos, light_I, K: int, t_eps: Optional[float] = None, receivers=None,
                 n_threads: Optional[int] = None, return_T: bool = False):
    """E [n_recv, Lt, K, 3] from point lights (Eq. forward rendering
    equation, direct illumination), DC coefficient only."""
    sc = _SceneRef(surfels)
    n = sc.n
    if t_eps is None:
        t_eps = default_t_eps(surfels)
    recv = np.ascontiguousarray(np.arange(n, dtype=np.int64) if receivers is None else np.asarray(receivers, np.int64))
    lp = np.ascontiguousarray(np.asarray(light_pos, np.float32).reshape(-1, 3))
    li = np.ascontiguousarray(np.asarray(light_I, np.float32).reshape(-1))
    alb = np.ascontiguousarray(np.asarray(albedo, np.float32).reshape(-1, 3))
    Lt = lp.shape[0]
    E = np.zeros((recv.shape[0], Lt, K, 3), np.float64)
    T = np.zeros((recv.shape[0], Lt), np.float64)
    lib().orc_direct_light(sc.ref, _ptr(alb, ctypes.c_float), _ptr(lp, ctypes.c_float), _ptr(li, ctypes.c_float),
                           Lt, int(K), float(t_eps), _ptr(recv, ctypes.c_int64), recv.shape[0],
                           _ptr(E, ctypes.c_double), _ptr(T, ctypes.c_double), _nthreads(n_threads))
    return (E, T) if return_T else E


# ---------------------------------------------------------------------------
# bounces and their adjoint
# ---------------------------------------------------------------------------
def _rho_cols(rho_arr, C):
    rho_arr = np.asarray(rho_arr, np.float64).reshape(-1, 3)
    return np.tile(rho_arr, (1, C // 3))


def reciprocity(F, area):
    """Reciprocity of an operator against the areas (A_i F_ij = A_j F_ji
    for exact form factors: classical radiosity reciprocity, not stated in
    the paper; an invariant of the estimator), over the stored entries of F, the
    mirror entry taken as 0 where F_ji is not stored:
    (sum |A_i F_ij - A_j F_ji| / sum A_i F_ij,
     max |A_i F_ij - A_j F_ji| / max(A_i F_ij, A_j F_ji))."""
    F = sp.csr_matrix(F, dtype=np.float64)
    A = np.asarray(area, np.float64)
    rows = np.repeat(np.arange(F.shape[0]), np.diff(F.indptr))
    cols = F.indices
    a = A[rows] * F.data
    Ft = F.T.tocsr()
    mirror = np.asarray(Ft[rows, cols]).ravel()     # F[j, i]
    b = A[cols] * mirror
    d = np.abs(a - b)
    m = np.maximum(a, b)
    rel = np.where(m > 0, d / np.where(m > 0, m, 1.0), 0.0)
    return (float(d.sum() / a.sum()) if a.sum() > 0 else 0.0), (float(rel.max()) if rel.size else 0.0)


def bounce(F, rho_arr, E, n_bounces: int, keep_tape: bool = False):
    """B^(0) = E, B^(k+1) = E + rho * (F B^(k)), k < n (Eq. final-radiosity,
    scalar Lambertian transfer applied to every SH coefficient and light).
    Returns B^(n) (shape of E) and, if asked, the tape [B^(0..n-1)]."""
    shape = np.shape(E)
    N = shape[0]
    E2 = np.asarray(E, np.float64).reshape(N, -1)
    C = E2.shape[1]
    rc = _rho_cols(rho_arr, C)
    F = sp.csr_matrix(F, dtype=np.float64)
    B = E2.copy()
    tape = []
    for _ in range(n_bounces):
        if keep_tape:
            tape.append(B)
        B = E2 + rc * (F @ B)
    return (B.reshape(shape), tape) if keep_tape else B.reshape(shape)


def adjoint(F, rho_arr, tape, g, chunk: int = 4096, want_grad_F: bool = True, dense_grad_F: bool = False):
    """Exact adjoint of ``bounce`` for a loss with dL/dB^(n) = g:
      lambda^(n) = g,  lambda^(k) = F^T (rho * lambda^(k+1))   (Eq. final_dL_dE,
                                                               division-free)
      grad_E     = sum_{k=0..n} lambda^(k)
      grad_rho   = sum_{k<n} sum_{coef, light} lambda^(k+1) * (F B^(k))   (the
                   truncated counterpart of Eq. final-dl-dbrdf)
      grad_F_ij  = sum_{k<n} <rho_i * lambda_i^(k+1), B_j^(k)>             (decay
                   term of Eq. dl-dgeo-0 per recorded pair (i, j))
    grad_F is returned aligned with F's CSR entries (F.indices order), or
    as None when not wanted.  With dense_grad_F the same sum is returned for
    every pair (i, j) as an [N][N] array (the gradient with respect to a
    dense F) in place of the stored-entry vector."""
    shape = np.shape(g)
    N = shape[0]
    lam = np.asarray(g, np.float64).reshape(N, -1).copy()
    C = lam.shape[1]
    rc = _rho_cols(rho_arr, C)
    F = sp.csr_matrix(F, dtype=np.float64)
    FT = F.T.tocsr()
    grad_E = lam.copy()
    grad_rho = np.zeros((N, 3))
    gF = np.zeros(F.nnz)
    gFd = np.zeros((N, N)) if dense_grad_F else None
    rows = np.repeat(np.arange(N), np.diff(F.indptr))
    for k in range(len(tape) - 1, -1, -1):
        Bk = tape[k]
        Q = F @ Bk
        grad_rho += (lam * Q).reshape(N, -1, 3).sum(axis=1)
        rl = rc * lam
        if dense_grad_F:
            gFd += rl @ Bk.T
        for s in range(0, F.nnz if (want_grad_F and not dense_grad_F) else 0, chunk * 64):
            e = min(F.nnz, s + chunk * 64)
            gF[s:e] += np.einsum("ec,ec->e", rl[rows[s:e]], Bk[F.indices[s:e]])
        lam = FT @ rl
        grad_E += lam
    if dense_grad_F:
        return grad_E.reshape(shape), grad_rho, gFd
    return grad_E.reshape(shape), grad_rho, (gF if want_grad_F else None)


def opacity_backward(surfels, albedo, R: int, seed: int, t_eps: float, t_min: float, gF_rows, grad_rho=None,
                     receivers=None, n_threads: Optional[int] = None):
    """dL/do and dL/da.  The F-part runs the compositing backward over the
    rays of the listed receivers (Eq. dl-dgeo-0, decay term, opacity only);
    gF_rows = (row_ptr, cols, vals) of dL/dF over those receivers.  The
    receiver part follows rho = o a: dL/do_i += sum_c dL/drho_ic a_ic (inside
    the clamp), dL/da = dL/drho * o."""
    sc = _SceneRef(surfels)
    n = sc.n
    recv = np.ascontiguousarray(np.arange(n, dtype=np.int64) if receivers is None else np.asarray(receivers, np.int64))
    gp, gc, gv = gF_rows
    gp = np.ascontiguousarray(np.asarray(gp, np.int64))
    gc = np.ascontiguousarray(np.asarray(gc, np.int32))
    gv = np.ascontiguousarray(np.asarray(gv, np.float64))
    go = np.zeros(n, np.float64)
    lib().orc_opacity_backward(sc.ref, _ptr(recv, ctypes.c_int64), recv.shape[0], _ptr(gp, ctypes.c_int64),
                               _ptr(gc, ctypes.c_int32), _ptr(gv, ctypes.c_double), int(R), int(seed),
                               float(t_eps), float(t_min), _ptr(go, ctypes.c_double), _nthreads(n_threads))
    o = np.asarray(surfels["opacity"], np.float32)
    alb = np.asarray(albedo, np.float64).reshape(-1, 3)
    ga = np.zeros((n, 3))
    if grad_rho is not None:
        inside = (o > 0) & (o < OPACITY_MAX)
        go += np.where(inside, (np.asarray(grad_rho) * alb).sum(axis=1), 0.0)
        ga = np.asarray(grad_rho, np.float64) * clamp_opacity(o).astype(np.float64)[:, None]
    return go, ga


GEOMETRY_FIELDS = ("px", "py", "pz", "tux", "tuy", "tuz", "tvx", "tvy", "tvz", "nx", "ny", "nz", "su", "sv",
                   "opacity")


def geometry_backward(surfels, R: int, seed: int, t_eps: float, t_min: float, gF_rows, receivers=None,
                      n_threads: Optional[int] = None):
    """Gradients of sum G F (ray-cast F of the listed receivers, G given as
    CSR rows over them) with respect to every surfel field: the decay term
    of Eq. dl-dgeo-0 through the compositing weights of the recorded hits,
    the hit points' dependence on the hit surfel's centre, frame and scales,
    and on the receiver's centre and frame (ray origin and direction).
    Returns {field: gradient [n]}."""
    sc = _SceneRef(surfels)
    n = sc.n
    recv = np.ascontiguousarray(np.arange(n, dtype=np.int64) if receivers is None else np.asarray(receivers, np.int64))
    gp, gc, gv = gF_rows
    gp = np.ascontiguousarray(np.asarray(gp, np.int64))
    gc = np.ascontiguousarray(np.asarray(gc, np.int32))
    gv = np.ascontiguousarray(np.asarray(gv, np.float64))
    out = np.zeros(n * 15)
    lib().orc_geometry_backward(sc.ref, _ptr(recv, ctypes.c_int64), recv.shape[0], _ptr(gp, ctypes.c_int64),
                                _ptr(gc, ctypes.c_int32), _ptr(gv, ctypes.c_double), int(R), int(seed),
                                float(t_eps), float(t_min), _ptr(out, ctypes.c_double), _nthreads(n_threads))
    out = out.reshape(n, 15)
    return {f: out[:, k] for k, f in enumerate(GEOMETRY_FIELDS)}


def direct_light_backward(surfels, albedo, light_pos, light_I, grad_E, t_eps: Optional[float] = None,
                          n_threads: Optional[int] = None):
    """Gradients of sum(grad_E * E) through ``direct_light`` (DC part):
    (dL/dlight_pos [Lt, 3], dL/dlight_I [Lt], dL/dalbedo [n, 3],
    {field: dL/dfield [n]} for the receivers' and occluders' surfel fields)."""
    sc = _SceneRef(surfels)
    n = sc.n
    if t_eps is None:
        t_eps = default_t_eps(surfels)
    lp = np.ascontiguousarray(np.asarray(light_pos, np.float32).reshape(-1, 3))
    li = np.ascontiguousarray(np.asarray(light_I, np.float32).reshape(-1))
    alb = np.ascontiguousarray(np.asarray(albedo, np.float32).reshape(-1, 3))
    Lt = lp.shape[0]
    gE = np.ascontiguousarray(np.asarray(grad_E, np.float64))
    K = gE.shape[2]
    g_lp = np.zeros(Lt * 3)
    g_li = np.zeros(Lt)
    g_alb = np.zeros(n * 3)
    gr = np.zeros(n * 15)
    lib().orc_direct_light_backward(sc.ref, _ptr(alb, ctypes.c_float), _ptr(lp, ctypes.c_float),
                                    _ptr(li, ctypes.c_float), Lt, int(K), float(t_eps), _ptr(gE, ctypes.c_double),
                                    _ptr(g_lp, ctypes.c_double), _ptr(g_li, ctypes.c_double),
                                    _ptr(g_alb, ctypes.c_double), _ptr(gr, ctypes.c_double), _nthreads(n_threads))
    gr = gr.reshape(n, 15)
    return g_lp.reshape(Lt, 3), g_li, g_alb.reshape(n, 3), {f: gr[:, k] for k, f in enumerate(GEOMETRY_FIELDS)}
