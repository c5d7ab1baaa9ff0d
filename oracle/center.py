"""FP64 oracle of the centre-to-centre form factors with a learnable scale
(Sec. 8, Eq. radiosity-approx-1 and the approximated forward rendering
equation; App. E for the effective area) and of their gradients.

TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the GPU path and never imports it.

For every listed pair (i, j) (in practice the pairs the ray cast recorded as
visible, Sec. 6), the decay between the centres, in the scalar Lambertian
form of the transport (F = V / pi):
    F_ij = lambda_j A_j T_ij |n_i . w| |n_j . w| / (pi r^2),  w = (p_j - p_i)/r
with A_j = int alpha_j dA (App. E closed form), T_ij the product of (1 - alpha)
over the surfels other than i and j that the open segment between the centres
crosses, and lambda_j > 0 the per-surfel scale of Sec. 8.

Readings: both faces occlude along the segment; its ends are trimmed by
t_eps / r (the segment starts and ends on the surfels' own planes, where
coplanar neighbours would otherwise register at t = 0 or 1); the paper's
absolute values |n . w| make the pair two-sided.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from .oracle import (OPACITY_MAX, _nthreads, _ptr, _SceneRef, clamp_opacity, default_t_eps, effective_area, lib,
                     opacity_constant)

FIELDS = ("px", "py", "pz", "tux", "tuy", "tuz", "tvx", "tvy", "tvz", "nx", "ny", "nz", "su", "sv", "opacity")


def _bind():
    L = lib()
    if not hasattr(L, "_center_bound"):
        P = ctypes.POINTER
        from .oracle import _Scene
        L.orc_center_ff.argtypes = [P(_Scene), P(ctypes.c_int64), P(ctypes.c_int32), ctypes.c_int64,
                                    P(ctypes.c_double), P(ctypes.c_double), ctypes.c_float, P(ctypes.c_double),
                                    P(ctypes.c_double), ctypes.c_int32]
        L.orc_center_backward.argtypes = [P(_Scene), P(ctypes.c_int64), P(ctypes.c_int32), ctypes.c_int64,
                                          P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double), ctypes.c_float,
                                          P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int32]
        L._center_bound = True
    return L


def area_and_derivative(surfels):
    """A_j (App. E) and dA_j/do_j (0 where the opacity clamp is active):
    A = (2 pi / 3.4) s_u s_v Ein(c), dEin/dc = (1 - e^-c)/c, dc/do = 1/(1 - o)."""
    su = np.asarray(surfels["su"], np.float64)
    sv = np.asarray(surfels["sv"], np.float64)
    o_raw = np.asarray(surfels["opacity"], np.float32)
    A = effective_area(surfels["su"], surfels["sv"], surfels["opacity"])
    c = opacity_constant(o_raw)
    o = clamp_opacity(o_raw).astype(np.float64)
    dEin = np.where(c > 1e-12, -np.expm1(-c) / np.where(c > 1e-12, c, 1.0), 1.0)
    inside = (o_raw > 0) & (o_raw < OPACITY_MAX)
    dA = np.where(inside, (2.0 * np.pi / 3.4) * su * sv * dEin / (1.0 - o), 0.0)
    return A, dA


def _pairs(rows, cols):
    r = np.ascontiguousarray(np.asarray(rows, np.int64))
    c = np.ascontiguousarray(np.asarray(cols, np.int32))
    assert r.shape == c.shape
    return r, c


def center_ff(surfels, rows, cols, lam, t_eps: Optional[float] = None, n_threads: Optional[int] = None):
    """F values and segment transmittances for the listed pairs."""
    sc = _SceneRef(surfels)
    r, c = _pairs(rows, cols)
    lam = np.ascontiguousarray(np.asarray(lam, np.float64))
    A, _ = area_and_derivative(surfels)
    A = np.ascontiguousarray(A)
    if t_eps is None:
        t_eps = default_t_eps(surfels)
    F = np.zeros(r.shape[0])
    T = np.zeros(r.shape[0])
    _bind().orc_center_ff(sc.ref, _ptr(r, ctypes.c_int64), _ptr(c, ctypes.c_int32), r.shape[0],
                          _ptr(lam, ctypes.c_double), _ptr(A, ctypes.c_double), float(t_eps),
                          _ptr(F, ctypes.c_double), _ptr(T, ctypes.c_double), _nthreads(n_threads))
    return F, T


def center_backward(surfels, rows, cols, lam, G, t_eps: Optional[float] = None, n_threads: Optional[int] = None):
    """Gradients of sum_e G_e F_e: (g_lambda [n], {field: gradient [n]} for
    the 15 surfel fields)."""
    sc = _SceneRef(surfels)
    n = sc.n
    r, c = _pairs(rows, cols)
    lam = np.ascontiguousarray(np.asarray(lam, np.float64))
    A, dA = area_and_derivative(surfels)
    A, dA = np.ascontiguousarray(A), np.ascontiguousarray(dA)
    G = np.ascontiguousarray(np.asarray(G, np.float64))
    if t_eps is None:
        t_eps = default_t_eps(surfels)
    gl = np.zeros(n)
    gr = np.zeros(n * 15)
    _bind().orc_center_backward(sc.ref, _ptr(r, ctypes.c_int64), _ptr(c, ctypes.c_int32), r.shape[0],
                                _ptr(lam, ctypes.c_double), _ptr(A, ctypes.c_double), _ptr(dA, ctypes.c_double),
                                float(t_eps), _ptr(G, ctypes.c_double), _ptr(gl, ctypes.c_double),
                                _ptr(gr, ctypes.c_double), _nthreads(n_threads))
    gr = gr.reshape(n, 15)
    return gl, {f: gr[:, k] for k, f in enumerate(FIELDS)}
