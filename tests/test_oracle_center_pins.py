"""Pins of the FP64 oracle of the centre-to-centre form factors (Sec. 8,
App. E) and of their gradients, CPU only: closed forms for an unoccluded
pair and a single occluder, the exact coaxial point-to-disc integral as the
discs shrink, and central finite differences of the oracle's own forward
for every surfel field, the scale lambda and the occluders."""
import math

import numpy as np
import pytest
import scipy.integrate

import scenes
from oracle import center
from oracle import oracle as orc


def _alpha(r2, o):
    c = -math.log1p(-o)
    return -math.expm1(-c * math.exp(-1.7 * r2))


def _pair_scene(h, tilt, s_j, o_j, extra=()):
    """Receiver 0 at the origin facing +z; sender 1 at (0, 0, h) facing down,
    tilted by `tilt` about the x axis; extra surfels appended."""
    nj = np.array([0.0, math.sin(tilt), -math.cos(tilt)])
    tu_j = np.array([1.0, 0.0, 0.0])
    tv_j = np.cross(nj, tu_j)
    p = [[0, 0, 0], [0, 0, h]]
    nrm = [[0, 0, 1], nj]
    tu = [[1, 0, 0], tu_j]
    tv = [[0, 1, 0], tv_j]
    su = [0.05, s_j]
    op = [0.9, o_j]
    for e in extra:
        p.append(e["p"]), nrm.append(e["n"]), tu.append(e["tu"]), tv.append(e["tv"]), su.append(e["s"]), op.append(e["o"])
    return scenes.surfels_from_arrays(np.array(p, float), np.array(nrm, float), np.array(tu, float),
                                      np.array(tv, float), su, su, op)


def test_unoccluded_pair_is_the_point_to_disc_closed_form():
    """F = lambda A cos(theta_i) cos(theta_j) / (pi r^2) with the App. E area."""
    for h, tilt, lam in [(1.0, 0.0, 1.0), (2.5, 0.6, 0.7), (0.8, 1.2, 1.9)]:
        sur = _pair_scene(h, tilt, 0.1, 0.8)
        F, T = center.center_ff(sur, [0], [1], np.array([1.0, lam]), t_eps=1e-6)
        A = orc.effective_area(sur["su"][1:], sur["sv"][1:], sur["opacity"][1:])[0]
        assert T[0] == 1.0
        assert abs(F[0] - lam * A * math.cos(tilt) / (math.pi * h * h)) < 1e-6 * F[0]


def test_single_occluder_transmittance_is_one_minus_alpha_at_the_crossing():
    """An occluder at z = h/2 facing +z, its centre offset by (-0.3 s, 0.2 s) in
    its own (t_u, t_v): the axis crosses it at (u, w) = (0.3, -0.2), so
    T = 1 - alpha(u^2 + w^2)."""
    h, s, o = 1.0, 0.2, 0.7
    ang = 0.4
    tu = np.array([math.cos(ang), math.sin(ang), 0.0])
    tv = np.array([-math.sin(ang), math.cos(ang), 0.0])
    p = -0.3 * s * tu + 0.2 * s * tv + np.array([0, 0, h / 2])
    occ = {"p": p, "n": [0, 0, 1], "tu": tu, "tv": tv, "s": s, "o": o}
    sur = _pair_scene(h, 0.0, 0.1, 0.8, extra=[occ])
    F, T = center.center_ff(sur, [0, 1], [1, 0], np.ones(3), t_eps=1e-6)
    ref = 1.0 - _alpha(0.3 ** 2 + 0.2 ** 2, float(np.float32(o)))
    assert abs(T[0] - ref) < 1e-6 and abs(T[1] - ref) < 1e-6


def test_small_discs_approach_the_exact_point_to_disc_integral():
    """Coaxial sender of scale s at height h: the exact decay of the Gaussian
    disc seen from the receiver's centre is 2 h^2 int alpha(rho/s) rho /
    (h^2 + rho^2)^2 drho (cos factors included); the centre-to-centre value
    differs from it by O((s/h)^2)."""
    h = 1.0
    for s in (0.01, 0.02, 0.04):
        sur = _pair_scene(h, 0.0, s, 0.8)
        F, _ = center.center_ff(sur, [0], [1], np.ones(2), t_eps=1e-7)
        o = float(np.float32(0.8))
        exact, _ = scipy.integrate.quad(lambda r: _alpha((r / s) ** 2, o) * r / (h * h + r * r) ** 2, 0, 3 * s,
                                        epsabs=0, epsrel=1e-12, limit=200)
        exact *= 2 * h * h
        # the App. E area integrates alpha over the whole plane; the 3-sigma
        # cut drops at most c e^(-15.3) / 3.4 of it
        assert abs(F[0] / exact - 1) < 5 * (s / h) ** 2 + 1e-6, s


def _grad_scene():
    """Receivers and senders on two facing planes (supports not overlapping
    their neighbours') with a few broad surfels between them, every pair's
    segment crossing occluders well inside their support."""
    rng = np.random.default_rng(4)
    p, nrm, tu, tv, s, o = [], [], [], [], [], []

    def add(pp, nn, ss, oo):
        nn = np.asarray(nn, float) / np.linalg.norm(nn)
        a, b = scenes.onb_from_normal(nn[None, :])
        p.append(pp), nrm.append(nn), tu.append(a[0]), tv.append(b[0]), s.append(ss), o.append(oo)

    for k in range(3):
        add([0.1 * k, 0.0, 0.0], [0.05 * k, 0.02, 1.0], 0.015, 0.9)         # receivers 0..2
    for k in range(3):
        add([0.1 * k - 0.05, 0.03, 1.0], [0.02, -0.03 * k, -1.0], 0.015, 0.8)  # senders 3..5
    for k in range(4):
        add([0.05 + 0.02 * rng.uniform(-1, 1), 0.01 * rng.uniform(-1, 1), 0.3 + 0.15 * k],
            [0.2 * rng.uniform(-1, 1), 0.2 * rng.uniform(-1, 1), 1.0], 0.35, 0.5)  # broad occluders 6..9
    sur = scenes.surfels_from_arrays(np.array(p), np.array(nrm), np.array(tu), np.array(tv), s, s, o)
    rows = np.array([0, 0, 1, 1, 2, 2, 3, 4], np.int64)
    cols = np.array([3, 4, 4, 5, 3, 5, 0, 2], np.int32)
    return sur, rows, cols


def test_gradients_match_central_differences():
    """dL/dlambda and dL/d(every surfel field) of L = sum_e G_e F_e against
    central differences of the oracle's forward.  Each step is the actual
    FP32 change of the perturbed input; steps are large enough that the FP32
    rounding of the inputs and of p_j - p_i stays below 1e-4 of the quotient."""
    sur, rows, cols = _grad_scene()
    n = sur["px"].shape[0]
    lam = np.linspace(0.8, 1.4, n)
    G = np.random.default_rng(5).standard_normal(rows.size)
    te = 1e-6
    F0, T0 = center.center_ff(sur, rows, cols, lam, t_eps=te)
    assert np.all(T0 < 0.97) and np.all(T0 > 0.01)             # every segment is occluded
    gl, gf = center.center_backward(sur, rows, cols, lam, G, t_eps=te)

    def L(s_, lam_):
        return float(np.sum(G * center.center_ff(s_, rows, cols, lam_, t_eps=te)[0]))

    for k in range(n):
        h = 1e-4 * lam[k]
        lp, lm = lam.copy(), lam.copy()
        lp[k] += h
        lm[k] -= h
        fd = (L(sur, lp) - L(sur, lm)) / (2 * h)
        assert abs(fd - gl[k]) <= 1e-6 * (abs(fd) + np.max(np.abs(gl))), ("lambda", k)
    scale = max(np.max(np.abs(v)) for v in gf.values())
    checked = 0
    for f in center.FIELDS:
        for k in range(n):
            x0 = np.float32(sur[f][k])
            step = np.float32(max(abs(float(x0)), 0.05) * 2e-3)
            sp_, sm_ = dict(sur), dict(sur)
            sp_[f] = sur[f].copy()
            sm_[f] = sur[f].copy()
            sp_[f][k] = np.float32(x0 + step)
            sm_[f][k] = np.float32(x0 - step)
            if f == "opacity" and not (0 < float(sm_[f][k]) and float(sp_[f][k]) < 0.9999):
                continue
            d = float(sp_[f][k]) - float(sm_[f][k])
            fd = (L(sp_, lam) - L(sm_, lam)) / d
            assert abs(fd - gf[f][k]) <= 2e-3 * (abs(fd) + 1e-3 * scale), (f, k, fd, gf[f][k])
            checked += 1
    assert checked > 140
