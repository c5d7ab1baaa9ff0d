"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Every test here runs on the CPU only.  None of them re-types the oracle's own
formula: each compares it with an independent route (a library generator,
a closed form, a quadrature, a linear solve, finite differences, or a
distributional law).
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.sparse as sp
import scipy.stats

import scenes


# ---------------------------------------------------------------------------
# helpers: analytic two-surfel set-ups
# ---------------------------------------------------------------------------
def _alpha_profile(r2, o):
    """App. E opacity profile with c = -ln(1-o): 1 - exp(-c exp(-1.7 r^2))."""
    c = -math.log1p(-o)
    return -np.expm1(-c * np.exp(-1.7 * r2))


def _two_surfels(p_j, n_j, s_j, o_j, s_i=0.05, o_i=0.9, spin=0.3):
    """Receiver 0 at the origin facing +z; sender 1 at p_j facing n_j."""
    n_j = np.asarray(n_j, float) / np.linalg.norm(n_j)
    tu_j, tv_j = scenes.onb_from_normal(n_j[None, :])
    ca, sa = math.cos(spin), math.sin(spin)
    tu_j, tv_j = ca * tu_j + sa * tv_j, -sa * tu_j + ca * tv_j
    p = np.array([[0.0, 0.0, 0.0], p_j], float)
    nrm = np.array([[0.0, 0.0, 1.0], n_j])
    tu = np.array([[1.0, 0.0, 0.0], tu_j[0]])
    tv = np.array([[0.0, 1.0, 0.0], tv_j[0]])
    return scenes.surfels_from_arrays(p, nrm, tu, tv, [s_i, s_j[0]], [s_i, s_j[1]], [o_i, o_j])


def _exact_point_to_disc(sur, j=1, n_rho=160, n_phi=256):
    """(1/pi) * integral over sender j's 3-sigma disc of alpha cos_i |cos_j| / r^2
    (FP64 Gauss-Legendre in polar (rho, phi) on the (u, v) plane): the
    expectation of the composited weight of a cosine-weighted ray from the
    origin (receiver normal +z).  Also returns E[w^2] for the MC error."""
    f = {k: np.float64(v[j]) for k, v in sur.items()}
    p = np.array([f["px"], f["py"], f["pz"]])
    tu = np.array([f["tux"], f["tuy"], f["tuz"]])
    tv = np.array([f["tvx"], f["tvy"], f["tvz"]])
    nj = np.array([f["nx"], f["ny"], f["nz"]])
    xr, wr = np.polynomial.legendre.leggauss(n_rho)
    xp, wp = np.polynomial.legendre.leggauss(n_phi)
    rho = 1.5 * (xr + 1.0)
    phi = math.pi * (xp + 1.0)
    R_, P_ = np.meshgrid(rho, phi, indexing="ij")
    W = np.outer(wr * 1.5, wp * math.pi) * R_
    u, v = R_ * np.cos(P_), R_ * np.sin(P_)
    x = p[None, None, :] + (f["su"] * u)[..., None] * tu + (f["sv"] * v)[..., None] * tv
    r = np.linalg.norm(x, axis=-1)
    cos_i = x[..., 2] / r
    cos_j = np.abs(x @ nj) / r
    a = _alpha_profile(u * u + v * v, float(f["opacity"]))
    jac = f["su"] * f["sv"]
    dens = np.where(cos_i > 0, cos_i * cos_j / (r * r) / math.pi, 0.0) * jac
    return float(np.sum(W * dens * a)), float(np.sum(W * dens * a * a))


# ---------------------------------------------------------------------------
# Philox and rays
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ctr,key", [((1, 0, 0, 0), (0, 0)), ((5, 7, 9, 11), (13, 17)),
                                     ((2 ** 64 - 1, 3, 2 ** 40, 1), (2 ** 63, 12345)),
                                     ((77, 1000000, 3, 0), (3, 0))])
def test_philox4x64_10_matches_numpy(orc, ctr, key):
    """numpy.random.Philox is an independent Philox4x64-10; its first block
    is the block of (counter + 1)."""
    prev = list(ctr)
    prev[0] -= 1
    g = np.random.Philox(counter=np.array(prev, np.uint64), key=np.array(key, np.uint64))
    assert np.array_equal(g.random_raw(4).astype(np.uint64), orc.philox4x64_10(ctr, key))


def test_philox_stream_matches_numpy_many_counters(orc):
    g = np.random.Philox(counter=np.array([0, 9, 8, 7], np.uint64), key=np.array([42, 0], np.uint64))
    ref = g.random_raw(4 * 256).reshape(256, 4)
    for k in range(256):
        assert np.array_equal(ref[k], orc.philox4x64_10((k + 1, 9, 8, 7), (42, 0)))


def test_ray_directions_are_cosine_distributed(orc):
    """Malley's method: cos^2(theta) = 1 - x^2 - y^2 is U[0,1] and the
    azimuth is U[0, 2pi) for uniform points of the disc."""
    sur = scenes.random_frame_surfels(3, seed=7)
    i = 1
    n = np.array([sur["nx"][i], sur["ny"][i], sur["nz"][i]], np.float64)
    tu = np.array([sur["tux"][i], sur["tuy"][i], sur["tuz"][i]], np.float64)
    tv = np.array([sur["tvx"][i], sur["tvy"][i], sur["tvz"][i]], np.float64)
    d = np.array([orc.ray_direction(sur, i, r, seed=99)[0] for r in range(8000)], np.float64)
    assert np.all(np.abs(np.linalg.norm(d, axis=1) - 1.0) < 1e-5)
    cz = d @ n
    assert np.all(cz >= 0)
    assert scipy.stats.kstest(cz ** 2, "uniform").pvalue > 1e-3
    az = np.arctan2(d @ tv, d @ tu) % (2 * math.pi)
    assert scipy.stats.kstest(az / (2 * math.pi), "uniform").pvalue > 1e-3
    # rays of different receivers / seeds are different streams
    d2 = np.array([orc.ray_direction(sur, i, r, seed=100)[0] for r in range(64)], np.float64)
    assert np.mean(np.all(d2 == d[:64], axis=1)) < 0.05


# ---------------------------------------------------------------------------
# hits: brute force against an independent FP64 linear solve
# ---------------------------------------------------------------------------
def test_hits_match_independent_fp64_solve(orc):
    """Every hit j of a ray solves o + t d = p_j + s_u u t_u + s_v v t_v with
    u^2 + v^2 <= 9 and t > t_eps.  The oracle decides this in FP32 (D_hit);
    here it is decided by numpy.linalg.solve in FP64.  The two agree except
    where the FP64 margin is tiny."""
    sur = scenes.random_frame_surfels(64, seed=11, extent=0.6, scale=(0.05, 0.2))
    te = orc.default_t_eps(sur)
    P = np.stack([sur["px"], sur["py"], sur["pz"]], 1).astype(np.float64)
    TU = np.stack([sur["tux"], sur["tuy"], sur["tuz"]], 1).astype(np.float64)
    TV = np.stack([sur["tvx"], sur["tvy"], sur["tvz"]], 1).astype(np.float64)
    NN = np.stack([sur["nx"], sur["ny"], sur["nz"]], 1).astype(np.float64)
    su, sv = sur["su"].astype(np.float64), sur["sv"].astype(np.float64)
    checked = hits_total = 0
    for i in range(0, 64, 3):
        for r in range(24):
            h = orc.trace_ray(sur, i, r, seed=5, t_eps=te, t_min=0.0)
            d = h["d"].astype(np.float64)
            o = P[i]
            ref, marg = {}, set()
            for j in range(64):
                if j == i:
                    continue
                den = d @ NN[j]
                A = np.stack([d, -su[j] * TU[j], -sv[j] * TV[j]], 1)
                try:
                    t, u, v = np.linalg.solve(A, P[j] - o)
                except np.linalg.LinAlgError:
                    continue
                r2 = u * u + v * v
                near = (abs(r2 - 9.0) < 1e-4 or abs(t - te) < 1e-4 * max(te, 1e-30) * 1e3
                        or abs(abs(den) - 1e-6) < 1e-7)
                ok = abs(den) > 1e-6 and t > te and r2 <= 9.0
                if near:
                    marg.add(j)
                elif ok:
                    ref[j] = (t, r2, den < 0)
            got = {int(j): k for k, j in enumerate(h["j"])}
            assert set(got) - marg == set(ref), (i, r)
            for j, (t, r2, front) in ref.items():
                k = got[j]
                assert abs(h["t"][k] - t) <= 1e-5 * abs(t) + 1e-7
                assert bool(h["front"][k]) == front
                # u, v by projection onto FP32 tangents (orthonormal to ~1e-7)
                # vs. by the solve: alpha agrees to ~1.7 * 9 * 1e-7 relative
                a_ref = _alpha_profile(r2, float(np.minimum(sur["opacity"][j], np.float32(0.9999))))
                assert abs(h["alpha"][k] - a_ref) <= 2e-5 * max(a_ref, 1e-300) + 1e-15
            # depth order, ties broken by index
            tj = list(zip(h["t"].tolist(), h["j"].tolist()))
            assert tj == sorted(tj)
            # transmittance in front of each hit is the product of (1 - alpha)
            T = np.concatenate([[1.0], np.cumprod(1.0 - h["alpha"])[:-1]]) if len(h["t"]) else np.zeros(0)
            assert np.allclose(h["T"], T, rtol=1e-12, atol=1e-300)
            checked += 1
            hits_total += len(ref)
    assert checked > 400 and hits_total > 50


def test_transmittance_cut(orc):
    """Compositing stops after the first hit that leaves T < t_min."""
    sur = scenes.random_frame_surfels(200, seed=3, extent=0.4, scale=(0.1, 0.2), opacity=(0.8, 0.99))
    te = orc.default_t_eps(sur)
    seen_cut = 0
    for i in range(0, 200, 7):
        for r in range(8):
            h = orc.trace_ray(sur, i, r, seed=1, t_eps=te, t_min=1e-3)
            m = h["n_comp"]
            T_after = h["T"] * (1.0 - h["alpha"])
            # the cut is decided on the FP32 transmittance (D_stop), which
            # follows the FP64 one to a few 1e-7 relative
            if m < len(h["t"]):
                seen_cut += 1
                assert T_after[m - 1] < 1e-3 * (1 + 1e-5) and np.all(T_after[: m - 1] >= 1e-3 * (1 - 1e-5))
            else:
                assert np.all(T_after[: max(m - 1, 0)] >= 1e-3 * (1 - 1e-5))
    assert seen_cut > 5


# ---------------------------------------------------------------------------
# form factors
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("h,s,o", [(1.0, 0.2, 0.9), (0.5, 0.1, 0.5), (0.3, 0.15, 0.99)])
def test_coaxial_disc_form_factor(orc, h, s, o):
    """Point-to-coaxial-disc form factor with the Gaussian opacity profile:
    F = 2 h^2 int_0^{3s} alpha(rho/s) rho / (h^2 + rho^2)^2 drho."""
    sur = _two_surfels([0.0, 0.0, h], [0.0, 0.0, -1.0], (s, s), o)
    R = 1 << 18
    rp, c, v, diag = orc.ff_rows(sur, [0], R, seed=2024, t_eps=1e-6, t_min=0.0)
    assert list(c) == [1]
    f1 = lambda r: _alpha_profile((r / s) ** 2, o) * 2 * h * h * r / (h * h + r * r) ** 2
    f2 = lambda r: _alpha_profile((r / s) ** 2, o) ** 2 * 2 * h * h * r / (h * h + r * r) ** 2
    F = scipy.integrate.quad(f1, 0, 3 * s, epsabs=1e-14, epsrel=1e-12)[0]
    EW2 = scipy.integrate.quad(f2, 0, 3 * s, epsabs=1e-14, epsrel=1e-12)[0]
    sigma = math.sqrt(max(EW2 - F * F, 0.0) / R)
    assert abs(v[0] - F) < 5 * sigma, (v[0], F, sigma)
    assert diag[0, 1] == 0.0          # nothing behind the receiver, no back faces


@pytest.mark.parametrize("pj,nj,sj,oj", [
    ([0.3, -0.2, 0.8], [0.2, 0.4, -1.0], (0.12, 0.07), 0.8),
    ([-0.5, 0.1, 0.6], [0.9, 0.0, -0.5], (0.05, 0.15), 0.95),
])
def test_oblique_disc_form_factor_and_back_face(orc, pj, nj, sj, oj):
    """A tilted, anisotropic sender: the estimator matches the area integral
    (1/pi) int alpha cos_i |cos_j| / r^2 dA; flipping the sender's normal
    moves the same weight from F to the back-face (occlusion-only) bucket."""
    R = 1 << 19
    sur = _two_surfels(pj, nj, sj, oj)
    F, EW2 = _exact_point_to_disc(sur)
    sigma = math.sqrt(max(EW2 - F * F, 0.0) / R)
    rp, c, v, diag = orc.ff_rows(sur, [0], R, seed=77, t_eps=1e-6, t_min=0.0)
    assert abs(v[0] - F) < 5 * sigma
    sur_b = _two_surfels(pj, -np.asarray(nj, float), sj, oj)
    rp, c, v, diag = orc.ff_rows(sur_b, [0], R, seed=77, t_eps=1e-6, t_min=0.0)
    assert len(c) == 0
    assert abs(diag[0, 1] - F) < 5 * sigma


def test_reciprocity_far_pair(orc):
    """A_i F_ij = A_j F_ji for the exact expectations up to O((3s/r)^2)
    (centre-origin reading), and the MC estimates agree within their error."""
    r = 2.0
    pj = np.array([0.4, 0.3, r])
    pj_dir = pj / np.linalg.norm(pj)
    nj = -pj_dir + np.array([0.3, -0.1, 0.0])
    sur = _two_surfels(pj, nj, (0.05, 0.03), 0.9, s_i=0.04, o_i=0.7)
    A = orc.effective_area(sur["su"], sur["sv"], sur["opacity"])
    F01, _ = _exact_point_to_disc(sur, j=1)
    # swap roles: put surfel 1 at the origin, facing +z, by a rigid motion
    P = np.stack([sur["px"], sur["py"], sur["pz"]], 1).astype(np.float64)
    N_ = np.stack([sur["nx"], sur["ny"], sur["nz"]], 1).astype(np.float64)
    TU = np.stack([sur["tux"], sur["tuy"], sur["tuz"]], 1).astype(np.float64)
    TV = np.stack([sur["tvx"], sur["tvy"], sur["tvz"]], 1).astype(np.float64)
    Rm = np.stack([TU[1], TV[1], N_[1]], 0)           # world -> frame of surfel 1
    p2 = (Rm @ (P[0] - P[1]))[None, :]
    rev = scenes.surfels_from_arrays(
        np.concatenate([[[0, 0, 0]], p2]), np.stack([[0, 0, 1.0], Rm @ N_[0]]),
        np.stack([[1.0, 0, 0], Rm @ TU[0]]), np.stack([[0, 1.0, 0], Rm @ TV[0]]),
        [sur["su"][1], sur["su"][0]], [sur["sv"][1], sur["sv"][0]], [sur["opacity"][1], sur["opacity"][0]])
    F10, _ = _exact_point_to_disc(rev, j=1)
    rel = abs(A[0] * F01 - A[1] * F10) / (A[0] * F01)
    assert rel < 9 * (3 * 0.05 / r) ** 2
    R = 1 << 21
    _, _, v01, _ = orc.ff_rows(sur, [0], R, seed=5, t_eps=1e-6, t_min=0.0)
    _, _, v10, _ = orc.ff_rows(rev, [0], R, seed=5, t_eps=1e-6, t_min=0.0)
    for est, ref in ((v01[0], F01), (v10[0], F10)):
        assert abs(est - ref) < 5 * math.sqrt(ref / R)


def test_row_sums_telescope_and_stay_below_one(orc):
    """sum_j F_ij + (back-face weight) = (1/R) sum_r (1 - T_r) <= 1: the
    compositing weights of one ray telescope (Eq. L_I)."""
    sc = scenes.make_config(1)
    te = orc.default_t_eps(sc.surfels)
    rp, c, v, diag = orc.ff_rows(sc.surfels, np.arange(0, 512, 9), sc.R, sc.seed, te, 1e-4)
    front = np.add.reduceat(v, rp[:-1]) if v.size else np.zeros(0)
    assert np.allclose(front, diag[:, 0], rtol=1e-12)
    assert np.allclose(diag[:, 0] + diag[:, 1], diag[:, 2], rtol=1e-10, atol=1e-13)
    assert np.all(diag[:, 2] <= 1.0 + 1e-12)


def test_topk_keeps_largest_entries(orc):
    sc = scenes.make_config(3, n=4000)
    te = orc.default_t_eps(sc.surfels)
    recv = np.arange(0, 4000, 400)
    rp0, c0, v0, d0 = orc.ff_rows(sc.surfels, recv, 32, 3, te, 1e-4, topk=0)
    rp1, c1, v1, d1 = orc.ff_rows(sc.surfels, recv, 32, 3, te, 1e-4, topk=40)
    for k in range(len(recv)):
        full = dict(zip(c0[rp0[k]:rp0[k + 1]].tolist(), v0[rp0[k]:rp0[k + 1]].tolist()))
        kept = dict(zip(c1[rp1[k]:rp1[k + 1]].tolist(), v1[rp1[k]:rp1[k + 1]].tolist()))
        assert len(kept) == min(40, len(full))
        assert all(full[j] == val for j, val in kept.items())
        if len(full) > 40:
            lo = min(kept.values())
            assert all(val <= lo for j, val in full.items() if j not in kept)
        assert list(kept) == sorted(kept)


# ---------------------------------------------------------------------------
# effective area (App. E) and direct light
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("o", [0.05, 0.5, 0.9, 0.99, 0.9999])
def test_effective_area_closed_form(orc, o):
    su, sv = 0.3, 0.07
    o = float(np.float32(o))
    quad = 2 * math.pi * su * sv * scipy.integrate.quad(
        lambda r: _alpha_profile(r * r, o) * r, 0, 3, epsabs=1e-15, epsrel=1e-13)[0]
    closed = orc.effective_area(np.array([su]), np.array([sv]), np.array([o], np.float32))[0]
    c = -math.log1p(-float(np.float32(o)))
    ein_q = scipy.integrate.quad(lambda y: -math.expm1(-y) / y, 0, c, epsabs=1e-15, epsrel=1e-13)[0]
    assert abs(orc.ein(np.array([c]))[0] - ein_q) < 1e-12 * max(1.0, ein_q)
    # the closed form integrates over the whole plane; the 3-sigma cut drops
    # the tail int_3^inf alpha r dr <= c exp(-1.7*9) / 3.4 (alpha <= c G^3.4)
    tail = 2 * math.pi * su * sv * c * math.exp(-1.7 * 9) / 3.4
    assert 0 <= closed - quad <= tail * (1 + 1e-6) + 1e-15


def test_direct_light_furnace(orc):
    """Light at the centre of the unit sphere of inward surfels: r = 1,
    cos = 1, nothing occludes, so E_00 = o a 2/sqrt(pi) and the radiance
    Y00 E_00 = o a I cos T / (pi r^2)."""
    sc = scenes.make_config(1)
    E = orc.direct_light(sc.surfels, sc.albedo, sc.light_pos, sc.light_I, sc.K)
    o = sc.surfels["opacity"].astype(np.float64)
    ref = (o[:, None] * sc.albedo.astype(np.float64) * 2 / math.sqrt(math.pi))
    assert np.allclose(E[:, 0, 0, :], ref, rtol=2e-6)
    assert np.allclose(E[:, 0, 0, :] / (2 * math.sqrt(math.pi)), ref / (2 * math.sqrt(math.pi)), rtol=2e-6)


def test_direct_light_single_occluder_and_back_face(orc):
    """One occluder centred on the segment to the light transmits exactly
    1 - o_occ; a light behind the receiver gives E = 0; SH degree >= 1
    coefficients stay zero."""
    p = np.array([[0, 0, 0], [0.1, 0.0, 1.0], [5.0, 5.0, 5.0]], float)
    nrm = np.array([[0, 0, 1.0], [0.3, 0.2, 1.0], [0, 0, 1.0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    tu, tv = scenes.onb_from_normal(nrm)
    sur = scenes.surfels_from_arrays(p, nrm, tu, tv, [0.1, 0.2, 0.1], [0.1, 0.3, 0.1], [0.6, 0.7, 0.5])
    alb = np.array([[0.5, 0.25, 0.75]] * 3, np.float32)
    lp = np.array([[0.2, 0.0, 2.0], [0.0, 0.0, -3.0]], np.float32)
    li = np.array([3.0, 2.0], np.float32)
    E, T = orc.direct_light(sur, alb, lp, li, K=4, t_eps=1e-6, receivers=[0], return_T=True)
    d = lp[0].astype(np.float64)
    r2 = d @ d
    cos = d[2] / math.sqrt(r2)
    # analytic transmittance: the occluder plane is crossed at t* = (p1.n1)/(d.n1)
    n1 = nrm[1]
    t_star = (p[1] @ n1) / (d @ n1)
    x = t_star * d - p[1]
    u = (x @ tu[1]) / 0.2
    v = (x @ tv[1]) / 0.3
    T_ref = 1.0 - _alpha_profile(u * u + v * v, float(np.float32(0.7)))
    assert abs(T[0, 0] - T_ref) < 1e-9
    ref = float(np.float32(0.6)) * alb[0].astype(np.float64) * 2 / math.sqrt(math.pi) * 3.0 * cos / r2 * T_ref
    assert np.allclose(E[0, 0, 0], ref, rtol=1e-9)
    assert np.all(E[0, 0, 1:] == 0) and np.all(E[0, 1] == 0)


# ---------------------------------------------------------------------------
# bounces and adjoint
# ---------------------------------------------------------------------------
def _random_operator(n, seed, density=0.2, row_sum=0.8):
    rng = np.random.default_rng(seed)
    F = sp.random(n, n, density=density, random_state=rng, format="csr")
    F.setdiag(0)
    F.eliminate_zeros()
    rs = np.asarray(F.sum(axis=1)).ravel()
    F = sp.diags(row_sum / np.maximum(rs, 1e-30)) @ F
    return sp.csr_matrix(F)


def test_closed_sphere_furnace_exact(orc):
    """Analytic closed-sphere operator F_ij = A_j / sum A (row stochastic)
    with uniform E: B^(n) = E sum_{k<=n} rho^k exactly, -> E / (1 - rho)."""
    n = 64
    A = np.random.default_rng(0).uniform(0.5, 1.5, n)
    F = sp.csr_matrix(np.tile(A / A.sum(), (n, 1)))
    rho = np.full((n, 3), 0.99 * 0.5)
    E = np.ones((n, 1, 1, 3))
    for nb in (0, 1, 6, 40):
        B = orc.bounce(F, rho, E, nb)
        assert np.allclose(B, sum(0.495 ** k for k in range(nb + 1)), rtol=1e-13)
    assert abs(orc.bounce(F, rho, E, 200)[0, 0, 0, 0] - 1 / (1 - 0.495)) < 1e-12


def test_bounce_is_neumann_partial_sum_and_converges_to_lu(orc):
    n, Lt, K = 80, 2, 4
    F = _random_operator(n, 1)
    rho = np.random.default_rng(2).uniform(0.1, 0.9, (n, 3))
    E = np.random.default_rng(3).uniform(0, 1, (n, Lt, K, 3))
    C = Lt * K * 3
    E2 = E.reshape(n, C)
    for col in range(3):
        M = sp.diags(rho[:, col]) @ F
        Md = M.toarray()
        for nb in (0, 3, 8):
            ref = sum(np.linalg.matrix_power(Md, k) for k in range(nb + 1)) @ E2[:, col::3]
            assert np.allclose(orc.bounce(F, rho, E, nb).reshape(n, C)[:, col::3], ref, rtol=1e-12, atol=1e-14)
        fixed = np.linalg.solve(np.eye(n) - Md, E2[:, col::3])
        assert np.allclose(orc.bounce(F, rho, E, 300).reshape(n, C)[:, col::3], fixed, rtol=1e-10)


def test_adjoint_dot_product_identity(orc):
    """B(E) is linear in E, so <g, B(E)> = <grad_E, E> exactly."""
    n, Lt, K, nb = 60, 3, 1, 7
    F = _random_operator(n, 4)
    rho = np.random.default_rng(5).uniform(0.1, 0.9, (n, 3))
    E = np.random.default_rng(6).uniform(0, 1, (n, Lt, K, 3))
    g = np.random.default_rng(7).standard_normal((n, Lt, K, 3))
    B, tape = orc.bounce(F, rho, E, nb, keep_tape=True)
    gE, grho, gF = orc.adjoint(F, rho, tape, g)
    assert abs(np.sum(g * B) - np.sum(gE * E)) < 1e-12 * np.sum(np.abs(g * B))


def test_adjoint_matches_central_differences(orc):
    n, Lt, K, nb = 40, 2, 4, 5
    F = _random_operator(n, 8, density=0.3)
    rho = np.random.default_rng(9).uniform(0.1, 0.9, (n, 3))
    E = np.random.default_rng(10).uniform(0, 1, (n, Lt, K, 3))
    g = np.random.default_rng(11).standard_normal((n, Lt, K, 3))
    B, tape = orc.bounce(F, rho, E, nb, keep_tape=True)
    gE, grho, gF = orc.adjoint(F, rho, tape, g)
    L = lambda F_, r_, E_: np.sum(g * orc.bounce(F_, r_, E_, nb))
    rng = np.random.default_rng(12)
    h = 1e-6
    for _ in range(16):
        i, c = rng.integers(n), rng.integers(3)
        rp, rm = rho.copy(), rho.copy()
        rp[i, c] += h
        rm[i, c] -= h
        fd = (L(F, rp, E) - L(F, rm, E)) / (2 * h)
        assert abs(fd - grho[i, c]) < 1e-6 * max(1.0, abs(fd))
    for _ in range(16):
        e = rng.integers(F.nnz)
        Fp, Fm = F.copy(), F.copy()
        Fp.data[e] += h
        Fm.data[e] -= h
        fd = (L(Fp, rho, E) - L(Fm, rho, E)) / (2 * h)
        assert abs(fd - gF[e]) < 1e-6 * max(1.0, abs(fd))
    for _ in range(8):
        idx = tuple(rng.integers(s) for s in E.shape)
        Ep, Em = E.copy(), E.copy()
        Ep[idx] += h
        Em[idx] -= h
        fd = (L(F, rho, Ep) - L(F, rho, Em)) / (2 * h)
        assert abs(fd - gE[idx]) < 1e-6 * max(1.0, abs(fd))


def test_dense_grad_F_matches_central_differences(orc):
    """The dense dL/dF (every pair, stored or not) against central
    differences of the loss in F_ij, and equal to the stored-entry vector on
    the stored entries."""
    n, Lt, K, nb = 30, 1, 4, 4
    F = _random_operator(n, 6, density=0.25)
    rho = np.random.default_rng(19).uniform(0.1, 0.9, (n, 3))
    E = np.random.default_rng(20).uniform(0, 1, (n, Lt, K, 3))
    g = np.random.default_rng(21).standard_normal((n, Lt, K, 3))
    B, tape = orc.bounce(F, rho, E, nb, keep_tape=True)
    _, _, gF = orc.adjoint(F, rho, tape, g)
    gE, grho, G = orc.adjoint(F, rho, tape, g, dense_grad_F=True)
    assert G.shape == (n, n)
    rows = np.repeat(np.arange(n), np.diff(F.indptr))
    assert np.allclose(G[rows, F.indices], gF, rtol=1e-12, atol=1e-14)
    Fd = F.toarray()
    L = lambda Fm: np.sum(g * orc.bounce(sp.csr_matrix(Fm), rho, E, nb))
    rng = np.random.default_rng(22)
    h = 1e-6
    for _ in range(20):
        i, j = rng.integers(n), rng.integers(n)
        Fp, Fm = Fd.copy(), Fd.copy()
        Fp[i, j] += h
        Fm[i, j] -= h
        fd = (L(Fp) - L(Fm)) / (2 * h)
        assert abs(fd - G[i, j]) < 1e-6 * max(1.0, abs(fd))


def test_paper_brdf_gradient_closed_form_at_fixed_point(orc):
    """Eq. final-dl-dbrdf: at the fixed point dL/df = dL/dE * (B - E) / f,
    per colour summed over coefficients and lights."""
    n, Lt, K = 50, 2, 4
    F = _random_operator(n, 13, row_sum=0.7)
    rho = np.random.default_rng(14).uniform(0.2, 0.9, (n, 3))
    E = np.random.default_rng(15).uniform(0, 1, (n, Lt, K, 3))
    g = np.random.default_rng(16).standard_normal((n, Lt, K, 3))
    nb = 160
    B, tape = orc.bounce(F, rho, E, nb, keep_tape=True)
    gE, grho, gF = orc.adjoint(F, rho, tape, g)
    paper = (gE * (B - E)).reshape(n, -1, 3).sum(axis=1) / rho
    assert np.allclose(grho, paper, rtol=1e-9, atol=1e-12)


def test_zero_bounces_is_direct_light(orc):
    n = 10
    F = _random_operator(n, 17)
    E = np.random.default_rng(18).uniform(0, 1, (n, 1, 9, 3))
    assert np.array_equal(orc.bounce(F, np.full((n, 3), 0.5), E, 0), E)


# ---------------------------------------------------------------------------
# opacity gradient through the compositing
# ---------------------------------------------------------------------------
def test_opacity_backward_matches_central_differences(orc):
    """dL/do for L = <W, F(o)> + <V, rho(o, a)>, hit sets fixed (t_min = 0,
    no truncation), against central differences of the oracle's own F."""
    n, R = 40, 24
    sur = scenes.random_frame_surfels(n, seed=21, extent=0.35, scale=(0.08, 0.2), opacity=(0.3, 0.95))
    alb = np.random.default_rng(22).uniform(0.1, 0.9, (n, 3)).astype(np.float32)
    te = orc.default_t_eps(sur)
    F, _ = orc.ff_matrix(sur, R, seed=9, t_eps=te, t_min=0.0)
    W = F.copy()
    W.data = np.random.default_rng(23).standard_normal(F.nnz)
    V = np.random.default_rng(24).standard_normal((n, 3))
    go, ga = orc.opacity_backward(sur, alb, R, 9, te, 0.0, (W.indptr, W.indices, W.data), grad_rho=V)

    def loss(op32):
        s2 = dict(sur)
        s2["opacity"] = op32
        F2, _ = orc.ff_matrix(s2, R, seed=9, t_eps=te, t_min=0.0)
        assert np.array_equal(F2.indices, F.indices)
        return np.sum(W.data * F2.data) + np.sum(V * orc.rho(op32, alb))

    rng = np.random.default_rng(25)
    hits = np.unique(F.indices)
    for m in rng.choice(hits, size=min(10, hits.size), replace=False):
        op_p, op_m = sur["opacity"].copy(), sur["opacity"].copy()
        op_p[m] = np.float32(op_p[m] + np.float32(2e-4))
        op_m[m] = np.float32(op_m[m] - np.float32(2e-4))
        fd = (loss(op_p) - loss(op_m)) / (float(op_p[m]) - float(op_m[m]))
        assert abs(fd - go[m]) < 2e-4 * max(1.0, abs(fd)), (m, fd, go[m])
    assert np.allclose(ga, V * orc.clamp_opacity(sur["opacity"])[:, None])


# ---------------------------------------------------------------------------
# ray-cast furnace (config 1): bounds that hold for any row sums
# ---------------------------------------------------------------------------
def test_raycast_furnace_bounds(orc):
    """With uniform E and rho, B^(n) lies between E sum (rho s_min)^k and
    E sum (rho s_max)^k (s = row sums of F), and row sums are <= 1."""
    sc = scenes.make_config(1)
    te = orc.default_t_eps(sc.surfels)
    F, diag = orc.ff_matrix(sc.surfels, sc.R, sc.seed, te, sc.t_min)
    s = np.asarray(F.sum(axis=1)).ravel()
    assert np.all(s <= 1.0) and s.min() > 0.2
    E = orc.direct_light(sc.surfels, sc.albedo, sc.light_pos, sc.light_I, sc.K)
    rho = orc.rho(sc.surfels["opacity"], sc.albedo)
    B = orc.bounce(F, rho, E, sc.n_bounces)
    r0 = rho[0, 0]
    lo = E[:, 0, 0, 0] * sum((r0 * s.min()) ** k for k in range(sc.n_bounces + 1))
    hi = E[:, 0, 0, 0] * sum((r0 * s.max()) ** k for k in range(sc.n_bounces + 1))
    assert np.all(B[:, 0, 0, 0] >= lo * (1 - 1e-12)) and np.all(B[:, 0, 0, 0] <= hi * (1 + 1e-12))
    # on a sphere the cosine-weighted rays land uniformly by area: the
    # expected row sum is close to the transmittance-limited fill factor
    assert 0.4 < s.mean() < 0.9


def test_exp_fx_is_within_three_ulp_of_exp(orc):
    """D_stop's exp_fx against the FP64 exponential over its whole range
    (dense grid plus the reduction boundaries k ln2 +- ln2/2)."""
    L = orc.lib()
    ys = np.concatenate([np.linspace(-80.0, 0.0, 200_001), -np.arange(0, 116) * np.log(2.0),
                         -(np.arange(0, 115) + 0.5) * np.log(2.0)]).astype(np.float32)
    ys = ys[ys > -80.0]
    got = np.array([L.orc_exp_fx(float(y)) for y in ys[::7]], np.float64)
    ref = np.exp(ys[::7].astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ref) / ulp) <= 3.0
    assert L.orc_exp_fx(0.0) == 1.0 and L.orc_exp_fx(-80.0) == 0.0 and L.orc_exp_fx(-100.0) == 0.0


def test_cut_transmittance_tracks_fp64(orc):
    """The FP32 transmittance of the cut (D_stop) follows the FP64 product
    of (1 - alpha) to FP32 accuracy along every ray."""
    worst = 0.0
    for sur, step in ((scenes.random_frame_surfels(300, seed=8, extent=0.4, scale=(0.1, 0.25), opacity=(0.3, 0.99)),
                       11),
                      (scenes.make_config("fruit_bowl", n=20000).surfels, 1999)):
        te = orc.default_t_eps(sur)
        for i in range(0, sur["px"].shape[0], step):
            for r in range(6):
                h = orc.trace_ray(sur, i, r, seed=4, t_eps=te, t_min=0.0)
                T64 = h["T"]
                keep = T64 > 1e-30
                if keep.any():
                    worst = max(worst, float(np.max(np.abs(h["T32"][keep] - T64[keep]) / T64[keep])))
    assert worst < 1e-5


def test_reciprocity_measure(orc):
    """Zero on an exactly reciprocal operator (closed sphere, F_ij = A_j / sum A);
    a single perturbed entry shows up with its exact relative size, and an
    entry whose mirror is missing counts fully."""
    rng = np.random.default_rng(5)
    A = rng.uniform(0.5, 2.0, 40)
    Fd = np.tile(A / A.sum(), (40, 1))
    np.fill_diagonal(Fd, 0.0)
    asym, mx = orc.reciprocity(sp.csr_matrix(Fd), A)
    assert asym < 1e-15 and mx < 1e-15
    Fp = Fd.copy()
    Fp[3, 7] *= 1.5
    a, b = A[3] * Fp[3, 7], A[7] * Fp[7, 3]
    asym, mx = orc.reciprocity(sp.csr_matrix(Fp), A)
    assert abs(mx - abs(a - b) / max(a, b)) < 1e-14
    assert abs(asym - 2 * abs(a - b) / (A[:, None] * Fp).sum()) < 1e-14
    Fm = Fd.copy()
    Fm[9, 2] = 0.0
    _, mx = orc.reciprocity(sp.csr_matrix(Fm), A)
    assert mx == 1.0


# ---------------------------------------------------------------------------
# the FP32 hit decisions against FP64 truth at workload scale
# ---------------------------------------------------------------------------
def _fp64_decisions(q, qq2, TU, TV, NN, su, sv, smax, i, d, te):
    """Exact (FP64) hit test of one ray from p_i against every surfel
    (q = p - p_i, qq2 = |q|^2): candidates whose centre lies within
    3 max(s_u, s_v) of the ray line, then a Cramer solve of
    o + t d = p_j + u s_u t_u + v s_v t_v."""
    qd = q @ d
    dist2 = qq2 - qd * qd
    cand = np.nonzero(dist2 <= (3.0 * smax) ** 2 * (1 + 1e-6) + 1e-12)[0]
    cand = cand[cand != i]
    b = -su[cand, None] * TU[cand]
    c = -sv[cand, None] * TV[cand]
    qq = q[cand]
    bc = np.cross(b, c)
    det = bc @ d
    t = np.einsum("ij,ij->i", qq, bc) / det
    u = np.cross(qq, c) @ d / det
    v = np.cross(b, qq) @ d / det
    den = NN[cand] @ d
    r2 = u * u + v * v
    ok = (np.abs(den) > 1e-6) & (t > te) & (r2 <= 9.0)
    return {int(j): (float(tt), float(rr), float(dd), bool(o)) for j, tt, rr, dd, o in zip(cand, t, r2, den, ok)}


@pytest.mark.parametrize("name,n,receivers,rays", [("fruit_bowl", 100_000, 1250, 8), ("box_room", 16_384, 1250, 8)])
def test_fp32_hit_decisions_against_fp64_at_workload_scale(orc, name, n, receivers, rays):
    """10^4 rays of the benchmark scenes (Eq. L_I: hits sorted by depth).
    Which surfels a ray hits and their depth order are decided in FP32 on
    both sides (D_hit).  Against an exact FP64 solve of the same rays:
    * every surfel where the two hit sets differ is a margin case (u^2+v^2
      within 1e-4 of the 3-sigma cut, t at t_eps, or grazing), whose alpha
      is at most c e^(-1.7 * 9) < 1e-5;
    * every adjacent pair of composited hits whose (t, j) order disagrees
      with the FP64 depth order is a tie at FP32 resolution (FP64 depths
      within 4 FP32 ulps): coplanar wall surfels are hit at the same depth
      in exact arithmetic, and the order of equal keys is the index;
    * the form-factor mass that such swapped pairs move, alpha_a alpha_b T
      per pair, is recorded (fruit bowl: a few 1e-5 of the composited
      mass)."""
    sc = scenes.make_config(name, n=n)
    sur = sc.surfels
    P = np.stack([sur["px"], sur["py"], sur["pz"]], 1).astype(np.float64)
    TU = np.stack([sur["tux"], sur["tuy"], sur["tuz"]], 1).astype(np.float64)
    TV = np.stack([sur["tvx"], sur["tvy"], sur["tvz"]], 1).astype(np.float64)
    NN = np.stack([sur["nx"], sur["ny"], sur["nz"]], 1).astype(np.float64)
    su, sv = sur["su"].astype(np.float64), sur["sv"].astype(np.float64)
    smax = float(max(su.max(), sv.max()))
    c = orc.opacity_constant(sur["opacity"])
    te = float(orc.default_t_eps(sur))
    recv = np.random.default_rng(7).choice(n, size=receivers, replace=False)
    n_rays = n_hits = n_diff = n_pairs = n_swap = 0
    moved = mass = 0.0
    for i in recv:
        q = P - P[i]
        qq2 = np.einsum("ij,ij->i", q, q)
        for r in range(rays):
            # every hit of the ray (also past the cut) and how many are composited
            h = orc.trace_ray(sur, int(i), r, sc.seed, te, sc.t_min)
            ref = _fp64_decisions(q, qq2, TU, TV, NN, su, sv, smax, int(i), h["d"].astype(np.float64), te)
            got = set(h["j"].tolist())
            want = {j for j, v in ref.items() if v[3]}
            n_rays += 1
            n_hits += len(want)
            for j in got ^ want:
                t, r2, den, _ = ref[j]
                margin = abs(r2 - 9.0) < 1e-4 or abs(t - te) < 1e-4 * te or abs(abs(den) - 1e-6) < 1e-7
                assert margin, (name, i, r, j, t, r2, den)
                assert c[j] * math.exp(-1.7 * min(r2, 9.0)) < 1e-5
                n_diff += 1
            m = h["n_comp"]
            J, al, T, t32 = h["j"][:m], h["alpha"][:m], h["T"][:m], h["t"][:m]
            mass += float(np.sum(al * T))
            for k in range(m - 1):
                n_pairs += 1
                ta, tb = ref[int(J[k])][0], ref[int(J[k + 1])][0]
                if ta > tb:
                    assert ta - tb <= 4 * float(np.spacing(np.float32(t32[k]))), (name, i, r, k, ta, tb)
                    n_swap += 1
                    moved += float(al[k] * al[k + 1] * T[k])
    print(f"\n{name}: {n_rays} rays, {n_hits} FP64 hits, {n_diff} margin differences, "
          f"{n_swap}/{n_pairs} adjacent pairs tied at FP32 resolution, moved mass {moved / max(mass, 1e-300):.2e}")
    assert n_rays == receivers * rays and n_hits > 10 * n_rays
    if name == "fruit_bowl":
        assert moved <= 1e-4 * mass


# ---------------------------------------------------------------------------
# geometry gradients through the ray-cast form factors (Eq. dl-dgeo-0)
# ---------------------------------------------------------------------------
def _layers_scene():
    """Four small receivers on z = 0 under three broad, tilted,
    semi-transparent layers (one facing up: it only occludes); the layers are
    so large that the rays cross them far inside their support."""
    p, nrm, s, o = [], [], [], []
    for k, tilt in enumerate([0.0, 0.15, -0.1, 0.25]):
        p.append([0.2 * k, 0.1 * (k % 2), 0.0])
        nrm.append([math.sin(tilt), 0.05 * k, math.cos(tilt)])
        s.append(0.02)
        o.append(0.9)
    for z, nn, op in [(0.3, [0.1, -0.2, -1.0], 0.45), (0.6, [-0.2, 0.1, 1.0], 0.35), (0.95, [0.15, 0.1, -1.0], 0.6)]:
        p.append([0.3, 0.05, z])
        nrm.append(nn)
        s.append(6.0)
        o.append(op)
    nrm = np.array(nrm, float)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    tu, tv = scenes.onb_from_normal(nrm)
    ang = np.linspace(0.2, 1.3, len(p))
    tu2 = np.cos(ang)[:, None] * tu + np.sin(ang)[:, None] * tv
    tv2 = -np.sin(ang)[:, None] * tu + np.cos(ang)[:, None] * tv
    return scenes.surfels_from_arrays(np.array(p, float), nrm, tu2, tv2, s, np.array(s) * 1.1, o)


def test_geometry_gradients_through_ray_cast_form_factors_match_central_differences(orc):
    """dL/d(every surfel field) of L = sum_ij G_ij F_ij (ray-cast F, no
    compositing cut) against central differences of the oracle's own form
    factors; steps are the actual FP32 changes of the perturbed inputs."""
    sur = _layers_scene()
    n = sur["px"].shape[0]
    recv = np.arange(4)
    R, seed, te = 48, 21, 1e-6
    rp, co, vo, _ = orc.ff_rows(sur, recv, R, seed, te, 0.0, 0)
    rng = np.random.default_rng(6)
    Gd = rng.standard_normal((4, n))
    gv = Gd[np.repeat(np.arange(4), np.diff(rp)), co]
    grads = orc.geometry_backward(sur, R, seed, te, 0.0, (rp, co, gv), receivers=recv)

    def L(s_):
        rp_, co_, vo_, _ = orc.ff_rows(s_, recv, R, seed, te, 0.0, 0)
        return float(np.sum(Gd[np.repeat(np.arange(4), np.diff(rp_)), co_] * vo_))

    # the opacity part equals the compositing backward's
    go, _ = orc.opacity_backward(sur, np.zeros((n, 3)), R, seed, te, 0.0, (rp, co, gv), receivers=recv)
    assert np.allclose(grads["opacity"], go, rtol=1e-12, atol=1e-15)
    scale = max(np.max(np.abs(v)) for v in grads.values())
    checked = 0
    for f in orc.GEOMETRY_FIELDS:
        for k in range(n):
            x0 = np.float32(sur[f][k])
            step = np.float32(max(abs(float(x0)), 0.05) * 1e-3)
            sp_, sm_ = dict(sur), dict(sur)
            sp_[f] = sur[f].copy()
            sm_[f] = sur[f].copy()
            sp_[f][k] = np.float32(x0 + step)
            sm_[f][k] = np.float32(x0 - step)
            d = float(sp_[f][k]) - float(sm_[f][k])
            fd = (L(sp_) - L(sm_)) / d
            assert abs(fd - grads[f][k]) <= 2e-3 * (abs(fd) + 1e-3 * scale), (f, k, fd, grads[f][k])
            checked += 1
    assert checked == 15 * n


def test_direct_light_gradients_match_central_differences(orc):
    """Light positions and intensities, albedo, receivers' and occluders'
    surfel fields through the direct light (with shadowing), against central
    differences of the oracle's own direct light."""
    sur = _layers_scene()
    n = sur["px"].shape[0]
    alb = np.random.default_rng(8).uniform(0.2, 0.8, (n, 3)).astype(np.float32)
    lp = np.array([[0.4, 0.2, 1.6], [-0.3, 0.4, 1.3]], np.float32)
    lI = np.array([3.0, 1.5], np.float32)
    te = 1e-6
    K = 4
    gE = np.random.default_rng(9).standard_normal((n, 2, K, 3))
    g_lp, g_li, g_alb, grads = orc.direct_light_backward(sur, alb, lp, lI, gE, t_eps=te)

    def L(s_=sur, alb_=alb, lp_=lp, li_=lI):
        return float(np.sum(gE * orc.direct_light(s_, alb_, lp_, li_, K, te)))

    def fd_of(arr, idx, call):
        x0 = np.float32(arr[idx])
        step = np.float32(max(abs(float(x0)), 0.05) * 1e-3)
        ap, am = arr.copy(), arr.copy()
        ap[idx] = np.float32(x0 + step)
        am[idx] = np.float32(x0 - step)
        return (call(ap) - call(am)) / (float(ap[idx]) - float(am[idx]))

    scale = max(np.max(np.abs(g_lp)), max(np.max(np.abs(v)) for v in grads.values()))
    for l in range(2):
        for c in range(3):
            fd = fd_of(lp, (l, c), lambda a: L(lp_=a))
            assert abs(fd - g_lp[l, c]) <= 2e-3 * (abs(fd) + 1e-3 * scale), ("light", l, c)
        fd = fd_of(lI, l, lambda a: L(li_=a))
        assert abs(fd - g_li[l]) <= 1e-5 * abs(fd)
    for i in range(n):
        for c in range(3):
            fd = fd_of(alb, (i, c), lambda a: L(alb_=a))
            assert abs(fd - g_alb[i, c]) <= 1e-5 * (abs(fd) + 1e-6)
    checked = 0
    for f in orc.GEOMETRY_FIELDS:
        for k in range(n):
            def call(a, f=f):
                s_ = dict(sur)
                s_[f] = a
                return L(s_=s_)
            fd = fd_of(sur[f], k, call)
            assert abs(fd - grads[f][k]) <= 2e-3 * (abs(fd) + 1e-3 * scale), (f, k, fd, grads[f][k])
            checked += 1
    assert checked == 15 * n
