"""Pins of the FP64 oracle of the directional (SH) transfer, CPU only.

Each test checks oracle/sh.py against an independent route: the addition
theorem and quadrature orthonormality for the SH basis, a Legendre
quadrature of the clamped Phong lobe for App. A's coefficients, the zonal
lobe about the mirror direction for the local-frame reading, the scalar
Lambertian transport, an explicitly assembled operator matrix, the
dot-product identity of the adjoint and central finite differences.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.sparse as sp
import scipy.special

import scenes
from oracle import oracle as orc
from oracle import sh


def _unit(rng, n):
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# SH basis (Sec. 3.2)
# ---------------------------------------------------------------------------
def test_sh_basis_addition_theorem_and_parities():
    """sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b); Y_lm(-w) = (-1)^l Y_lm(w);
    the rotation by pi about z multiplies Y_lm by (-1)^m."""
    rng = np.random.default_rng(0)
    a, b = _unit(rng, 500), _unit(rng, 500)
    K = 16
    Ya, Yb = sh.sh_basis(a, K), sh.sh_basis(b, K)
    ls, ms = sh.sh_l_of(K), sh.sh_m_of(K)
    cosab = np.sum(a * b, axis=1)
    for l in range(4):
        sel = ls == l
        lhs = np.sum(Ya[:, sel] * Yb[:, sel], axis=1)
        rhs = (2 * l + 1) / (4 * math.pi) * scipy.special.eval_legendre(l, cosab)
        assert np.max(np.abs(lhs - rhs)) < 1e-13
    assert np.allclose(sh.sh_basis(-a, K), Ya * (-1.0) ** ls, atol=1e-14)
    rot = a * np.array([-1.0, -1.0, 1.0])
    assert np.allclose(sh.sh_basis(rot, K), Ya * (-1.0) ** ms, atol=1e-14)


def test_sh_basis_orthonormal_and_textbook_low_orders():
    """Gauss-Legendre x uniform-azimuth quadrature gives the identity Gram
    matrix; the first orders equal the textbook polynomials."""
    K = 16
    xs, ws = np.polynomial.legendre.leggauss(24)
    phis = np.linspace(0, 2 * math.pi, 48, endpoint=False)
    z = np.repeat(xs, phis.size)
    w = np.repeat(ws, phis.size) * (2 * math.pi / phis.size)
    ph = np.tile(phis, xs.size)
    r = np.sqrt(1 - z * z)
    d = np.stack([r * np.cos(ph), r * np.sin(ph), z], 1)
    Y = sh.sh_basis(d, K)
    G = (Y * w[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(K))) < 1e-12
    rng = np.random.default_rng(1)
    v = _unit(rng, 50)
    x, y, zz = v[:, 0], v[:, 1], v[:, 2]
    Y = sh.sh_basis(v, 9)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 0], 0.5 / math.sqrt(math.pi))
    assert np.allclose(Y[:, 1:4], c1 * np.stack([y, zz, x], 1))
    assert np.allclose(Y[:, 4], 0.5 * math.sqrt(15 / math.pi) * x * y)
    assert np.allclose(Y[:, 6], 0.25 * math.sqrt(5 / math.pi) * (3 * zz * zz - 1))
    assert np.allclose(Y[:, 8], 0.25 * math.sqrt(15 / math.pi) * (x * x - y * y))


# ---------------------------------------------------------------------------
# BRDF coefficients (Eq. brdf, App. A)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("s", [1.0, 2.5, 7.0, 20.0])
def test_phong_coefficients_match_the_legendre_projection_of_the_clamped_lobe(s):
    """App. A's ratio g_l(s) is (s+1) int_0^1 x^s P_l(x) dx: the coefficient of
    the lobe (s+1)/(2 pi) max(0, x)^s on (2l+1)/(4 pi) P_l (pi-normalised so
    that the lobe integrates to 1 over the hemisphere)."""
    for l in range(8):
        q, _ = scipy.integrate.quad(lambda x: x ** s * scipy.special.eval_legendre(l, x), 0, 1, epsabs=1e-14,
                                    epsrel=1e-13)
        assert abs(sh.phong_lobe(s, l) - (s + 1) * q) < 1e-10, l
        h = 1e-6
        fd = (sh.phong_lobe(s + h, l) - sh.phong_lobe(s - h, l)) / (2 * h)
        assert abs(sh.phong_lobe_ds(s, l) - fd) < 1e-7


def test_brdf_in_the_local_frame_is_a_lobe_about_the_mirror_direction():
    """Local-frame reading of c_lm = (-1)^m c_l0: the response
    Y(w_O)^T (f^c (.) Ybar(w_I)) is sum_l c_l0 (2l+1)/(4 pi) P_l(w_O . m) with m
    the mirror image of the light direction d = -w_I about the normal z."""
    rng = np.random.default_rng(2)
    K = 16
    k, ad, as_, s = np.array([0.3]), np.array([[0.5, 0.4, 0.3]]), np.array([[0.6, 0.7, 0.8]]), np.array([5.0])
    fc = sh.brdf_coefficients(k, ad, as_, s, K)[0, :, 0]
    d = _unit(rng, 200)
    wo = _unit(rng, 200)
    mirror = d * np.array([-1.0, -1.0, 1.0])
    lhs = np.sum(sh.sh_basis(wo, K) * fc[None, :] * sh.sh_basis(d, K), axis=1)
    cosm = np.sum(wo * mirror, axis=1)
    c_l0 = [fc[l * l + l] for l in range(4)]
    rhs = sum(c_l0[l] * (2 * l + 1) / (4 * math.pi) * scipy.special.eval_legendre(l, cosm) for l in range(4))
    assert np.max(np.abs(lhs - rhs)) < 1e-13
    # Lambertian part: 4 k a^d Y00^2 = k a^d / pi, and the specular DC is (1-k) a^s / (4 pi)
    assert abs(fc[0] / (4 * math.pi) - (0.3 * 0.5 / math.pi + 0.7 * 0.6 / (4 * math.pi))) < 1e-15


def test_brdf_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    N, K = 6, 16
    o = rng.uniform(0.5, 0.95, N).astype(np.float32)
    k = rng.uniform(0.1, 0.9, N)
    ad, as_ = rng.uniform(0.1, 0.9, (N, 3)), rng.uniform(0.1, 0.9, (N, 3))
    s = rng.uniform(1.5, 12.0, N)
    G = rng.standard_normal((N, K, 3))

    def L(o_, k_, ad_, as__, s_):
        return float(np.sum(G * sh.reflectance_sh(o_, k_, ad_, as__, s_, K)))

    g_o, g_k, g_ad, g_as, g_s = sh.brdf_backward(o, k, ad, as_, s, K, G)
    h = 1e-6
    for i in range(N):
        def bump(arr, idx, dh):
            b = np.array(arr, np.float64, copy=True)
            b[idx] += dh
            return b
        fd = (L(o, bump(k, i, h), ad, as_, s) - L(o, bump(k, i, -h), ad, as_, s)) / (2 * h)
        assert abs(fd - g_k[i]) < 1e-6 * (1 + abs(fd))
        fd = (L(o, k, ad, as_, bump(s, i, h)) - L(o, k, ad, as_, bump(s, i, -h))) / (2 * h)
        assert abs(fd - g_s[i]) < 1e-6 * (1 + abs(fd))
        for c in range(3):
            fd = (L(o, k, bump(ad, (i, c), h), as_, s) - L(o, k, bump(ad, (i, c), -h), as_, s)) / (2 * h)
            assert abs(fd - g_ad[i, c]) < 1e-6 * (1 + abs(fd))
            fd = (L(o, k, ad, bump(as_, (i, c), h), s) - L(o, k, ad, bump(as_, (i, c), -h), s)) / (2 * h)
            assert abs(fd - g_as[i, c]) < 1e-6 * (1 + abs(fd))
    # opacity: R is linear in o (inside the clamp)
    assert np.allclose(g_o, np.pi * np.sum(G * sh.brdf_coefficients(k, ad, as_, s, K), axis=(1, 2)))


# ---------------------------------------------------------------------------
# transfer and bounces (Eq. final-radiosity)
# ---------------------------------------------------------------------------
def _small(n=40, seed=4, k=6):
    sur = scenes.random_frame_surfels(n, seed=seed, extent=1.0, scale=(0.05, 0.1))
    rp, c, v = scenes.seeded_csr(n, k, seed=seed + 1, row_sum=0.6)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(n, n))
    return sur, F


def test_lambertian_transfer_equals_the_scalar_transport():
    """k = 1 (f^c = (4a, 0, ...)) and E with only DC coefficients: every
    coefficient of B equals the scalar B = E + o a F B (A1)."""
    sur, F = _small()
    n, K, nb = F.shape[0], 16, 5
    rng = np.random.default_rng(5)
    alb = rng.uniform(0.2, 0.8, (n, 3))
    R = sh.reflectance_sh(sur["opacity"], np.ones(n), alb, np.zeros((n, 3)), np.full(n, 3.0), K)
    E = np.zeros((n, 2, K, 3))
    E[:, :, 0, :] = rng.uniform(0, 1, (n, 2, 3))
    B = sh.bounce(F, sur, R, E, nb)
    Bs = orc.bounce(F, orc.rho(sur["opacity"], alb), E, nb)
    assert np.max(np.abs(B - Bs)) < 1e-14 * np.max(np.abs(Bs))


def test_transfer_and_its_adjoint_equal_the_assembled_operator():
    """transfer / transfer_T against the (N K 3)^2 matrix assembled entry by
    entry: forward is M X, the adjoint is M^T U (App. C: the backward
    propagates with the decay term reversed)."""
    sur, F = _small(n=12, k=4)
    n, K = F.shape[0], 9
    rng = np.random.default_rng(6)
    R = rng.uniform(0.1, 2.0, (n, K, 3))
    M = sh.dense_operator(F, sur, R, K)
    X = rng.standard_normal((n, 1, K, 3))
    U = rng.standard_normal((n, 1, K, 3))
    bases = sh.pair_bases(F, sur, K)
    fwd = sh._times_R(R, sh.transfer(F, bases, X, K), K)
    assert np.allclose(fwd.reshape(-1), M @ X.reshape(-1), atol=1e-13)
    adj = sh.transfer_T(F, bases, sh._times_R(R, U, K), K)
    assert np.allclose(adj.reshape(-1), M.T @ U.reshape(-1), atol=1e-13)


def test_bounce_matches_neumann_series_and_linear_solve():
    """B^(n) = sum_{k<=n} M^k E with the assembled M; n -> infinity equals
    (I - M)^-1 E."""
    sur, F = _small(n=10, k=3)
    n, K = F.shape[0], 4
    rng = np.random.default_rng(7)
    R = rng.uniform(0.1, 1.0, (n, K, 3))
    M = sh.dense_operator(F, sur, R, K)
    E = rng.uniform(0, 1, (n, 1, K, 3))
    e = E.reshape(-1)
    ref, p = e.copy(), e.copy()
    for _ in range(6):
        p = M @ p
        ref += p
    assert np.allclose(sh.bounce(F, sur, R, E, 6).reshape(-1), ref, atol=1e-13)
    rad = np.max(np.abs(np.linalg.eigvals(M)))
    assert rad < 0.9
    Binf = sh.bounce(F, sur, R, E, 400).reshape(-1)
    assert np.allclose(Binf, np.linalg.solve(np.eye(M.shape[0]) - M, e), atol=1e-12)


def test_adjoint_dot_product_and_finite_differences():
    """<g, B(E)> = <grad_E, E> (B is linear in E); central differences in R
    and in F entries for grad_R and grad_F."""
    sur, F = _small(n=30, k=5)
    n, K, Lt, nb = F.shape[0], 9, 2, 4
    rng = np.random.default_rng(8)
    R = rng.uniform(0.1, 1.5, (n, K, 3))
    E = rng.uniform(0, 1, (n, Lt, K, 3))
    g = rng.standard_normal((n, Lt, K, 3))
    B, tape = sh.bounce(F, sur, R, E, nb, keep_tape=True)
    gE, gR, gF = sh.adjoint(F, sur, R, tape, g)
    assert abs(np.sum(g * B) - np.sum(gE * E)) < 1e-12 * abs(np.sum(g * B))

    def loss(R_, F_):
        return float(np.sum(g * sh.bounce(F_, sur, R_, E, nb)))

    h = 1e-6
    for _ in range(12):
        i, a, c = rng.integers(n), rng.integers(K), rng.integers(3)
        Rp, Rm = R.copy(), R.copy()
        Rp[i, a, c] += h
        Rm[i, a, c] -= h
        fd = (loss(Rp, F) - loss(Rm, F)) / (2 * h)
        assert abs(fd - gR[i, a, c]) < 1e-6 * (1 + abs(fd))
    for _ in range(12):
        e = rng.integers(F.nnz)
        Fp, Fm = F.copy(), F.copy()
        Fp.data[e] += h
        Fm.data[e] -= h
        fd = (loss(R, Fp) - loss(R, Fm)) / (2 * h)
        assert abs(fd - gF[e]) < 1e-6 * (1 + abs(fd))


def test_direct_light_with_the_brdf():
    """Lambertian surfels: the SH direct light equals the scalar one on the
    DC coefficient and is zero elsewhere.  A pure-specular surfel lit along
    its normal sends towards the mirror direction (the normal) the peak of
    the truncated lobe, o I / h^2 sum_l c_l0 (2l+1)/(4 pi)."""
    sc = scenes.make_config("fruit_bowl", n=800)
    sur = sc.surfels
    n, K = sc.n, 16
    R = sh.reflectance_sh(sur["opacity"], np.ones(n), sc.albedo, np.zeros((n, 3)), np.full(n, 4.0), K)
    te = orc.default_t_eps(sur)
    Es, T = orc.direct_light(sur, sc.albedo, sc.light_pos, sc.light_I, K, te, return_T=True)
    E = sh.direct_light(sur, R, sc.light_pos, sc.light_I, T)
    # the scalar oracle forms the light vector in FP32 (the shadow ray's
    # direction), this one in FP64: they differ by that rounding only
    assert np.max(np.abs(E - Es)) < 1e-6 * np.max(np.abs(Es))
    assert not E[:, :, 1:, :].any()
    # one specular surfel at the origin facing +z, light on the normal at height h:
    # the outgoing radiance towards the mirror direction (the normal) is the
    # truncated lobe's peak o I / h^2 sum_l c_l (2l+1)/(4 pi)
    s1 = scenes.surfels_from_arrays([[0, 0, 0]], [[0, 0, 1]], [[1, 0, 0]], [[0, 1, 0]], [0.1], [0.1], [0.8])
    Rs = sh.reflectance_sh(s1["opacity"], np.zeros(1), np.zeros((1, 3)), np.full((1, 3), 0.5), np.array([6.0]), K)
    h = 2.0
    E1 = sh.direct_light(s1, Rs, [[0, 0, h]], [3.0], np.ones((1, 1)))
    Bup = sh.sh_basis(np.array([[0, 0, 1.0]]), K)[0] @ E1[0, 0, :, 0]
    peak = sum(0.5 * sh.phong_lobe(6.0, l) * (2 * l + 1) / (4 * math.pi) for l in range(4))
    assert abs(Bup - float(np.float32(0.8)) * 3.0 / h ** 2 * peak) < 1e-12
