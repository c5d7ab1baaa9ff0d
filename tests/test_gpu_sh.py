"""The directional (SH) transfer with the diffuse + Phong BRDF on the GPU
(libgsrad through its C ABI) against the FP64 oracle (oracle/sh.py):
BRDF coefficients and their backward, direct light through the BRDF,
bounces and the exact adjoint on ray-cast and seeded operators, at the
FP32 bar of 1e-4 relative max-norm; the Lambertian limit against the
scalar path; determinism; the 100k fruit bowl's launch on sampled rows."""
import numpy as np
import pytest
import scipy.sparse as sp

import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests.gpu_common import dev, dev_surfels, gpu_csr, rel_err  # noqa: E402

TOL = 1e-4


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_18497_amd as g
    g.gsrad.lib()
    return g


@pytest.fixture(scope="module")
def osh():
    from oracle import sh
    return sh


def _mats(n, seed):
    m = scenes.phong_materials(n, seed)
    return m, {k: dev(v) for k, v in m.items()}


def _R(g, bvh, md, K):
    return g.brdf_reflectance(bvh, md["k"], md["albedo_d"], md["albedo_s"], md["shininess"], K)


@pytest.mark.parametrize("K", [1, 4, 9, 16])
def test_brdf_reflectance_and_backward(g, osh, K):
    sc = scenes.make_config("fruit_bowl", n=1000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    m, md = _mats(sc.n, 3)
    R = _R(g, bvh, md, K).cpu().numpy()
    Ro = osh.reflectance_sh(sc.surfels["opacity"], m["k"], m["albedo_d"], m["albedo_s"], m["shininess"], K)
    assert rel_err(R, Ro) < TOL
    G = scenes.seeded_array((sc.n, K, 3), seed=4, lo=-1, hi=1)
    outs = g.brdf_backward(bvh, md["k"], md["albedo_d"], md["albedo_s"], md["shininess"], dev(G))
    refs = osh.brdf_backward(sc.surfels["opacity"], m["k"], m["albedo_d"], m["albedo_s"], m["shininess"], K, G)
    for name, a, b in zip(("o", "k", "ad", "as", "s"), outs, refs):
        if K == 1 and name == "s":
            assert not a.any()
            continue
        assert rel_err(a.cpu().numpy(), b) < TOL, name


@pytest.mark.parametrize("K", [4, 16])
def test_direct_light_through_the_brdf(g, orc, osh, K):
    sc = scenes.make_config("fruit_bowl", n=3000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    m, md = _mats(sc.n, 5)
    R = _R(g, bvh, md, K)
    lp = np.array([[0.3, 1.5, 0.2], [-0.6, 0.9, 0.4]], np.float32)
    lI = np.array([4.0, 2.0], np.float32)
    E = g.direct_light_sh(bvh, R, dev(lp), dev(lI)).cpu().numpy()
    te = orc.default_t_eps(sc.surfels)
    _, T = orc.direct_light(sc.surfels, sc.albedo, lp, lI, 1, te, return_T=True)
    Ro = osh.reflectance_sh(sc.surfels["opacity"], m["k"], m["albedo_d"], m["albedo_s"], m["shininess"], K)
    Eo = osh.direct_light(sc.surfels, Ro, lp, lI, T)
    assert rel_err(E, Eo) < TOL
    assert np.abs(Eo[:, :, 1:]).max() > 0.05 * np.abs(Eo).max()      # the specular part is there


def _ray_cast(g, name, n, R, seed, topk=0):
    sc = scenes.make_config(name, n=n)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, R, sc.seed if seed is None else seed, t_min=1e-4, topk=topk)
    return sc, bvh, ff


@pytest.mark.parametrize("name,n,K,Lt,nb,topk", [("fruit_bowl", 3000, 16, 1, 4, 0), ("box_room", 2500, 9, 2, 3, 64),
                                                 ("fruit_bowl", 2000, 4, 3, 1, 0)])
def test_transfer_bounces_and_adjoint_on_ray_cast_operators(g, osh, name, n, K, Lt, nb, topk):
    sc, bvh, ff = _ray_cast(g, name, n, 32, None, topk)
    F = gpu_csr(ff)
    m, md = _mats(sc.n, 6)
    R = _R(g, bvh, md, K)
    E = scenes.seeded_array((sc.n, Lt, K, 3), seed=7)
    gB = scenes.seeded_array((sc.n, Lt, K, 3), seed=8, lo=-1, hi=1)
    B, tape = g.transport_solve_sh(ff, bvh, R, dev(E), nb)
    gE, gR, gF = g.transport_backward_sh(ff, bvh, tape, R, dev(gB))
    Ro = R.cpu().numpy().astype(np.float64)           # the same FP32 R on both sides
    Bo, tp = osh.bounce(F, sc.surfels, Ro, E, nb, keep_tape=True)
    gEo, gRo, gFo = osh.adjoint(F, sc.surfels, Ro, tp, gB)
    assert rel_err(B.cpu().numpy(), Bo) < TOL
    assert rel_err(gE.cpu().numpy(), gEo) < TOL
    assert rel_err(gR.cpu().numpy(), gRo) < TOL
    assert rel_err(gF.cpu().numpy(), gFo) < TOL


@pytest.mark.parametrize("n,k,K,Lt,nb", [(700, 40, 16, 1, 2), (1500, 130, 9, 2, 3), (65, 64, 16, 1, 1),
                                         (3, 2, 4, 1, 5)])
def test_transfer_on_seeded_operators_and_tiny_sizes(g, osh, n, k, K, Lt, nb):
    """Rows longer than one wave (130 entries), empty rows, n = 3 and 65."""
    sur = scenes.random_frame_surfels(n, seed=n, extent=1.0, scale=(0.05, 0.1))
    bvh = g.build_bvh(dev_surfels(sur))
    rp, c, v = scenes.seeded_csr(n, k, seed=n + 1)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(n, n))
    Rh = scenes.seeded_array((n, K, 3), seed=2, lo=0.0, hi=2.0)
    E = scenes.seeded_array((n, Lt, K, 3), seed=3)
    gB = scenes.seeded_array((n, Lt, K, 3), seed=4, lo=-1, hi=1)
    B, tape = g.transport_solve_sh(ff, bvh, dev(Rh), dev(E), nb)
    gE, gR, gF = g.transport_backward_sh(ff, bvh, tape, dev(Rh), dev(gB))
    Bo, tp = osh.bounce(F, sur, Rh, E, nb, keep_tape=True)
    gEo, gRo, gFo = osh.adjoint(F, sur, Rh, tp, gB)
    assert rel_err(B.cpu().numpy(), Bo) < TOL
    assert rel_err(gE.cpu().numpy(), gEo) < TOL
    assert rel_err(gR.cpu().numpy(), gRo) < TOL
    if F.nnz:
        assert rel_err(gF.cpu().numpy(), gFo) < TOL


def test_lambertian_limit_equals_the_scalar_path_and_is_deterministic(g):
    """k = 1 materials and point-light E (DC only): the directional transfer
    equals gsrad_transport_solve (within FP32 rounding) on every coefficient,
    and repeated runs are bit-identical."""
    sc, bvh, ff = _ray_cast(g, "fruit_bowl", 3000, 32, None)
    K, nb = 9, 4
    alb = dev(sc.albedo)
    kk = torch.ones(sc.n, device="cuda")
    R = g.brdf_reflectance(bvh, kk, alb, torch.zeros_like(alb), torch.full_like(kk, 5.0), K)
    E = g.direct_light(bvh, alb, dev(sc.light_pos), dev(sc.light_I), K)
    Esh = g.direct_light_sh(bvh, R, dev(sc.light_pos), dev(sc.light_I))
    assert rel_err(Esh.cpu().numpy(), E.cpu().numpy()) < 1e-6
    rho = g.reflectance(bvh, alb)
    Bs, _ = g.transport_solve(ff, rho, E, nb)
    B1, _ = g.transport_solve_sh(ff, bvh, R, E, nb)
    B2, _ = g.transport_solve_sh(ff, bvh, R, E, nb)
    assert rel_err(B1.cpu().numpy(), Bs.cpu().numpy()) < 1e-5
    assert torch.equal(B1, B2)
    gB = dev(scenes.seeded_array(tuple(E.shape), seed=9, lo=-1, hi=1))
    _, t1 = g.transport_solve_sh(ff, bvh, R, E, nb)
    a = g.transport_backward_sh(ff, bvh, t1, R, gB)
    b = g.transport_backward_sh(ff, bvh, t1, R, gB)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_sh_tape_is_refused_by_the_scalar_backward(g):
    sc, bvh, ff = _ray_cast(g, "furnace", None, 16, None)
    K = 4
    R = dev(scenes.seeded_array((sc.n, K, 3), seed=1))
    E = dev(scenes.seeded_array((sc.n, 1, K, 3), seed=2))
    _, tape = g.transport_solve_sh(ff, bvh, R, E, 2)
    with pytest.raises(g.GsradError):
        g.transport_backward(ff, tape, dev(np.full((sc.n, 3), 0.5, np.float32)), E)


def test_sh_tape_is_refused_after_the_geometry_is_rebuilt(g):
    """The directional transfer's tape records the BVH (the pair directions)
    it used: after an in-place rebuild the backward refuses it."""
    sc, bvh, ff = _ray_cast(g, "furnace", None, 16, None)
    K = 4
    R = dev(scenes.seeded_array((sc.n, K, 3), seed=1))
    E = dev(scenes.seeded_array((sc.n, 1, K, 3), seed=2))
    gB = dev(scenes.seeded_array((sc.n, 1, K, 3), seed=3, lo=-1, hi=1))
    _, tape = g.transport_solve_sh(ff, bvh, R, E, 2)
    g.transport_backward_sh(ff, bvh, tape, R, gB)
    g.build_bvh(dev_surfels(sc.surfels), bvh)
    with pytest.raises(g.GsradError):
        g.transport_backward_sh(ff, bvh, tape, R, gB)
