"""Geometry gradients through the ray-cast form factors on the GPU (from
the recorded hits) against the FP64 oracle's (oracle.geometry_backward):
every surfel field at the FP32 bar of 1e-4 relative max-norm; the opacity
field against the compositing backward; determinism; the records
requirement."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("name,n,R,topk", [("fruit_bowl", 1500, 16, 0), ("box_room", 1200, 16, 48),
                                           ("layers", None, 24, 0)])
def test_geometry_gradients_match_oracle(g, orc, name, n, R, topk):
    if name == "layers":
        sur, seed = scenes.layer_stack(), 5
    else:
        sc = scenes.make_config(name, n=n)
        sur, seed = sc.surfels, sc.seed
    nn = sur["px"].shape[0]
    bvh = g.build_bvh(dev_surfels(sur))
    ff = g.form_factors(bvh, R, seed, t_min=1e-4, topk=topk)
    F = gpu_csr(ff)
    gF = np.random.default_rng(2).standard_normal(F.nnz).astype(np.float32)
    got = g.geometry_backward(bvh, ff, dev(gF))
    te = orc.default_t_eps(sur)
    ref = orc.geometry_backward(sur, R, seed, te, 1e-4, (F.indptr, F.indices, gF.astype(np.float64)))
    for f in orc.GEOMETRY_FIELDS:
        assert rel_err(got[f].cpu().numpy(), ref[f]) < TOL, f
    # the opacity field is the F part of the compositing backward
    go, _ = g.opacity_backward(bvh, ff, dev(gF), None, None)
    assert rel_err(got["opacity"].cpu().numpy(), go.cpu().numpy()) < 1e-6
    again = g.geometry_backward(bvh, ff, dev(gF))
    for f in orc.GEOMETRY_FIELDS:
        assert torch.equal(got[f], again[f]), f
    assert nn > 0


def test_geometry_backward_needs_records(g):
    sc = scenes.make_config("fruit_bowl", n=800)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, 8, sc.seed, records=False)
    with pytest.raises(g.GsradError) as ei:
        g.geometry_backward(bvh, ff, dev(np.ones(ff.info()[1], np.float32)))
    assert ei.value.status == g.gsrad.ESTATE


@pytest.mark.parametrize("name,n,Lt", [("fruit_bowl", 2000, 2), ("box_room", 1500, 3), ("layers", None, 2)])
def test_direct_light_gradients_match_oracle(g, orc, name, n, Lt):
    if name == "layers":
        sur = scenes.layer_stack()
        nn = sur["px"].shape[0]
        alb = np.full((nn, 3), 0.5, np.float32)
        lp = np.array([[0.0, 0.0, 2.5], [0.3, -0.2, 3.0]], np.float32)
    else:
        sc = scenes.make_config(name, n=n)
        sur, alb, nn = sc.surfels, sc.albedo, sc.n
        lp = np.random.default_rng(3).uniform(-0.5, 0.5, (Lt, 3)).astype(np.float32)
        lp[:, 1] += 1.2 if name == "fruit_bowl" else 2.5
    lI = np.linspace(1.0, 3.0, Lt).astype(np.float32)
    K = 4
    gE = np.random.default_rng(4).standard_normal((nn, Lt, K, 3)).astype(np.float32)
    bvh = g.build_bvh(dev_surfels(sur))
    glp, gli, gal, gs = g.direct_light_backward(bvh, dev(alb), dev(lp), dev(lI), dev(gE))
    te = orc.default_t_eps(sur)
    rlp, rli, ral, rs = orc.direct_light_backward(sur, alb, lp, lI, gE, t_eps=te)
    assert rel_err(glp.cpu().numpy(), rlp) < TOL
    assert rel_err(gli.cpu().numpy(), rli) < TOL
    assert rel_err(gal.cpu().numpy(), ral) < TOL
    for f in orc.GEOMETRY_FIELDS:
        assert rel_err(gs[f].cpu().numpy(), rs[f]) < TOL, f
    again = g.direct_light_backward(bvh, dev(alb), dev(lp), dev(lI), dev(gE))
    assert torch.equal(again[0], glp) and torch.equal(again[1], gli)
    for f in orc.GEOMETRY_FIELDS:
        assert torch.equal(again[3][f], gs[f]), f
