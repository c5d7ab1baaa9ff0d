"""Centre-to-centre form factors with a learnable scale (Sec. 8) and their
gradients on the GPU against the FP64 oracle (oracle/center.py), on the
pattern a ray cast recorded: values and every gradient field at the FP32
bar of 1e-4 relative max-norm, determinism, provenance checks."""
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


@pytest.fixture(scope="module")
def ocenter():
    from oracle import center
    return center


def _setup(g, name, n, R, seed=0):
    sc = scenes.make_config(name, n=n)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    pat = g.form_factors(bvh, R, sc.seed, t_min=1e-4)
    lam = scenes.seeded_array((sc.n,), seed=seed + 7, lo=0.5, hi=1.5)
    return sc, bvh, pat, lam


@pytest.mark.parametrize("name,n,R", [("fruit_bowl", 1500, 16), ("box_room", 1200, 16), ("furnace", None, 32)])
def test_center_form_factors_match_oracle(g, ocenter, name, n, R):
    sc, bvh, pat, lam = _setup(g, name, n, R)
    ff = g.ff_center(bvh, pat, dev(lam))
    Fp = gpu_csr(pat)
    Fc = gpu_csr(ff)
    assert np.array_equal(Fc.indptr, Fp.indptr) and np.array_equal(Fc.indices, Fp.indices)
    rows = np.repeat(np.arange(sc.n), np.diff(Fp.indptr))
    Fo, T = ocenter.center_ff(sc.surfels, rows, Fp.indices, lam)
    assert rel_err(Fc.data, Fo) < TOL
    if name == "furnace":
        assert np.min(T) == 1.0       # inside a sphere nothing occludes a chord
    else:
        assert np.min(T) < 0.9        # some segments are occluded
    # usable as a transport operator
    E = dev(scenes.seeded_array((sc.n, 1, 1, 3), seed=3))
    B, _ = g.transport_solve(ff, dev(np.full((sc.n, 3), 0.5, np.float32)), E, 3)
    assert torch.isfinite(B).all()


@pytest.mark.parametrize("name,n,R", [("fruit_bowl", 1500, 16), ("box_room", 1200, 16)])
def test_center_gradients_match_oracle(g, ocenter, name, n, R):
    sc, bvh, pat, lam = _setup(g, name, n, R, seed=1)
    ff = g.ff_center(bvh, pat, dev(lam))
    Fp = gpu_csr(ff)
    G = np.random.default_rng(9).standard_normal(Fp.nnz).astype(np.float32)
    gl, gf = g.ff_center_backward(bvh, ff, dev(lam), dev(G))
    rows = np.repeat(np.arange(sc.n), np.diff(Fp.indptr))
    glo, gfo = ocenter.center_backward(sc.surfels, rows, Fp.indices, lam, G)
    assert rel_err(gl.cpu().numpy(), glo) < TOL
    for f in ocenter.FIELDS:
        assert rel_err(gf[f].cpu().numpy(), gfo[f]) < TOL, f
    # bit-identical between runs
    gl2, gf2 = g.ff_center_backward(bvh, ff, dev(lam), dev(G))
    assert torch.equal(gl, gl2)
    for f in ocenter.FIELDS:
        assert torch.equal(gf[f], gf2[f]), f


def test_center_provenance(g):
    sc, bvh, pat, lam = _setup(g, "fruit_bowl", 800, 8)
    ff = g.ff_center(bvh, pat, dev(lam))
    G = dev(np.ones(ff.info()[1], np.float32))
    with pytest.raises(g.GsradError):                      # not a ray cast: no compositing backward
        g.opacity_backward(bvh, ff, G, None, None)
    with pytest.raises(g.GsradError):                      # the output must differ from the pattern
        g.ff_center(bvh, pat, dev(lam), ff=pat)
    d = dev_surfels(sc.surfels)
    g.build_bvh(d, bvh=bvh)                                 # rebuilt in place
    with pytest.raises(g.GsradError):
        g.ff_center_backward(bvh, ff, dev(lam), G)
    ff = g.ff_center(bvh, pat, dev(lam), ff=ff)
    gl, _ = g.ff_center_backward(bvh, ff, dev(lam), G)
    assert torch.isfinite(gl).all()
