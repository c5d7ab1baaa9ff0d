"""Edge cases of the centre-to-centre form factors, the geometry gradients,
the directional transfer and the Monte-Carlo solver on the GPU against the
FP64 oracle: hand-made patterns with ragged rows (empty rows, rows longer
than a wave), scenes of one, two and three surfels, an empty operator,
zero upstream gradients, and the extreme group counts of the solver."""
import math

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


def _facing(k):
    """k surfels: receiver 0 at the origin facing +z, the others on a
    tilted ring at height 1 facing down toward it."""
    p, nrm = [[0.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]]
    for q in range(1, k):
        a = 2 * math.pi * q / max(k - 1, 1)
        c = np.array([0.3 * math.cos(a), 0.3 * math.sin(a), 1.0])
        p.append(c.tolist())
        d = -c / np.linalg.norm(c)
        nrm.append(d.tolist())
    nrm = np.array(nrm)
    tu, tv = scenes.onb_from_normal(nrm)
    s = np.full(k, 0.1)
    return scenes.surfels_from_arrays(np.array(p), nrm, tu, tv, s, s, np.full(k, 0.8))


def _csr_pattern(n, rows_len, seed):
    """A pattern with the given row lengths (distinct columns, no diagonal)."""
    rng = np.random.default_rng(seed)
    rp, cols = [0], []
    for i, m in enumerate(rows_len):
        cand = np.setdiff1d(np.arange(n), [i])
        c = np.sort(rng.choice(cand, size=min(m, cand.size), replace=False))
        cols.append(c)
        rp.append(rp[-1] + c.size)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    return np.array(rp, np.int64), col


def test_center_on_a_ragged_hand_made_pattern(g):
    """Rows of 0, 1, 63, 64, 65 and 130 entries (empty, within, at and past a
    wave's lanes) between arbitrary surfels of the box room, most segments
    crossing occluders."""
    from oracle import center
    sc = scenes.make_config("box_room", n=800)
    n = sc.n
    lens = [0, 1, 63, 64, 65, 130] + [7] * (n - 6)
    rp, col = _csr_pattern(n, lens, seed=3)
    lam = scenes.seeded_array((n,), seed=4, lo=0.5, hi=1.5)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    pat = g.ff_from_csr(dev(rp), dev(col), dev(np.ones(col.size, np.float32)))
    ff = g.ff_center(bvh, pat, dev(lam))
    F = gpu_csr(ff)
    rows = np.repeat(np.arange(n), np.diff(rp))
    Fo, T = center.center_ff(sc.surfels, rows, col, lam)
    assert np.array_equal(F.indices, col)
    assert rel_err(F.data, Fo) < TOL
    assert np.mean(T < 0.5) > 0.1
    G = np.random.default_rng(5).standard_normal(col.size).astype(np.float32)
    gl, gf = g.ff_center_backward(bvh, ff, dev(lam), dev(G))
    glo, gfo = center.center_backward(sc.surfels, rows, col, lam, G)
    assert rel_err(gl.cpu().numpy(), glo) < TOL
    for f in center.FIELDS:
        assert rel_err(gf[f].cpu().numpy(), gfo[f]) < TOL, f
    # zero upstream gradient: every output exactly zero
    gl0, gf0 = g.ff_center_backward(bvh, ff, dev(lam), dev(np.zeros_like(G)))
    assert not gl0.any() and all(not v.any() for v in gf0.values())


@pytest.mark.parametrize("k", [1, 2, 3])
def test_center_on_tiny_scenes(g, k):
    from oracle import center
    sur = _facing(k)
    rp, col = _csr_pattern(k, [k - 1] * k, seed=1)
    lam = np.linspace(0.7, 1.3, k).astype(np.float32)
    bvh = g.build_bvh(dev_surfels(sur))
    pat = g.ff_from_csr(dev(rp), dev(col), dev(np.ones(max(col.size, 0), np.float32)))
    ff = g.ff_center(bvh, pat, dev(lam))
    F = gpu_csr(ff)
    assert F.nnz == col.size
    G = np.linspace(-1, 2, col.size).astype(np.float32)
    gl, gf = g.ff_center_backward(bvh, ff, dev(lam), dev(G))
    if col.size == 0:
        assert not gl.any() and all(not v.any() for v in gf.values())
        return
    rows = np.repeat(np.arange(k), np.diff(rp))
    Fo, _ = center.center_ff(sur, rows, col, lam.astype(np.float64))
    assert rel_err(F.data, Fo) < TOL
    glo, gfo = center.center_backward(sur, rows, col, lam.astype(np.float64), G)
    assert rel_err(gl.cpu().numpy(), glo) < TOL
    for f in center.FIELDS:
        assert rel_err(gf[f].cpu().numpy(), gfo[f]) < TOL, f


@pytest.mark.parametrize("k", [1, 2, 3])
def test_geometry_gradients_on_tiny_scenes(g, orc, k):
    sur = _facing(k)
    R, seed = 64, 11
    bvh = g.build_bvh(dev_surfels(sur))
    ff = g.form_factors(bvh, R, seed, t_min=1e-4)
    F = gpu_csr(ff)
    gF = np.linspace(-1, 1, max(F.nnz, 1)).astype(np.float32)[:F.nnz]
    got = g.geometry_backward(bvh, ff, dev(gF) if F.nnz else torch.zeros(0, device="cuda"))
    if F.nnz == 0:
        assert all(not v.any() for v in got.values())
        return
    te = orc.default_t_eps(sur)
    ref = orc.geometry_backward(sur, R, seed, te, 1e-4, (F.indptr, F.indices, gF.astype(np.float64)))
    for f in orc.GEOMETRY_FIELDS:
        assert rel_err(got[f].cpu().numpy(), ref[f]) < TOL, f
    zero = g.geometry_backward(bvh, ff, dev(np.zeros(F.nnz, np.float32)))
    assert all(not v.any() for v in zero.values())


def test_directional_transfer_on_an_empty_operator(g):
    """One surfel (no pairs): every bounce leaves B = E; the adjoint gives
    grad_E = grad_B and zero grad_R."""
    sur = _facing(1)
    bvh = g.build_bvh(dev_surfels(sur))
    ff = g.form_factors(bvh, 32, 3)
    assert ff.info()[1] == 0
    K = 9
    R = dev(scenes.seeded_array((1, K, 3), seed=1))
    E = dev(scenes.seeded_array((1, 2, K, 3), seed=2))
    gB = dev(scenes.seeded_array((1, 2, K, 3), seed=3, lo=-1, hi=1))
    B, tape = g.transport_solve_sh(ff, bvh, R, E, 4)
    assert torch.equal(B, E)
    gE, gR, gF = g.transport_backward_sh(ff, bvh, tape, R, gB)
    assert torch.equal(gE, gB) and not gR.any()


@pytest.mark.parametrize("groups", [1, "n"])
def test_one_point_estimate_unbiased_at_extreme_group_counts(g, groups):
    """One group (the member draw covers every surfel) and one group per
    surfel (the group draw alone decides): the estimate's mean over 768
    seeds equals E + rho (F B) within six standard errors."""
    from oracle import center
    from oracle import oracle as orc
    sc = scenes.make_config("box_room", n=200)
    sur, n = sc.surfels, sc.n
    bvh = g.build_bvh(dev_surfels(sur))
    lam = np.full(n, 0.5, np.float32)
    rho = orc.rho(sur["opacity"], sc.albedo).astype(np.float32)
    E = orc.direct_light(sur, sc.albedo, sc.light_pos, sc.light_I, 1).astype(np.float32)
    rows, cols = np.nonzero(~np.eye(n, dtype=bool))
    Fv, _ = center.center_ff(sur, rows, cols.astype(np.int32), lam)
    F = sp.csr_matrix((Fv, (rows, cols)), shape=(n, n))
    Bcur = E + 0.05 * scenes.seeded_array(E.shape, seed=3, lo=0.5, hi=1.5)
    expect = E + rho[:, None, None, :] * (F @ Bcur.reshape(n, -1)).reshape(Bcur.shape)
    mc = g.mc_create(bvh, groups=(n if groups == "n" else 1), kmeans_iters=4)
    lam_d, rho_d, E_d, B_d = dev(lam), dev(rho), dev(E), dev(Bcur)
    M = 768
    acc = torch.zeros_like(E_d, dtype=torch.float64)
    acc2 = torch.zeros_like(E_d, dtype=torch.float64)
    for s in range(M):
        d = g.mc_estimate(mc, lam_d, rho_d, E_d, B_d, seed=77 + s).double()
        acc += d
        acc2 += d * d
    mean = (acc / M).cpu().numpy()
    var = (acc2 / M).cpu().numpy() - mean ** 2
    se = np.sqrt(np.maximum(var, 0) / M)
    excess = np.abs(mean - expect) - 6 * se - 1e-6 * np.abs(expect)
    assert np.all(excess <= 0), float(np.max(excess))
