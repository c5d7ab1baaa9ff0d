"""GPU path (libgsrad through its C ABI) against the FP64 oracle.

Bars: ray directions and hit lists bit-exact; FP32 results within a
relative max-norm error of 1e-4 (form factors, direct light, bounces,
gradients), as stated for FP32 results of this path.
"""
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


def _scene(name, n=None, **kw):
    return scenes.make_config(name, n=n, **kw)


SMALL = [
    ("furnace", dict(), 64, 0),
    ("box_room", dict(n=2500), 32, 0),
    ("fruit_bowl", dict(n=3000), 32, 0),
    ("fruit_bowl", dict(n=3000), 32, 48),
]


# ---------------------------------------------------------------------------
# geometry, rays and hits
# ---------------------------------------------------------------------------
def test_t_eps_and_area_match_oracle(g, orc):
    sc = _scene("fruit_bowl", n=5000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    n, te = bvh.info()
    assert n == sc.n
    assert np.float32(te) == orc.default_t_eps(sc.surfels)
    A = g.effective_area(bvh).cpu().numpy()
    ref = orc.effective_area(sc.surfels["su"], sc.surfels["sv"], sc.surfels["opacity"])
    assert np.max(np.abs(A - ref) / ref) < 1e-12
    assert 0 < bvh.height() < 48


@pytest.mark.parametrize("name,kw,R,seed", [("fruit_bowl", dict(n=3000), 32, 3), ("box_room", dict(n=2000), 32, 2),
                                            ("furnace", dict(), 64, 1)])
def test_ray_directions_and_hit_lists_bit_exact(g, orc, name, kw, R, seed):
    sc = _scene(name, **kw)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    te = orc.default_t_eps(sc.surfels)
    rng = np.random.default_rng(0)
    recv = np.sort(rng.choice(sc.n, size=12, replace=False)).astype(np.int64)
    out = g.ray_hits(bvh, dev(recv), R, seed, t_min=1e-4, max_hits=512)
    dirs = out["dirs"].cpu().numpy()
    cnt = out["count"].cpu().numpy()
    hj = out["j"].cpu().numpy()
    ht = out["t"].cpu().numpy()
    hf = out["front"].cpu().numpy()
    hT = out["T"].cpu().numpy()
    compared = 0
    for k, i in enumerate(recv):
        for r in range(R):
            ref = orc.trace_ray(sc.surfels, int(i), r, seed, te, 1e-4)
            assert np.array_equal(dirs[k, r].view(np.uint32), ref["d"].view(np.uint32)), (i, r)
            # the cut is decided on the same FP32 transmittance on both sides
            m = ref["n_comp"]
            assert int(cnt[k, r]) == m, (i, r, int(cnt[k, r]), m)
            assert np.array_equal(hj[k, r, :m], ref["j"][:m]), (i, r)
            assert np.array_equal(ht[k, r, :m].view(np.uint32), ref["t"][:m].view(np.uint32)), (i, r)
            assert np.array_equal(hf[k, r, :m].astype(bool), ref["front"][:m]), (i, r)
            assert np.array_equal(hT[k, r, :m].view(np.uint32), ref["T32"][:m].view(np.uint32)), (i, r)
            compared += 1
    assert compared == len(recv) * R


# ---------------------------------------------------------------------------
# form factors
# ---------------------------------------------------------------------------
def _ff_compare(g, orc, sc, R, topk, seed=None):
    seed = sc.seed if seed is None else seed
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, R, seed, t_min=1e-4, topk=topk)
    Fg = gpu_csr(ff)
    te = orc.default_t_eps(sc.surfels)
    Fo, diag = orc.ff_matrix(sc.surfels, R, seed, te, 1e-4, topk)
    return Fg, Fo, bvh, ff


@pytest.mark.parametrize("name,kw,R,topk", SMALL)
def test_form_factors_match_oracle(g, orc, name, kw, R, topk):
    sc = _scene(name, **kw)
    Fg, Fo, _, _ = _ff_compare(g, orc, sc, R, topk)
    D = (Fg - Fo).toarray() if sc.n <= 4000 else None
    err = np.max(np.abs(D)) / np.max(np.abs(Fo.data))
    assert err < TOL, err
    if topk == 0:
        # same sparsity except entries created or dropped by a cut that sits
        # on the threshold (weights <= t_min / R)
        diff = (Fg != 0).astype(int) - (Fo != 0).astype(int)
        assert abs(diff).sum() <= max(4, Fo.nnz // 20000)
    else:
        assert np.all(np.diff(Fg.indptr) <= topk)
    # rows are sorted and F's row sums stay below one
    for i in range(0, sc.n, max(1, sc.n // 50)):
        cols = Fg.indices[Fg.indptr[i]:Fg.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
    assert np.asarray(Fg.sum(axis=1)).max() <= 1.0 + 1e-6


def test_reused_handles_follow_new_surfels(g, orc):
    """An optimisation loop reuses its BVH and F handles while opacities
    and positions change: each re-cast on the reused handles equals a cast
    on fresh handles bit for bit, and matches the oracle."""
    sc = _scene("fruit_bowl", n=2500)
    sur = {k: v.copy() for k, v in sc.surfels.items()}
    bvh = g.build_bvh(dev_surfels(sur))
    ff = g.form_factors(bvh, 32, sc.seed, t_min=1e-4, topk=48)
    rng = np.random.default_rng(5)
    for it in range(3):
        sur["opacity"] = np.clip(sur["opacity"] * rng.uniform(0.8, 1.0, sur["opacity"].shape), 0.05, 0.99
                                 ).astype(np.float32)
        sur["px"] = (sur["px"] + rng.normal(0, 1e-3, sur["px"].shape)).astype(np.float32)
        bvh = g.build_bvh(dev_surfels(sur), bvh)
        ff = g.form_factors(bvh, 32, sc.seed, t_min=1e-4, topk=48, ff=ff)
        fresh = g.form_factors(g.build_bvh(dev_surfels(sur)), 32, sc.seed, t_min=1e-4, topk=48)
        for x, y in zip(ff.csr(), fresh.csr()):
            assert torch.equal(x, y), it
    Fg = gpu_csr(ff)
    Fo, _ = orc.ff_matrix(sur, 32, sc.seed, orc.default_t_eps(sur), 1e-4, 48)
    assert rel_err(Fg.toarray(), Fo.toarray()) < TOL


def test_form_factors_are_deterministic(g):
    sc = _scene("fruit_bowl", n=6000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    a = g.form_factors(bvh, 64, 11, topk=64).csr()
    b = g.form_factors(bvh, 64, 11, topk=64).csr()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("n", [1, 2, 3, 65])
def test_form_factors_tiny_scenes(g, orc, n):
    sur = scenes.random_frame_surfels(n, seed=40 + n, extent=0.3, scale=(0.1, 0.3), opacity=(0.5, 0.99))
    bvh = g.build_bvh(dev_surfels(sur))
    ff = g.form_factors(bvh, 100, 5, t_min=1e-4)
    Fg = gpu_csr(ff)
    Fo, _ = orc.ff_matrix(sur, 100, 5, None, 1e-4, 0)
    if Fo.nnz == 0:
        assert Fg.nnz == 0
    else:
        assert rel_err(Fg.toarray(), Fo.toarray()) < TOL


def test_form_factors_rays_not_multiple_of_wave(g, orc):
    sc = _scene("box_room", n=1500)
    Fg, Fo, _, _ = _ff_compare(g, orc, sc, 45, 0, seed=9)
    assert rel_err(Fg.toarray(), Fo.toarray()) < TOL


@pytest.mark.parametrize("R,topk,n", [(1, 1, 800), (1, 0, 800), (1100, 0, 300), (64, 1, 800)])
def test_form_factors_degenerate_ray_counts_and_topk(g, orc, R, topk, n):
    """One ray per receiver, more rays than one 1024-ray pool, and top-1
    rows (the selection keeps the largest entry, ties by column)."""
    sc = _scene("box_room", n=n)
    Fg, Fo, _, _ = _ff_compare(g, orc, sc, R, topk, seed=21)
    assert rel_err(Fg.toarray(), Fo.toarray()) < TOL
    if topk:
        assert np.all(np.diff(Fg.indptr) <= topk)


# ---------------------------------------------------------------------------
# direct light
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,kw,K", [("furnace", {}, 1), ("box_room", dict(n=3000), 9),
                                       ("fruit_bowl", dict(n=4000), 16), ("multi_light", dict(n=2000), 4)])
def test_direct_light_matches_oracle(g, orc, name, kw, K):
    sc = _scene(name, **kw)
    lights = sc.light_pos[:8]
    li = sc.light_I[:8]
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    E = g.direct_light(bvh, dev(sc.albedo), dev(lights), dev(li), K).cpu().numpy()
    ref = orc.direct_light(sc.surfels, sc.albedo, lights, li, K)
    assert rel_err(E, ref) < TOL
    assert np.all(E[:, :, 1:, :] == 0)


# ---------------------------------------------------------------------------
# bounces and adjoint (operator level: seeded F, E, rho, grad_B)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,k,Lt,K,nb", [(700, 40, 1, 16, 8), (513, 17, 3, 9, 5), (300, 64, 1, 1, 3),
                                         (400, 20, 1, 16, 12),   # more bounces than the fast SDDMM holds
                                         (257, 0, 2, 4, 2), (1000, 30, 2, 16, 0), (129, 5, 1, 9, 1)])
def test_bounce_and_adjoint_match_oracle(g, orc, n, k, Lt, K, nb):
    rp, c, v = scenes.seeded_csr(n, k, seed=n + k)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(n, n))
    rho = scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9)
    E = scenes.seeded_array((n, Lt, K, 3), seed=2)
    gB = scenes.seeded_array((n, Lt, K, 3), seed=3, lo=-1, hi=1)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    B, tape = g.transport_solve(ff, dev(rho), dev(E), nb)
    Bo, tp = orc.bounce(F, rho, E, nb, keep_tape=True)
    assert rel_err(B.cpu().numpy(), Bo) < TOL
    gE, gr, gF = g.transport_backward(ff, tape, dev(rho), dev(gB))
    gEo, gro, gFo = orc.adjoint(F, rho, tp, gB)
    assert rel_err(gE.cpu().numpy(), gEo) < TOL
    if nb > 0:
        assert rel_err(gr.cpu().numpy(), gro) < TOL
        if F.nnz:
            assert rel_err(gF.cpu().numpy(), gFo) < TOL
    else:
        assert np.all(gr.cpu().numpy() == 0)


def test_ray_cast_operator_rows_in_morton_order(g, orc):
    """A ray-cast F hands its rows to the sparse kernels in the receivers'
    Morton order; the same F imported as a plain CSR (rows in index order)
    gives the same bits, and both match the FP64 oracle."""
    sc = _scene("fruit_bowl", n=3000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, 32, sc.seed, t_min=1e-4, topk=64)
    rp, col, val = ff.csr()
    plain = g.ff_from_csr(rp.clone(), col.clone(), val.clone())
    n, K, nb = sc.n, 9, 5
    rho = scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9)
    E = scenes.seeded_array((n, 2, K, 3), seed=2)
    gB = scenes.seeded_array((n, 2, K, 3), seed=3, lo=-1, hi=1)
    out = []
    for f in (ff, plain):
        B, tape = g.transport_solve(f, dev(rho), dev(E), nb)
        out.append((B,) + tuple(g.transport_backward(f, tape, dev(rho), dev(gB))))
    for a, b in zip(*out):
        assert torch.equal(a, b)
    F = sp.csr_matrix((val.cpu().numpy().astype(np.float64), col.cpu().numpy(), rp.cpu().numpy()), shape=(n, n))
    Bo, tp = orc.bounce(F, rho, E, nb, keep_tape=True)
    gEo, gro, gFo = orc.adjoint(F, rho, tp, gB)
    assert rel_err(out[0][0].cpu().numpy(), Bo) < TOL
    assert rel_err(out[0][1].cpu().numpy(), gEo) < TOL
    assert rel_err(out[0][2].cpu().numpy(), gro) < TOL
    assert rel_err(out[0][3].cpu().numpy(), gFo) < TOL


def test_solve_without_tape_and_determinism(g):
    n = 2000
    rp, c, v = scenes.seeded_csr(n, 50, seed=5)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    rho = dev(scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9))
    E = dev(scenes.seeded_array((n, 2, 9, 3), seed=2))
    B1, _ = g.transport_solve(ff, rho, E, 6, keep_tape=False)
    B2, _ = g.transport_solve(ff, rho, E, 6)
    assert torch.equal(B1, B2)


def test_tape_is_refused_after_the_operator_is_refilled(g):
    """A tape records the fill of F it was made on: after the handle is
    refilled (same size), the backward refuses it; a new solve gives a
    usable tape again."""
    n = 600
    rp, c, v = scenes.seeded_csr(n, 30, seed=5)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    rho = dev(scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9))
    E = dev(scenes.seeded_array((n, 1, 4, 3), seed=2))
    gB = dev(scenes.seeded_array((n, 1, 4, 3), seed=3, lo=-1, hi=1))
    _, tape = g.transport_solve(ff, rho, E, 3)
    rp2, c2, v2 = scenes.seeded_csr(n, 30, seed=6)
    g.ff_from_csr(dev(rp2), dev(c2), dev(v2), ff=ff)
    with pytest.raises(g.GsradError):
        g.transport_backward(ff, tape, rho, gB)
    _, tape = g.transport_solve(ff, rho, E, 3, tape=tape)
    gE, _, _ = g.transport_backward(ff, tape, rho, gB)
    assert torch.isfinite(gE).all()


def test_check_residual_and_nan(g):
    n = 800
    rp, c, v = scenes.seeded_csr(n, 30, seed=8, row_sum=0.5)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    rho = dev(scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9))
    E = dev(scenes.seeded_array((n, 1, 4, 3), seed=2))
    B, _ = g.transport_solve(ff, rho, E, 60, keep_tape=False)
    res = g.check(ff, rho, E, B)
    assert res["residual"] < 1e-6 and not res["non_finite"]
    assert abs(res["max_row_sum"] - np.max(np.add.reduceat(v.astype(np.float64), rp[:-1])[np.diff(rp) > 0])) < 1e-6
    E2 = E.clone()
    E2[3, 0, 0, 1] = float("nan")
    assert g.check(ff, rho, E2, B)["non_finite"]


# ---------------------------------------------------------------------------
# opacity gradient
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,kw,R,topk", [("fruit_bowl", dict(n=2500), 16, 0), ("fruit_bowl", dict(n=2500), 16, 24),
                                            ("box_room", dict(n=1500), 16, 0)])
def test_opacity_backward_matches_oracle(g, orc, name, kw, R, topk):
    sc = _scene(name, **kw)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, R, sc.seed, t_min=1e-4, topk=topk)
    Fg = gpu_csr(ff)
    rng = np.random.default_rng(3)
    gF = rng.standard_normal(Fg.nnz).astype(np.float32)
    grho = rng.standard_normal((sc.n, 3)).astype(np.float32)
    go, ga = g.opacity_backward(bvh, ff, dev(gF), dev(grho), dev(sc.albedo))
    te = orc.default_t_eps(sc.surfels)
    # the oracle gets the same dL/dF on its own F's pattern (entries present
    # in both); the tiny cut-boundary entries carry no gradient
    Fo, _ = orc.ff_matrix(sc.surfels, R, sc.seed, te, 1e-4, topk)
    W = sp.csr_matrix((gF.astype(np.float64), Fg.indices, Fg.indptr), shape=Fg.shape)
    Wo = W.multiply(Fo != 0).tocsr()
    Wo.sort_indices()
    goo, gao = orc.opacity_backward(sc.surfels, sc.albedo, R, sc.seed, te, 1e-4,
                                    (Wo.indptr, Wo.indices, Wo.data), grad_rho=grho)
    assert rel_err(go.cpu().numpy(), goo) < TOL
    assert rel_err(ga.cpu().numpy(), gao) < TOL


def test_autograd_function_chain(g, orc):
    sc = _scene("fruit_bowl", n=2000)
    R, nb = 16, 4
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, R, sc.seed, t_min=1e-4)
    K = 4
    E = dev(scenes.seeded_array((sc.n, 1, K, 3), seed=4)).requires_grad_(True)
    op = dev(sc.surfels["opacity"]).requires_grad_(True)
    alb = dev(sc.albedo).requires_grad_(True)
    B = g.RadiosityFn.apply(op, alb, E, bvh, ff, nb)
    target = dev(scenes.seeded_array((sc.n, 1, K, 3), seed=5))
    loss = ((B - target) ** 2).mean()
    loss.backward()
    # oracle chain on the GPU's F pattern values from the oracle itself
    te = orc.default_t_eps(sc.surfels)
    Fo, _ = orc.ff_matrix(sc.surfels, R, sc.seed, te, 1e-4, 0)
    rho = orc.rho(sc.surfels["opacity"], sc.albedo)
    Eo = E.detach().cpu().numpy().astype(np.float64)
    Bo, tp = orc.bounce(Fo, rho, Eo, nb, keep_tape=True)
    gB = 2 * (Bo - target.cpu().numpy()) / Bo.size
    gEo, gro, gFo = orc.adjoint(Fo, rho, tp, gB)
    goo, gao = orc.opacity_backward(sc.surfels, sc.albedo, R, sc.seed, te, 1e-4,
                                    (Fo.indptr, Fo.indices, gFo), grad_rho=gro)
    assert rel_err(B.detach().cpu().numpy(), Bo) < TOL
    assert rel_err(E.grad.cpu().numpy(), gEo) < TOL
    assert rel_err(alb.grad.cpu().numpy(), gao) < TOL
    assert rel_err(op.grad.cpu().numpy(), goo) < TOL


def test_opacity_backward_is_bit_identical_between_runs(g):
    """The per-sender sums are 64-bit fixed point (integer adds commute), so
    the gradient does not depend on the order of the atomics."""
    sc = _scene("fruit_bowl", n=3000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    for records in (True, False):
        ff = g.form_factors(bvh, 32, sc.seed, t_min=1e-4, records=records)
        nnz = ff.info()[1]
        gF = dev(np.random.default_rng(4).standard_normal(nnz).astype(np.float32))
        runs = [g.opacity_backward(bvh, ff, gF, None, None)[0] for _ in range(3)]
        assert torch.isfinite(runs[0]).all()
        assert runs[0].abs().max() > 0
        for r in runs[1:]:
            assert torch.equal(r, runs[0])


@pytest.mark.parametrize("R", [1, 100, 1500])
def test_recorded_hits_equal_the_walk_for_ragged_ray_pools(g, R):
    """The form-factor trace hands rays out to lanes from pools of up to 1024
    (R = 1: one ray of each of 1024 receivers; R = 100: pools of 1000;
    R = 1500: a full pool and a ragged one per receiver).  The opacity
    gradient from its records equals, bit for bit, the one recomputed by the
    plain per-ray walk, so every ray's recorded hits are the walk's."""
    sc = _scene("fruit_bowl", n=1500)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    out = []
    for records in (True, False):
        ff = g.form_factors(bvh, R, sc.seed, t_min=1e-4, records=records)
        nnz = ff.info()[1]
        gF = dev(np.random.default_rng(7).standard_normal(nnz).astype(np.float32))
        out.append((gpu_csr(ff), g.opacity_backward(bvh, ff, gF, None, None)[0]))
    (Fa, ga), (Fb, gb) = out
    assert np.array_equal(Fa.indptr, Fb.indptr) and np.array_equal(Fa.indices, Fb.indices)
    assert np.array_equal(Fa.data.view(np.uint32), Fb.data.view(np.uint32))
    assert ga.abs().max() > 0
    assert torch.equal(ga, gb)


def test_opacity_backward_scale_follows_the_gradient_size(g, orc):
    """The fixed-point scale is derived from max |dL/dF|: a dL/dF scaled by
    2^-60 or 2^40 gives the gradient scaled exactly the same way."""
    sc = _scene("fruit_bowl", n=2000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, 16, sc.seed, t_min=1e-4)
    nnz = ff.info()[1]
    gF = np.random.default_rng(5).standard_normal(nnz).astype(np.float32)
    base = g.opacity_backward(bvh, ff, dev(gF), None, None)[0].cpu().numpy()
    for e in (-60, 40):
        s = np.float32(2.0 ** e)
        go = g.opacity_backward(bvh, ff, dev(gF * s), None, None)[0].cpu().numpy()
        assert rel_err(go / s, base) < 1e-6
    zero = g.opacity_backward(bvh, ff, dev(np.zeros(nnz, np.float32)), None, None)[0]
    assert not zero.any()
    bad = gF.copy()
    bad[7] = np.inf
    assert torch.isnan(g.opacity_backward(bvh, ff, dev(bad), None, None)[0]).all()


# ---------------------------------------------------------------------------
# handle state after failures and rebuilds
# ---------------------------------------------------------------------------
def test_failed_refill_leaves_the_handle_unusable(g):
    """A reused F handle whose ray cast fails (more than 8192 distinct
    senders in one row) refuses later use with ESTATE instead of exposing
    half-written buffers; a successful cast makes it usable again."""
    ok_sc = _scene("fruit_bowl", n=1500)
    ok_bvh = g.build_bvh(dev_surfels(ok_sc.surfels))
    ff = g.form_factors(ok_bvh, 16, ok_sc.seed)
    rho = dev(np.full((ok_sc.n, 3), 0.5, np.float32))
    E = dev(scenes.seeded_array((ok_sc.n, 1, 1, 3), seed=2))
    g.transport_solve(ff, rho, E, 2)
    # 20k nearly transparent surfels in a cube, no compositing cut: each
    # receiver's 1024 rays composite ~250 surfels each, and central
    # receivers see over 8192 distinct front-facing senders
    sur = scenes.random_frame_surfels(20000, seed=9, extent=1.0, scale=(0.05, 0.06), opacity=(0.04, 0.05))
    bvh = g.build_bvh(dev_surfels(sur))
    with pytest.raises(g.GsradError) as ei:
        g.form_factors(bvh, 1024, 3, t_min=0.0, records=False, ff=ff)
    assert ei.value.status == g.gsrad.EOVERFLOW
    with pytest.raises(g.GsradError) as ei:
        g.transport_solve(ff, rho, E, 2)
    assert ei.value.status == g.gsrad.ESTATE
    with pytest.raises(g.GsradError) as ei:
        g.opacity_backward(ok_bvh, ff, dev(np.zeros(4, np.float32)), None, None)
    assert ei.value.status == g.gsrad.ESTATE
    g.form_factors(ok_bvh, 16, ok_sc.seed, ff=ff)
    B = g.transport_solve(ff, rho, E, 2)[0]
    assert torch.isfinite(B).all()


def test_opacity_backward_refuses_an_f_from_before_a_rebuild(g):
    """Rebuilding a BVH handle in place (same size, new opacity) makes the F
    cast from it before the rebuild unusable for the opacity backward."""
    sc = _scene("fruit_bowl", n=1500)
    d = dev_surfels(sc.surfels)
    bvh = g.build_bvh(d)
    ff = g.form_factors(bvh, 16, sc.seed)
    gF = dev(np.ones(ff.info()[1], np.float32))
    g.opacity_backward(bvh, ff, gF, None, None)
    d["opacity"] = d["opacity"] * 0.5
    g.build_bvh(d, bvh=bvh)
    with pytest.raises(g.GsradError) as ei:
        g.opacity_backward(bvh, ff, gF, None, None)
    assert ei.value.status == g.gsrad.EINVAL
    ff = g.form_factors(bvh, 16, sc.seed, ff=ff)
    go = g.opacity_backward(bvh, ff, dev(np.ones(ff.info()[1], np.float32)), None, None)[0]
    assert torch.isfinite(go).all()


# ---------------------------------------------------------------------------
# errors
# ---------------------------------------------------------------------------
def test_errors_surface_as_status(g):
    sc = _scene("furnace")
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    with pytest.raises(g.GsradError) as ei:
        g.form_factors(bvh, 0, 1)
    assert ei.value.status == g.gsrad.EINVAL
    ff = g.form_factors(bvh, 16, 1)
    E = dev(scenes.seeded_array((sc.n, 1, 3, 3), seed=2))
    with pytest.raises(g.GsradError):
        g.transport_solve(ff, dev(sc.albedo), E, 2)   # K = 3 is not a valid SH size


# ---------------------------------------------------------------------------
# dense stacks: rays with hundreds of composited hits (slab growth, record
# overflow and the traversal fallback of the backward)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("records", [True, False])
def test_layer_stack_forward_and_opacity_backward(g, orc, records):
    sur = scenes.layer_stack()
    n = sur["px"].shape[0]
    R, seed = 24, 5
    bvh = g.build_bvh(dev_surfels(sur))
    ff = g.form_factors(bvh, R, seed, t_min=1e-4, records=records)
    Fg = gpu_csr(ff)
    te = orc.default_t_eps(sur)
    Fo, _ = orc.ff_matrix(sur, R, seed, te, 1e-4, 0)
    assert rel_err(Fg.toarray(), Fo.toarray()) < TOL
    rng = np.random.default_rng(1)
    gF = rng.standard_normal(Fg.nnz).astype(np.float32)
    alb = np.full((n, 3), 0.5, np.float32)
    grho = rng.standard_normal((n, 3)).astype(np.float32)
    go, ga = g.opacity_backward(bvh, ff, dev(gF), dev(grho), dev(alb))
    W = sp.csr_matrix((gF.astype(np.float64), Fg.indices, Fg.indptr), shape=Fg.shape).multiply(Fo != 0).tocsr()
    W.sort_indices()
    goo, _ = orc.opacity_backward(sur, alb, R, seed, te, 1e-4, (W.indptr, W.indices, W.data), grad_rho=grho)
    assert rel_err(go.cpu().numpy(), goo) < TOL


# ---------------------------------------------------------------------------
# a tree deeper than the shallow traversal stack: the form-factor trace is
# run again with the deep stack and still matches the oracle
# ---------------------------------------------------------------------------
def test_deep_tree_retraces_with_deep_stack(g, orc):
    sur = scenes.deep_chain()
    n = sur["px"].shape[0]
    R, seed = 8, 3
    bvh = g.build_bvh(dev_surfels(sur))
    assert bvh.height() >= 34
    g.profile_enable(True)
    try:
        ff = g.form_factors(bvh, R, seed, t_min=1e-4)
        torch.cuda.synchronize()
        rep = g.profile_report()
    finally:
        g.profile_enable(False)
    assert rep["ff_trace"]["count"] >= 2, rep   # shallow attempt, then deep (and record growth)
    Fg = gpu_csr(ff)
    te = orc.default_t_eps(sur)
    Fo, _ = orc.ff_matrix(sur, R, seed, te, 1e-4, 0)
    assert rel_err(Fg.toarray(), Fo.toarray()) < TOL
    # the shadow rays and the backward traversal use the deep stack directly
    alb = np.full((n, 3), 0.5, np.float32)
    E = g.direct_light(bvh, dev(alb), dev(np.array([[2.0, 2.0, 2.0]], np.float32)),
                       dev(np.array([3.0], np.float32)), 1)
    Eo = orc.direct_light(sur, alb, np.array([[2.0, 2.0, 2.0]]), np.array([3.0]), 1, te)
    assert rel_err(E.cpu().numpy(), Eo) < TOL


# ---------------------------------------------------------------------------
# FP64 reciprocity check of the estimated operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,kw,R", [("furnace", {}, 64), ("box_room", dict(n=1500), 32)])
def test_reciprocity_check_matches_oracle(g, orc, name, kw, R):
    sc = _scene(name, **kw)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, R, sc.seed, t_min=1e-4)
    rec = g.check_reciprocity(bvh, ff)
    te = orc.default_t_eps(sc.surfels)
    Fo, _ = orc.ff_matrix(sc.surfels, R, sc.seed, te, 1e-4, 0)
    A = orc.effective_area(sc.surfels["su"], sc.surfels["sv"], sc.surfels["opacity"])
    asym, mx = orc.reciprocity(Fo, A)
    assert abs(rec["asymmetry"] - asym) <= 1e-4 * asym
    assert abs(rec["max_entry"] - mx) <= 1e-4 * max(mx, 1e-12)


def test_chunked_ray_cast_equals_one_pass(g):
    """Without kept records the receivers are traced in chunks whose record
    slabs fit a fixed budget (10k receivers x 1024 rays: more than one
    chunk), each chunk's rays pooled and taken by the persistent workgroups
    anew; the form factors must be those of the single pass with records,
    bit for bit (the same rays, fixed-point sums)."""
    sc = _scene("fruit_bowl", n=10000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    one = g.form_factors(bvh, 1024, sc.seed, t_min=1e-4, topk=256)
    chunked = g.form_factors(bvh, 1024, sc.seed, t_min=1e-4, topk=256, records=False)
    for x, y in zip(one.csr(), chunked.csr()):
        assert torch.equal(x, y)
    assert one.info()[1] > 0
