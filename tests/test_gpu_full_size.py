"""The benchmark workloads at full size, checked against the FP64 oracle on
outputs it can compute at that size.  The 100k-surfel fruit bowl in the
launch configuration the benchmark times (128 rays per surfel, top-512
rows, SH degree 3, 8 bounces):

* form-factor rows and direct-light rows of sampled receivers (the oracle
  casts only those receivers' rays, by brute force over all surfels);
* bounces and adjoint on a seeded 100k operator with 512 entries per row,
  with E and grad_B non-zero on two SH coefficients only.  The transport is
  separable over coefficient columns (rho acts per colour, F is shared), so
  B and lambda vanish on every other column and the oracle's FP64 run on
  the two non-zero coefficients gives the exact B, grad_E, grad_rho and
  grad_F of the full 48-column launch.

The 32,768-surfel multi-light room (all-entry F rows past the first
aggregation table; the dense BF16 launch over 2700 columns on two lights),
and the 64-scene uneven batch (bit-identical to the scene-by-scene path,
the smallest scenes against the oracle).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests.gpu_common import dev, dev_surfels, rel_err  # noqa: E402

TOL = 1e-4
N = 100_000


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_18497_amd as g
    g.gsrad.lib()
    return g


@pytest.fixture(scope="module")
def bowl(g):
    sc = scenes.make_config("fruit_bowl", n=N)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, sc.R, sc.seed, t_min=sc.t_min, topk=sc.topk)
    return sc, bvh, ff


def test_full_size_form_factor_rows(g, orc, bowl):
    sc, bvh, ff = bowl
    rp, col, val = (x.cpu().numpy() for x in ff.csr())
    assert rp.shape[0] == N + 1 and np.all(np.diff(rp) <= sc.topk)
    recv = np.sort(np.random.default_rng(17).choice(N, size=12, replace=False)).astype(np.int64)
    te = orc.default_t_eps(sc.surfels)
    rpo, co, vo, _ = orc.ff_rows(sc.surfels, recv, sc.R, sc.seed, te, sc.t_min, sc.topk)
    num = den = 0.0
    swaps = 0
    for k, i in enumerate(recv):
        a = dict(zip(col[rp[i]:rp[i + 1]].tolist(), val[rp[i]:rp[i + 1]].tolist()))
        b = dict(zip(co[rpo[k]:rpo[k + 1]].tolist(), vo[rpo[k]:rpo[k + 1]].tolist()))
        assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)
        full = len(a) == sc.topk and len(b) == sc.topk
        tha = min(a.values()) if a else 0.0
        thb = min(b.values()) if b else 0.0
        for j in set(a) | set(b):
            # kept on one side only: valid only as a swap at the top-k threshold
            if full and j not in b and a[j] <= thb * (1 + 1e-5):
                swaps += 1
                continue
            if full and j not in a and b[j] <= tha * (1 + 1e-5):
                swaps += 1
                continue
            num = max(num, abs(a.get(j, 0.0) - b.get(j, 0.0)))
        den = max(den, max(b.values()) if b else 0.0)
        assert sum(a.values()) <= 1.0 + 1e-6
    assert num / den < 1e-5, (num / den, swaps)
    assert swaps <= 2 * len(recv)


def test_full_size_direct_light_rows(g, orc, bowl):
    sc, bvh, _ = bowl
    E = g.direct_light(bvh, dev(sc.albedo), dev(sc.light_pos), dev(sc.light_I), sc.K).cpu().numpy()
    recv = np.sort(np.random.default_rng(18).choice(N, size=256, replace=False)).astype(np.int64)
    Eo = orc.direct_light(sc.surfels, sc.albedo, sc.light_pos, sc.light_I, sc.K, receivers=recv)
    assert rel_err(E[recv], Eo) < TOL
    # Lambertian emission: only the DC coefficient is non-zero
    assert np.all(E[:, :, 1:, :] == 0)


def test_full_size_opacity_gradient_on_sampled_rows(g, orc, bowl):
    """dL/dopacity through the compositing (decay term of Eq. dl-dgeo-0) in
    the benchmark's launch, with dL/dF non-zero on 64 sampled receiver rows
    only: every sender that those receivers' rays composite gets a
    contribution, and the oracle's brute-force compositing backward over the
    same 64 receivers gives the exact gradient of every surfel."""
    sc, bvh, ff = bowl
    rp, col, _ = (x.cpu().numpy() for x in ff.csr())
    nnz = rp[-1]
    recv = np.sort(np.random.default_rng(19).choice(N, size=64, replace=False)).astype(np.int64)
    rng = np.random.default_rng(20)
    gF = np.zeros(nnz, np.float32)
    gp = [0]
    gc, gv = [], []
    for i in recv:
        v = rng.standard_normal(rp[i + 1] - rp[i]).astype(np.float32)
        gF[rp[i]:rp[i + 1]] = v
        gc.append(col[rp[i]:rp[i + 1]])
        gv.append(v.astype(np.float64))
        gp.append(gp[-1] + v.shape[0])
    go = g.opacity_backward(bvh, ff, dev(gF), None, None)[0].cpu().numpy()
    te = orc.default_t_eps(sc.surfels)
    goo, _ = orc.opacity_backward(sc.surfels, sc.albedo, sc.R, sc.seed, te, sc.t_min,
                                  (np.asarray(gp, np.int64), np.concatenate(gc), np.concatenate(gv)),
                                  receivers=recv)
    assert np.count_nonzero(goo) > 1000
    assert rel_err(go, goo) < TOL
    go2 = g.opacity_backward(bvh, ff, dev(gF), None, None)[0].cpu().numpy()
    assert np.array_equal(go, go2)


def test_records_kept_beyond_the_former_fixed_budget(g):
    """A 200k-surfel fruit bowl at R = 128 needs a 52 GB record slab: it is
    kept (the geometry backward, which needs the records, runs), and the
    opacity gradient from the records equals, bit for bit, the one that
    recomputes every ray by traversal (a cast without records)."""
    sc = scenes.make_config("fruit_bowl", n=200_000)
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, sc.R, sc.seed, t_min=sc.t_min, topk=sc.topk)
    rp, col, _ = (x.cpu().numpy() for x in ff.csr())
    gF = np.zeros(rp[-1], np.float32)
    rng = np.random.default_rng(3)
    for i in rng.choice(sc.n, size=64, replace=False):
        gF[rp[i]:rp[i + 1]] = rng.standard_normal(rp[i + 1] - rp[i]).astype(np.float32)
    geo = g.geometry_backward(bvh, ff, dev(gF))
    assert torch.isfinite(geo["px"]).all()
    go = g.opacity_backward(bvh, ff, dev(gF), None, None)[0]
    del ff
    ff2 = g.form_factors(bvh, sc.R, sc.seed, t_min=sc.t_min, topk=sc.topk, records=False)
    go2 = g.opacity_backward(bvh, ff2, dev(gF), None, None)[0]
    assert torch.equal(go, go2)
    assert int((go != 0).sum()) > 1000


def test_full_size_transport_on_two_coefficients(g, orc):
    K, Lt, nb, topk = 16, 1, 8, 512
    slots = [0, 15]
    rp, c, v = scenes.seeded_csr(N, topk, seed=31)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(N, N))
    rho = scenes.seeded_array((N, 3), seed=1, lo=0.1, hi=0.9)
    Es = scenes.seeded_array((N, Lt, len(slots), 3), seed=2)
    gBs = scenes.seeded_array((N, Lt, len(slots), 3), seed=3, lo=-1, hi=1)
    E = np.zeros((N, Lt, K, 3), np.float32)
    gB = np.zeros((N, Lt, K, 3), np.float32)
    E[:, :, slots, :] = Es
    gB[:, :, slots, :] = gBs
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    B, tape = g.transport_solve(ff, dev(rho), dev(E), nb)
    gE, gr, gF = g.transport_backward(ff, tape, dev(rho), dev(gB))
    B, gE, gr, gF = (x.cpu().numpy() for x in (B, gE, gr, gF))
    Bo, tp = orc.bounce(F, rho, Es, nb, keep_tape=True)
    gEo, gro, gFo = orc.adjoint(F, rho, tp, gBs)
    others = [k for k in range(K) if k not in slots]
    assert np.all(B[:, :, others, :] == 0) and np.all(gE[:, :, others, :] == 0)
    assert rel_err(B[:, :, slots, :], Bo) < TOL
    assert rel_err(gE[:, :, slots, :], gEo) < TOL
    assert rel_err(gr, gro) < TOL
    assert rel_err(gF, gFo) < TOL


def test_all_entry_rows_past_the_first_table(g, orc):
    """The 32,768-surfel box room with 256 rays and every entry kept: many
    receivers see more distinct senders than the first 4096-entry
    aggregation table holds, so their rows are aggregated again with the
    8192 table.  The longest rows and a random sample against the oracle, and a
    second cast on the same handle (which may start from the larger table)
    bit for bit equal to the first."""
    sc = scenes.make_config("multi_light")
    n = sc.n
    bvh = g.build_bvh(dev_surfels(sc.surfels))
    ff = g.form_factors(bvh, sc.R, sc.seed, t_min=sc.t_min, topk=0, records=False)
    rp, col, val = (x.cpu().numpy() for x in ff.csr())
    lens = np.diff(rp)
    assert lens.max() > 4096          # rows that only the second table can hold
    longest = np.argsort(lens)[-4:]
    rnd = np.random.default_rng(23).choice(n, size=4, replace=False)
    recv = np.unique(np.concatenate([longest, rnd])).astype(np.int64)
    te = orc.default_t_eps(sc.surfels)
    rpo, co, vo, _ = orc.ff_rows(sc.surfels, recv, sc.R, sc.seed, te, sc.t_min, 0, cap_row=8192)
    for k, i in enumerate(recv):
        assert np.array_equal(col[rp[i]:rp[i + 1]], co[rpo[k]:rpo[k + 1]]), i
        b = vo[rpo[k]:rpo[k + 1]]
        assert np.max(np.abs(val[rp[i]:rp[i + 1]] - b)) / np.max(b) < 1e-5, i
    ff2 = g.form_factors(bvh, sc.R, sc.seed, t_min=sc.t_min, topk=0, records=False, ff=ff)
    rp2, col2, val2 = (x.cpu().numpy() for x in ff2.csr())
    assert np.array_equal(rp2, rp) and np.array_equal(col2, col) and np.array_equal(val2, val)


def _slice_rel(x, ref):
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def test_full_size_dense_multi_light_on_two_lights(g, orc):
    """The dense BF16 launch of the multi-light workload (32,768 rows,
    100 lights x 9 SH x 3 = 2700 columns, 8 bounces) on a seeded operator
    with ~190 entries per row, E and grad_B non-zero for lights 0 and 57
    only.  The transport is separable over columns, so the oracle's FP64 run
    on those two lights gives B, dL/dE, dL/drho and dL/dF of the whole
    launch; the other lights' outputs must be exactly zero."""
    N, k, Lt, K, nb, lights = 32768, 190, 100, 9, 8, [0, 57]
    rp, c, v = scenes.seeded_csr(N, k, seed=41)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(N, N))
    rho = scenes.seeded_array((N, 3), seed=1, lo=0.1, hi=0.9)
    Es = scenes.seeded_array((N, len(lights), K, 3), seed=2)
    gBs = scenes.seeded_array((N, len(lights), K, 3), seed=3, lo=-1, hi=1)
    E = np.zeros((N, Lt, K, 3), np.float32)
    gB = np.zeros((N, Lt, K, 3), np.float32)
    E[:, lights] = Es
    gB[:, lights] = gBs
    ff = g.ff_dense(g.ff_from_csr(dev(rp), dev(c), dev(v)))
    B, tape = g.transport_solve(ff, dev(rho), dev(E), nb, precision=g.BF16)
    gE, gr, gF = g.transport_backward(ff, tape, dev(rho), dev(gB))
    B, gE, gr, gF = (x.cpu().numpy() for x in (B, gE, gr, gF))
    Bo, tp = orc.bounce(F, rho, Es, nb, keep_tape=True)
    gEo, gro, gFo = orc.adjoint(F, rho, tp, gBs)
    others = np.setdiff1d(np.arange(Lt), lights)
    assert not B[:, others].any() and not gE[:, others].any()
    assert _slice_rel(B[:, lights], Bo) < 1e-3
    assert _slice_rel(gE[:, lights], gEo) < 1e-3
    assert _slice_rel(gr, gro) < 1e-3
    assert _slice_rel(gF, gFo) < 1e-3


def test_full_size_uneven_batch(g, orc):
    """The uneven batch of the benchmark (64 cluster rooms, 2k-65k surfels,
    1-4 lights each, 1.19 M surfels, top-512 F, K = 9, 8 bounces): one batch
    solve and backward, bit for bit equal to the scene-by-scene path on
    every scene, and the two smallest scenes against the FP64 oracle on the
    ray-cast F."""
    rooms = scenes.uneven_batch(lights=(1, 4))
    K, R, nb = rooms[0].K, rooms[0].R, rooms[0].n_bounces
    ffs, Es, rhos, Lts = [], [], [], []
    for sc in rooms:
        bvh = g.build_bvh(dev_surfels(sc.surfels))
        ffs.append(g.form_factors(bvh, R, sc.seed, t_min=sc.t_min, topk=512, records=False))
        alb = dev(sc.albedo)
        Es.append(g.direct_light(bvh, alb, dev(sc.light_pos), dev(sc.light_I), K))
        rhos.append(g.reflectance(bvh, alb))
        Lts.append(sc.n_lights)
    assert sum(sc.n for sc in rooms) > 1_000_000
    batch = g.batch_create(ffs, Lts, K)
    rho = torch.cat(rhos)
    E = batch.pack(Es)
    gB = dev(scenes.seeded_array((E.shape[0],), seed=98, lo=-1, hi=1))
    Bb = batch.unpack(g.batch_transport_solve(batch, rho, E, nb))
    gEb, grb, gFb = g.batch_transport_backward(batch, rho, gB)
    gEb = batch.unpack(gEb)
    gBs = batch.unpack(gB)
    smallest = set(np.argsort([sc.n for sc in rooms])[:2].tolist())
    r0 = e0 = 0
    for s, (sc, ff) in enumerate(zip(rooms, ffs)):
        n = sc.n
        nnz = ff.info()[1]
        Bs, tape = g.transport_solve(ff, rhos[s], Es[s], nb)
        gEs, grs, gFs = g.transport_backward(ff, tape, rhos[s], gBs[s].contiguous())
        assert torch.equal(Bb[s], Bs), s
        assert torch.equal(gEb[s], gEs), s
        assert torch.equal(grb[r0:r0 + n], grs), s
        assert torch.equal(gFb[e0:e0 + nnz], gFs), s
        if s in smallest:
            rp, col, val = (x.cpu().numpy() for x in ff.csr())
            F = sp.csr_matrix((val.astype(np.float64), col, rp), shape=(n, n))
            rh = rhos[s].cpu().numpy()
            Bo, tp = orc.bounce(F, rh, Es[s].cpu().numpy(), nb, keep_tape=True)
            gEo, gro, gFo = orc.adjoint(F, rh, tp, gBs[s].cpu().numpy())
            assert rel_err(Bs.cpu().numpy(), Bo) < TOL
            assert rel_err(gEs.cpu().numpy(), gEo) < TOL
            assert rel_err(grs.cpu().numpy(), gro) < TOL
            assert rel_err(gFs.cpu().numpy(), gFo) < TOL
        r0 += n
        e0 += nnz
