"""Dense BF16 transport on the matrix cores (precision BF16) against the
FP64 oracle.

* Exactness of the matrix-core products: with F, E and rho dyadic numbers
  of few bits, every BF16 operand and FP32 sum is exact, so B (one and two
  bounces) must equal the oracle bit for bit; this pins the tile, fragment
  and accumulator layouts over several 256 x 256 tiles and ragged edges.
* Seeded operators: B, dL/dE, dL/drho, dL/dF at the stored entries and
  the dense dL/dF within 1e-3 relative max-norm (the BF16 bar).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests.gpu_common import dev, rel_err  # noqa: E402

TOL_BF16 = 1e-3


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_18497_amd as g
    g.gsrad.lib()
    return g


def _dyadic_operator(n, k, seed):
    """CSR with k entries per row at random columns, values m/64 with
    m in 1..7 (exact in BF16)."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        c = np.sort(rng.choice(n, size=min(k, n), replace=False))
        rows.append(np.full(c.shape[0], i))
        cols.append(c)
    r = np.concatenate(rows)
    c = np.concatenate(cols).astype(np.int32)
    v = (rng.integers(1, 8, size=r.shape[0]) / 64.0).astype(np.float32)
    F = sp.csr_matrix((v, c, np.concatenate([[0], np.cumsum([x.shape[0] for x in rows])]).astype(np.int64)),
                      shape=(n, n))
    return F


@pytest.mark.parametrize("n,k,Lt,K,nb", [(700, 12, 3, 9, 1), (700, 12, 3, 9, 2), (257, 5, 1, 16, 2),
                                         (513, 20, 2, 4, 1)])
def test_dense_products_are_exact_on_dyadic_inputs(g, orc, n, k, Lt, K, nb):
    F = _dyadic_operator(n, k, seed=n + k)
    rng = np.random.default_rng(3)
    E = (rng.integers(0, 16, size=(n, Lt, K, 3)) / 16.0).astype(np.float32)
    rho = (rng.integers(1, 4, size=(n, 3)) / 4.0).astype(np.float32)
    ff = g.ff_from_csr(dev(F.indptr.astype(np.int64)), dev(F.indices.astype(np.int32)), dev(F.data))
    g.ff_dense(ff)
    B, _ = g.transport_solve(ff, dev(rho), dev(E), nb, keep_tape=False, precision=g.BF16)
    Bo = orc.bounce(sp.csr_matrix(F, dtype=np.float64), rho, E, nb)
    assert np.array_equal(B.cpu().numpy(), Bo.astype(np.float32))


@pytest.mark.parametrize("n,kk,Lt,K,nb", [(1000, 40, 1, 9, 8), (300, 30, 10, 9, 3), (777, 25, 2, 16, 5),
                                          (256, 16, 1, 1, 1), (2600, 20, 1, 4, 2)])
def test_dense_bf16_matches_oracle(g, orc, n, kk, Lt, K, nb):
    rp, c, v = scenes.seeded_csr(n, kk, seed=n + kk)
    F = sp.csr_matrix((v.astype(np.float64), c, rp), shape=(n, n))
    rho = scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9)
    E = scenes.seeded_array((n, Lt, K, 3), seed=2)
    gB = scenes.seeded_array((n, Lt, K, 3), seed=3, lo=-1, hi=1)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    g.ff_dense(ff)
    B, tape = g.transport_solve(ff, dev(rho), dev(E), nb, precision=g.BF16)
    Bo, tp = orc.bounce(F, rho, E, nb, keep_tape=True)
    assert rel_err(B.cpu().numpy(), Bo) < TOL_BF16
    gE, gr, gF = g.transport_backward(ff, tape, dev(rho), dev(gB))
    gEo, gro, Go = orc.adjoint(F, rho, tp, gB, dense_grad_F=True)
    assert rel_err(gE.cpu().numpy(), gEo) < TOL_BF16
    assert rel_err(gr.cpu().numpy(), gro) < TOL_BF16
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert rel_err(gF.cpu().numpy(), Go[rows, c]) < TOL_BF16
    Gd = g.tape_grad_F_dense(tape, n).cpu().numpy()
    assert rel_err(Gd, Go) < TOL_BF16
    # the FP32 sparse path on the same operator agrees as well
    B32, _ = g.transport_solve(ff, dev(rho), dev(E), nb, keep_tape=False)
    assert rel_err(B.cpu().numpy(), B32.cpu().numpy()) < TOL_BF16


def test_dense_needs_copies_and_handles_zero_bounces(g):
    n = 300
    rp, c, v = scenes.seeded_csr(n, 10, seed=4)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    rho = dev(scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9))
    E = dev(scenes.seeded_array((n, 1, 4, 3), seed=2))
    with pytest.raises(g.GsradError):
        g.transport_solve(ff, rho, E, 2, precision=g.BF16)
    g.ff_dense(ff)
    B, tape = g.transport_solve(ff, rho, E, 0, precision=g.BF16)
    assert torch.equal(B, E)
    with pytest.raises(g.GsradError):
        g.tape_grad_F_dense(tape, n)
    # new values in F drop the dense copies
    g.ff_from_csr(dev(rp), dev(c), dev(v), ff=ff)
    with pytest.raises(g.GsradError):
        g.transport_solve(ff, rho, E, 2, precision=g.BF16)


def test_dense_is_deterministic(g):
    n = 600
    rp, c, v = scenes.seeded_csr(n, 30, seed=6)
    ff = g.ff_dense(g.ff_from_csr(dev(rp), dev(c), dev(v)))
    rho = dev(scenes.seeded_array((n, 3), seed=1, lo=0.1, hi=0.9))
    E = dev(scenes.seeded_array((n, 2, 9, 3), seed=2))
    B1, _ = g.transport_solve(ff, rho, E, 4, keep_tape=False, precision=g.BF16)
    B2, _ = g.transport_solve(ff, rho, E, 4, keep_tape=False, precision=g.BF16)
    assert torch.equal(B1, B2)
