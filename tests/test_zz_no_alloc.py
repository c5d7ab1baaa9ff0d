"""The allocation-free bounce entry point against gsrad_transport_solve:
two calls in a row on one GPU (the second with a smaller operator and a
different light count) give bit-identical B, and an operator larger than the
fixed scratch array is refused."""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests.gpu_common import dev  # noqa: E402


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_18497_amd as g
    g.gsrad.lib()
    return g


def _case(g, n, k, Lt, K, seed):
    rp, c, v = scenes.seeded_csr(n, k, seed=seed)
    ff = g.ff_from_csr(dev(rp), dev(c), dev(v))
    rho = dev(scenes.seeded_array((n, 3), seed=seed + 1, lo=0.1, hi=0.9))
    E = dev(scenes.seeded_array((n, Lt, K, 3), seed=seed + 2))
    return ff, rho, E


@pytest.mark.parametrize("nb", [0, 1, 2, 8])
def test_noalloc_solve_equals_transport_solve_on_two_calls(g, nb):
    for n, k, Lt, K, seed in [(20000, 64, 2, 9, 11), (3001, 17, 1, 4, 12)]:
        ff, rho, E = _case(g, n, k, Lt, K, seed)
        ref = g.transport_solve(ff, rho, E, nb, keep_tape=False)[0]
        out = torch.full_like(E, float("nan"))
        g.transport_solve_noalloc(ff, rho, E, nb, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, nb)


def test_noalloc_solve_refuses_operators_beyond_the_scratch(g):
    n, Lt, K = 200000, 1, 16          # 2 * 200000 * 48 * 4 bytes > 64 MiB
    ff, rho, E = _case(g, n, 4, Lt, K, 13)
    out = torch.empty_like(E)
    with pytest.raises(g.GsradError) as ei:
        g.transport_solve_noalloc(ff, rho, E, 4, out)
    assert ei.value.status == g.gsrad.EINVAL
    # one bounce needs no iterate of its own: allowed at any size
    g.transport_solve_noalloc(ff, rho, E, 1, out)
    ref = g.transport_solve(ff, rho, E, 1, keep_tape=False)[0]
    assert torch.equal(out, ref)
