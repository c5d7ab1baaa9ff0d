"""Shared helpers of the GPU tests: move scenes to the device, densify CSR,
and the relative max-norm error used for every parity claim."""
import numpy as np
import scipy.sparse as sp
import torch

import scenes


def dev_surfels(sur):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in sur.items()}


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_err(x, ref):
    """max |x - ref| / max |ref| (0 if both are zero)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(x - ref)) if ref.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


def gpu_csr(ff):
    rp, col, val = ff.csr()
    n = rp.shape[0] - 1
    return sp.csr_matrix((val.cpu().numpy().astype(np.float64), col.cpu().numpy(), rp.cpu().numpy()), shape=(n, n))


def seeded_operator(n, k, seed, row_sum=0.6):
    rp, c, v = scenes.seeded_csr(n, k, seed, row_sum=row_sum)
    return rp, c, v
