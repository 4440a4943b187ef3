"""jacobi_eigh_noalloc (the entry point for callers that cannot allocate device memory)
against jacobi_eigh_ex through the C ABI: two calls in a row, the second smaller, each
giving the same bits, rotation count and status as the allocating call (both run the same
kernels; only the workspace and the rotation-log length differ, and a log drain changes no
result).  Sizes above JE_NOALLOC_MAX_N are refused before any device work."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2607_23187_amd import inputs as I
from paper_2607_23187_amd import jacobi as J

U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(n, seed, precond, pivot):
    p = I.clustered(n, seed=seed, size=8, offset=1e-10)
    a = torch.from_numpy(p.a).cuda()
    tol = 10 * n * U * float(np.max(np.abs(p.lam))) / float(np.linalg.norm(p.a))
    ref = J.eigh(a, tol=tol, pivot=pivot, precond=precond)
    got = J.eigh(a, tol=tol, pivot=pivot, precond=precond, noalloc=True)
    return ref, got


@pytest.mark.gpu
@pytest.mark.parametrize("precond", ["fp32", "none"])
def test_noalloc_equals_ex_twice(precond):
    # the second call is smaller; without the preconditioner the 400-row solve needs more
    # rotations than the fixed log holds, so its V is assembled over several drains
    for n, seed, pivot in ((J.NOALLOC_MAX_N if precond == "fp32" else 400, 9901, "gap"),
                           (100, 9902, "greedy")):
        say("noalloc", precond, n, pivot)
        ref, got = _pair(n, seed, precond, pivot)
        assert got.status == ref.status == J.OK
        assert got.stats["rotations"] == ref.stats["rotations"]
        assert torch.equal(got.w, ref.w)
        assert torch.equal(got.v, ref.v)


@pytest.mark.gpu
def test_noalloc_refuses_too_large():
    n = J.NOALLOC_MAX_N + 1
    a = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    L = J.load()
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    r = L.jacobi_eigh_noalloc(a.data_ptr(), n, n, w.data_ptr(), None, n, 1e-12, 1, 1, None,
                              None, None)
    assert r == J.ERR_TOO_LARGE
