"""GPU parity of the one-sided Jacobi SVD (Algorithm 2, Sec. 4.2 relative score) with the
oracle, through the C ABI.

Without preconditioning both sides perform the same IEEE operations in the same order (the
Gram entries are dot products summed in index order, one lane per entry), so the pivot
sequence, S, U and V must agree bit for bit.  With the FP32 preconditioner the two FP32
stages differ (parallel blocked vs. cyclic Jacobi), so the singular values are compared
to the accuracy both reach.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_23187_amd import inputs as I
from paper_2607_23187_amd import jacobi as J

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_svd(b, tol, pivot, precond="none", cap=0, **kw):
    print(f"svd m={b.shape[0]} n={b.shape[1]} pivot={pivot} precond={precond}", flush=True)
    r = J.svd(dev(b), tol=tol, pivot=pivot, precond=precond, pivot_log_cap=cap, **kw)
    torch.cuda.synchronize()
    return r


CASES = [(40, 25, 1), (33, 33, 2), (70, 9, 3), (130, 100, 4), (64, 64, 5), (300, 260, 6)]


SCORES = [("gap", O.GAP, U), ("relative", O.RELATIVE, U), ("greedy", O.GREEDY, 1e-11)]
# greedy runs at the shapes up to n = 100 (its rotation count grows fastest with n)
PARITY = [(*sc, *case) for case in CASES for sc in SCORES
          if not (case[1] > 200 and sc[0] == "greedy")]


@pytest.mark.parametrize("pivot,piv_o,tol,m,n,seed", PARITY)
def test_svd_bitwise_parity(pivot, piv_o, tol, m, n, seed):
    b = I.svd_graded(m, n, seed=seed, decades=8.0)
    cap = 40 * n * n + 64
    g = gpu_svd(b, tol, pivot, cap=cap)
    thr = g.stats["thr"]
    o = O.svd(b, tol, pivot=piv_o, abs_thr=thr, logcap=cap)
    assert abs(thr - O.svd_threshold(piv_o, tol, n, o.normF)) <= 1e-13 * thr
    assert g.status == o.status == O.OK
    assert g.stats["rotations"] == o.rotations > 0
    assert g.stats["rescans"] == o.rescans
    assert np.array_equal(g.pivots.cpu().numpy(), o.pivots)
    assert np.array_equal(g.s.cpu().numpy(), o.s)
    assert np.array_equal(g.u.cpu().numpy(), o.u)
    assert np.array_equal(g.v.cpu().numpy(), o.v)


def test_svd_hilbert_c100_matches_oracle_run():
    # the Sec. 4.2 experiment: fl64(C_100), relative score, no preconditioning
    with open(os.path.join(GOLDEN, "hilbert_cholesky_sv.json")) as f:
        gold = json.load(f)
    ref = np.array([float(x) for x in gold["sv"]["100"]])
    c = I.hilbert_cholesky(100)
    g = gpu_svd(c, U, "relative", cap=400000, max_rotations=400000)
    want = gold["c100_relative"]
    assert g.status == want["status"] == O.OK
    assert g.stats["rotations"] == want["rotations"]
    assert hashlib.sha256(g.pivots.cpu().numpy().astype(np.int32).tobytes()
                          ).hexdigest() == want["pivots_sha256"]
    s = g.s.cpu().numpy()
    assert hashlib.sha256(np.ascontiguousarray(s).tobytes()).hexdigest() == want["sv_sha256"]
    assert np.max(np.abs(s[:10] - ref[:10]) / ref[:10]) <= 1e-13


@pytest.mark.parametrize("m,n,seed", [(80, 60, 21), (256, 200, 22)])
def test_svd_preconditioned(m, n, seed):
    b = I.svd_graded(m, n, seed=seed, decades=4.0)
    g = gpu_svd(b, U, "gap", precond="fp32")
    o = O.svd(b, U, pivot=O.GAP, precond="fp32")
    plain = O.svd(b, U, pivot=O.GAP)
    assert g.status == O.OK
    s = g.s.cpu().numpy()
    ls = np.linalg.svd(b, compute_uv=False)
    assert np.max(np.abs(s - o.s)) <= 100 * m * U * ls[0]
    assert np.max(np.abs(s - ls)) <= 100 * m * U * ls[0]
    assert g.stats["rotations"] < plain.rotations / 3
    u, v = g.u.cpu().numpy(), g.v.cpu().numpy()
    assert np.linalg.norm(b @ v - u * s[None, :]) <= 30 * n * U * np.linalg.norm(b)
    assert np.linalg.norm(v.T @ v - np.eye(n)) <= 100 * n * U


def test_svd_edge_cases():
    b = np.arange(1.0, 6.0)[:, None]
    g = gpu_svd(b, U, "gap")
    assert g.status == O.OK and g.stats["rotations"] == 0
    assert g.s.cpu().numpy()[0] == np.sqrt(np.sum(b * b))
    assert g.v.cpu().numpy().tolist() == [[1.0]]
    z = I.svd_graded(10, 4, seed=1)
    z[:, 2] = 0.0
    g = gpu_svd(z, U, "relative")
    o = O.svd(z, U, pivot=O.RELATIVE, abs_thr=g.stats["thr"])
    assert np.array_equal(g.s.cpu().numpy(), o.s) and g.s.cpu().numpy()[-1] == 0.0
    assert np.array_equal(g.u.cpu().numpy(), o.u)
    nan = z.copy()
    nan[3, 1] = np.nan
    r = J.svd(dev(nan), pivot="gap", check=False)
    assert r.status == J.ERR_NONFINITE
    r = J.svd(dev(np.ones((3, 5))), check=False)   # m < n
    assert r.status == -2
    cap = 3
    b = I.svd_graded(20, 12, seed=9)
    g = gpu_svd(b, U, "gap", cap=cap, max_rotations=7)
    assert g.status == J.WARN_MAXROT and g.stats["rotations"] == 7
    o = O.svd(b, U, pivot=O.GAP, abs_thr=g.stats["thr"], maxrot=7)
    assert np.array_equal(g.pivots.cpu().numpy(), o.pivots[:cap])
    assert np.array_equal(g.s.cpu().numpy(), o.s)
