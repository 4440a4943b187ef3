"""Batched solves (one launch sequence for many matrices of uneven size) through the C ABI.

* precond='none': each matrix's eigenvalues and rotation count are bit-identical to the
  single-problem path (whose pivot sequences equal the oracle's; the per-rotation
  arithmetic does not depend on the workgroup shape) and to the oracle itself.
* precond='fp32': every matrix meets the FP64 accuracy bar against its known spectrum
  (10 n u ||A||_2) with ||V^T V - I||_F <= 10 n u, and its status is OK.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_23187_amd import inputs as I
from paper_2607_23187_amd import jacobi as J

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
SIZES = [2, 3, 17, 40, 64, 65, 100, 128, 129, 200, 300, 520]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problems(sizes, seed):
    out = []
    for i, n in enumerate(sizes):
        if n >= 8:
            p = I.clustered(n, seed=seed + i, size=4, offset=1e-9)
            out.append((p.a, p.lam))
        else:
            a = I.random_symmetric(n, seed=seed + i)
            out.append((a, np.linalg.eigvalsh(a)))
    return out


def tol_for(a, lam):
    n = a.shape[0]
    return 10 * n * U * np.max(np.abs(lam)) / np.linalg.norm(a)


@pytest.mark.parametrize("pivot", ["greedy", "gap"])
def test_batched_plain_equals_single_and_oracle(pivot):
    probs = problems(SIZES, 7100)
    # one tolerance for the whole batch: the tightest of the members
    tol = min(tol_for(a, lam) for a, lam in probs)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    say("batched plain", pivot, [a.shape[0] for a, _ in probs])
    status, res = J.eigh_batched(mats, tol=tol, pivot=pivot, precond="none")
    assert status == J.OK
    for (a, lam), m, r in zip(probs, mats, res):
        n = a.shape[0]
        assert r.status == J.OK
        one = J.eigh(m, tol=tol, pivot=pivot, precond="none")
        assert r.stats["rotations"] == one.stats["rotations"], n
        assert torch.equal(r.w, one.w), n
        normF = np.linalg.norm(a)
        thr = O.threshold(O.STOP_CERT, tol, n, normF)
        ref = O.jacobi(a, pivot=O.GAP if pivot == "gap" else O.GREEDY, stop=O.STOP_CERT,
                       thr=thr, scan=1, want_vj=False)
        assert r.stats["rotations"] == ref.rotations, n
        assert np.array_equal(r.w.cpu().numpy(), np.sort(np.diag(ref.a))), n
        v = r.v.cpu().numpy()
        assert np.linalg.norm(v.T @ v - np.eye(n)) <= 10 * n * U


@pytest.mark.parametrize("pivot", ["greedy", "gap"])
def test_batched_preconditioned_accuracy(pivot, fp32_block=0):
    sizes = [2, 5, 31, 32, 33, 64, 97, 128, 160, 256, 333, 512]
    probs = problems(sizes, 7300)
    tol = min(tol_for(a, lam) for a, lam in probs)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    say("batched fp32", pivot, sizes, "block rows", fp32_block)
    status, res = J.eigh_batched(mats, tol=tol, pivot=pivot, precond="fp32",
                                 fp32_block=fp32_block)
    assert status == J.OK
    for (a, lam), r in zip(probs, res):
        n = a.shape[0]
        assert r.status == J.OK, n
        w = r.w.cpu().numpy()
        lam2 = np.max(np.abs(lam))
        assert np.max(np.abs(w - np.sort(lam))) <= 10 * n * U * lam2, n
        v = r.v.cpu().numpy()
        assert np.linalg.norm(v.T @ v - np.eye(n)) <= 10 * n * U, n
        # eigenpairs: the certificate bounds every remaining L_ij by thr, hence every
        # remaining |a_ij| by sqrt(thr (|delta| + |a_ij|)) <= sqrt(4 thr ||A||_2); the
        # residual of the pairs is at most the Frobenius norm of those entries
        normF = np.linalg.norm(a)
        thr = tol * normF / (2.0 * n * (n - 1))
        resid = np.linalg.norm(a @ v - v * w[None, :])
        assert resid <= n * np.sqrt(4 * thr * lam2) + 100 * n * U * normF, n


def test_batched_sixteen_row_blocks():
    """The batched FP32 stage with 16-row blocks (opts.fp32_block = 16) meets the same bar."""
    test_batched_preconditioned_accuracy("gap", fp32_block=16)


def test_batched_repeatable_and_order_independent():
    """The same matrix gives the same bits alone, in a batch, and at another batch position."""
    probs = problems([150, 40, 300, 64], 7500)
    tol = min(tol_for(a, lam) for a, lam in probs)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    _, r1 = J.eigh_batched(mats, tol=tol, pivot="gap", precond="fp32")
    _, r2 = J.eigh_batched(mats[::-1], tol=tol, pivot="gap", precond="fp32")
    _, r3 = J.eigh_batched([mats[2]], tol=tol, pivot="gap", precond="fp32")
    for i in range(4):
        assert torch.equal(r1[i].w, r2[3 - i].w)
        assert torch.equal(r1[i].v, r2[3 - i].v)
    assert torch.equal(r1[2].w, r3[0].w)


def test_batched_nonfinite_member():
    probs = problems([40, 60], 7700)
    a_bad = probs[1][0].copy()
    a_bad[3, 5] = a_bad[5, 3] = np.nan
    mats = [torch.from_numpy(probs[0][0]).cuda(), torch.from_numpy(a_bad).cuda()]
    status, res = J.eigh_batched(mats, tol=1e-12, pivot="gap", precond="fp32")
    assert res[0].status == J.OK
    assert res[1].status == J.ERR_NONFINITE
    assert status == J.ERR_NONFINITE


def test_tuned_shapes_do_not_change_results():
    """The workgroup shapes picked by the size-class tuner change no bit of the results."""
    probs = problems([40, 100, 128, 150, 300, 500], 7900)
    tol = min(tol_for(a, lam) for a, lam in probs)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    _, r0 = J.eigh_batched(mats, tol=tol, pivot="gap", precond="fp32", tune=False)
    _, r1 = J.eigh_batched(mats, tol=tol, pivot="gap", precond="fp32", tune=True)
    for x, y in zip(r0, r1):
        assert x.stats["rotations"] == y.stats["rotations"]
        assert torch.equal(x.w, y.w)
        assert torch.equal(x.v, y.v)


@pytest.mark.parametrize("threads", [128, 256])
@pytest.mark.parametrize("pivot", ["greedy", "gap"])
def test_forced_shapes_give_the_same_bits(pivot, threads):
    """The other workgroup shapes the tuner may pick for the HBM-resident members
    (opts.batch_threads: 128 threads x up to 4 rows, 256 x up to 2) give the bits of the
    default 512 x 1."""
    probs = problems([70, 100, 129, 200, 300, 500], 8300)
    tol = min(tol_for(a, lam) for a, lam in probs)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    say("forced shape", pivot, threads)
    s0, r0 = J.eigh_batched(mats, tol=tol, pivot=pivot, precond="fp32", tune=False)
    s1, r1 = J.eigh_batched(mats, tol=tol, pivot=pivot, precond="fp32", tune=False,
                            batch_threads=threads)
    assert s0 == s1 == J.OK
    for x, y in zip(r0, r1):
        assert x.stats["rotations"] == y.stats["rotations"]
        assert torch.equal(x.w, y.w)
        assert torch.equal(x.v, y.v)


@pytest.mark.parametrize("pivot", ["greedy", "gap"])
def test_batched_timestamp_and_mirror_modes_agree(pivot):
    """The persistent batched launch keeps A current either by mirrored column stores
    (update_mode mirror) or by per-row write timestamps (the default): same arithmetic, so the same
    rotation counts and bits, including across log drains (without the preconditioner the
    520-row matrix needs more rotations than one log holds)."""
    probs = problems([129, 200, 300, 520], 8100)
    tol = min(tol_for(a, lam) for a, lam in probs)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    say("batched modes", pivot)
    _, rm = J.eigh_batched(mats, tol=tol, pivot=pivot, precond="none", update_mode="mirror")
    _, rt = J.eigh_batched(mats, tol=tol, pivot=pivot, precond="none")
    for x, y in zip(rm, rt):
        assert x.status == y.status == J.OK
        assert x.stats["rotations"] == y.stats["rotations"]
        assert torch.equal(x.w, y.w)
        assert torch.equal(x.v, y.v)


@pytest.mark.parametrize("precond", ["none", "fp32"])
def test_graph_replay_equals_direct_launches(precond):
    """opts.graph: the FP32 rounds, the Newton-Schulz steps and the persistent FP64
    launches replayed from captured graphs (many replays per solve, host synchronisations
    between them, a re-capture whenever members leave) give the same bits as direct
    launches; a second graph solve on a smaller batch starts from fresh graphs."""
    probs = problems(SIZES, 7600)
    tol = min(tol_for(a, lam) for a, lam in probs)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    say("graph replay", precond, SIZES)
    st0, direct = J.eigh_batched(mats, tol=tol, pivot="gap", precond=precond)
    for sub in (mats, mats[3:9]):
        st1, graph = J.eigh_batched(sub, tol=tol, pivot="gap", precond=precond, graph=True)
        assert st1 == st0 == J.OK
        off = 0 if sub is mats else 3
        for i, r in enumerate(graph):
            d = direct[i + off]
            assert r.status == J.OK
            assert r.stats["rotations"] == d.stats["rotations"], i
            assert torch.equal(r.w, d.w), i
            assert torch.equal(r.v, d.v), i
    # and through the server (cohorts admitted while others run)
    srv = J.Server(workers=2, hbm_budget=64 << 20, tol=tol, pivot="gap", precond=precond,
                   graph=True)
    for t, m in enumerate(mats):
        srv.submit(m, t)
    got = 0
    while got < len(mats):
        for rec in srv.poll(wait=True):
            got += 1
            d = direct[rec["tag"]]
            assert rec["status"] == J.OK
            assert torch.equal(rec["w"], d.w), rec["n"]
            if rec["n"] >= 2:
                assert torch.equal(rec["v"], d.v), rec["n"]
    srv.close()
