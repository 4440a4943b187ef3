"""The request server (jacobi_server_*) through the C ABI: continuous batching.

* A mix of sizes submitted to two lanes with a small device budget: every result has the
  same bits as the same problem solved in a batch of its own, and agrees with the oracle --
  bit for bit without the preconditioner (and without the polish, whose products round
  differently on the two sides), within 10 n u ||A||_2 with it.
* Requests that arrive while a cohort is running are admitted at a step boundary and start
  before that cohort has finished; finished members leave before their cohort ends.
* A budget that holds only a few workspaces: requests wait for memory and all complete.
"""
import sys
import time

import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_23187_amd import inputs as I
from paper_2607_23187_amd import jacobi as J

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
SIZES = [1, 2, 9, 33, 64, 100, 129, 200, 257, 64, 40, 300, 17, 128]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problems(seed, sizes=SIZES):
    out = []
    for i, n in enumerate(sizes):
        if n >= 8:
            p = I.clustered(n, seed=seed + i, size=4, offset=1e-9)
            out.append((p.a, p.lam))
        else:
            a = I.random_symmetric(n, seed=seed + i)
            out.append((a, np.linalg.eigvalsh(a)))
    return out


def serve(mats, **kw):
    srv = J.Server(**kw)
    for t, m in enumerate(mats):
        srv.submit(m, t)
    recs = []
    while len(recs) < len(mats):
        recs += srv.poll(wait=True)
    srv.close()
    return recs


@pytest.mark.parametrize("precond", ["none", "fp32"])
def test_served_equals_alone_and_oracle(precond):
    probs = problems(8100)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    tol = 1e-13
    say("serving mix", precond, SIZES)
    polish = precond == "fp32"
    recs = serve(mats, workers=2, hbm_budget=16 << 20, tol=tol, pivot="gap", precond=precond,
                 polish_v=polish)
    assert sorted(r["tag"] for r in recs) == list(range(len(mats)))
    assert max(r["batch"] for r in recs) > 1          # requests were batched
    for r in recs:
        a, lam = probs[r["tag"]]
        m = mats[r["tag"]]
        n = r["n"]
        assert r["status"] == J.OK
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
        # the same problem in a batch of its own: same bits
        _, res = J.eigh_batched([m], tol=tol, pivot="gap", precond=precond, polish_v=polish)
        one = res[0]
        assert torch.equal(r["w"], one.w), n
        if n >= 2:
            assert r["rotations"] == one.stats["rotations"]
            assert torch.equal(r["v"], one.v), n
        # the oracle on the same bytes
        if n < 2:
            continue
        lam2 = float(np.max(np.abs(lam)))
        if precond == "none":
            thr = one.stats["thr"]
            ref = O.jacobi(a, pivot=O.GAP, stop=O.STOP_CERT, thr=thr, scan=1, want_vj=True)
            d = np.diag(ref.a).copy()
            order = np.argsort(d, kind="stable")
            assert ref.rotations == r["rotations"], n
            assert np.array_equal(r["w"].cpu().numpy(), d[order]), n
            assert np.array_equal(r["v"].cpu().numpy(), ref.vj[:, order]), n
        else:
            ref = O.eigh(a, tol=tol, pivot=O.GAP, precond="fp32", stop=O.STOP_CERT,
                         want_v=False)
            assert np.max(np.abs(r["w"].cpu().numpy() - ref.w)) <= 10 * n * U * lam2, n


@pytest.mark.parametrize("lanes", [1, 2])
def test_continuous_admission(lanes):
    """A long cohort (n = 1500) is running when small requests arrive: they are admitted at
    a step boundary (of the running lane, or of an idle one) and start before the long one
    has finished; with a second lane they also finish first."""
    big = torch.from_numpy(I.clustered(1500, seed=8400, size=8, offset=1e-10).a).cuda()
    small = [torch.from_numpy(a).cuda() for a, _ in problems(8500, [40, 64, 100, 130])]
    say("continuous admission", lanes)
    srv = J.Server(workers=lanes, hbm_budget=2 << 30, tol=1e-13, pivot="gap", precond="fp32")
    srv.submit(big, 0)
    time.sleep(0.03)  # the big cohort is on the device
    for t, m in enumerate(small):
        srv.submit(m, t + 1)
    recs = []
    while len(recs) < 1 + len(small):
        recs += srv.poll(wait=True)
    srv.close()
    by = {r["tag"]: r for r in recs}
    assert all(r["status"] == J.OK for r in recs)
    t_big_done = by[0]["t_done"]
    assert by[0]["t_start"] < by[1]["t_submit"]       # the big one was running first
    for t in range(1, 1 + len(small)):
        assert by[t]["t_start"] < t_big_done, t      # admitted while the big one ran
        if lanes > 1:
            assert by[t]["t_done"] < t_big_done, t   # and left before it


def test_admission_by_footprint():
    """A budget of a few workspaces: requests wait until memory is returned, all complete
    with the same bits as alone; a request larger than the whole budget is refused."""
    probs = problems(8600, [100, 200, 300, 150, 250, 120, 180, 220])
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    budget = 24 << 20  # about three workspaces of n = 300
    say("footprint admission", budget)
    recs = serve(mats, workers=2, hbm_budget=budget, tol=1e-13, pivot="gap", precond="fp32")
    assert all(r["status"] == J.OK for r in recs)
    for r in recs:
        _, res = J.eigh_batched([mats[r["tag"]]], tol=1e-13, pivot="gap", precond="fp32")
        assert torch.equal(r["w"], res[0].w)
    srv = J.Server(workers=1, hbm_budget=1 << 20, tol=1e-13, pivot="gap", precond="fp32")
    with pytest.raises(RuntimeError):
        srv.submit(mats[2], 0)
    srv.close()


def test_trickle():
    probs = problems(8300)
    mats = [torch.from_numpy(a).cuda() for a, _ in probs]
    srv = J.Server(workers=2, hbm_budget=16 << 20, tol=1e-13, pivot="gap", precond="fp32")
    for t, m in enumerate(mats):
        srv.submit(m, t)
        time.sleep(0.002)
    got = set()
    while len(got) < len(mats):
        for r in srv.poll(wait=True):
            assert r["status"] == J.OK
            got.add(r["tag"])
    assert srv.pending() == 0
    srv.close()
