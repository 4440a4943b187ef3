"""The request server (jacobi_server_*) through the C ABI.

* A mix of sizes submitted at once to two workers with a small device budget (so that the
  requests are spread over several concurrent batches): every result has the same bits as
  the same problem solved alone -- by the single-problem call without preconditioner, by a
  batch of one with it -- and every record's times are ordered.
* Requests trickling in while workers are busy are all completed.
"""
import sys
import time

import numpy as np
import pytest
import torch

from paper_2607_23187_amd import inputs as I
from paper_2607_23187_amd import jacobi as J

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
SIZES = [1, 2, 9, 33, 64, 100, 129, 200, 257, 64, 40, 300, 17, 128]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mats(seed):
    out = []
    for i, n in enumerate(SIZES):
        if n >= 8:
            out.append(torch.from_numpy(I.clustered(n, seed=seed + i, size=4, offset=1e-9).a).cuda())
        else:
            out.append(torch.from_numpy(I.random_symmetric(n, seed=seed + i)).cuda())
    return out


@pytest.mark.parametrize("precond", ["none", "fp32"])
def test_served_equals_alone(precond):
    ms = mats(8100)
    tol = 1e-13
    say("serving mix", precond, SIZES)
    srv = J.Server(workers=2, hbm_budget=8 << 20, tol=tol, pivot="gap", precond=precond)
    for t, m in enumerate(ms):
        srv.submit(m, t)
    recs = []
    while len(recs) < len(ms):
        recs += srv.poll(wait=True)
    srv.close()
    assert sorted(r["tag"] for r in recs) == list(range(len(ms)))
    assert max(r["batch"] for r in recs) > 1          # requests were batched
    assert len({(r["t_start"], r["t_done"]) for r in recs}) > 1  # over several batches
    for r in recs:
        m = ms[r["tag"]]
        assert r["status"] == J.OK
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
        if precond == "none":
            one = J.eigh(m, tol=tol, pivot="gap", precond="none")
        else:
            _, res = J.eigh_batched([m], tol=tol, pivot="gap", precond="fp32")
            one = res[0]
        assert torch.equal(r["w"], one.w), r["n"]
        if r["n"] >= 2:
            assert r["rotations"] == one.stats["rotations"]
            assert torch.equal(r["v"], one.v), r["n"]


def test_trickle():
    ms = mats(8300)
    srv = J.Server(workers=2, hbm_budget=4 << 20, tol=1e-13, pivot="gap", precond="fp32")
    for t, m in enumerate(ms):
        srv.submit(m, t)
        time.sleep(0.002)
    got = set()
    while len(got) < len(ms):
        for r in srv.poll(wait=True):
            assert r["status"] == J.OK
            got.add(r["tag"])
    assert srv.pending() == 0
    srv.close()
