"""Writes c2_oracle_counts.json: the oracle's FP32 sweep and FP64 rotation counts for the
n = 1024 benchmark matrix (half clusters of 16 with relative spread 1e-8, half
log-uniform eigenvalues over [1e-3, 1e3]), used to scale the benchmark's timed CPU
sample to one whole solve.  Calls only the oracle and the input generators."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2607_23187_amd import inputs as I  # noqa: E402


def main():
    p = I.config_c2()
    n = p.a.shape[0]
    u = 2.0 ** -53
    lam2 = float(np.max(np.abs(p.lam)))
    tol = 10 * n * u * lam2 / float(np.linalg.norm(p.a))
    out = {"workload": "c2 recipe n=1024 seed %d" % I.SEED_C2, "tol": tol, "runs": {}}
    for name, pivot, precond, passes in (("gap", O.GAP, "fp32", 2), ("greedy", O.GREEDY, "fp32", 2),
                                         ("gap_1pass", O.GAP, "fp32", 1)):
        t = time.time()
        e = O.eigh(p.a, tol=tol, pivot=pivot, precond=precond, passes=passes, want_v=False)
        out["runs"][name] = {
            "sweeps32": int(e.sweeps32), "rotations": int(e.rotations), "status": int(e.status),
            "max_abs_err_over_nu_norm2": float(np.max(np.abs(e.w - p.lam)) / (n * u * lam2)),
            "seconds_here": time.time() - t,
        }
        print(name, out["runs"][name], flush=True)
    with open(os.path.join(HERE, "c2_oracle_counts.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
