"""Writes full_size_parity.json: the oracle's FP64 pivoted-Jacobi results on an n = 1024
nearly diagonal input (the shape of a preconditioned matrix; inputs.nearly_diagonal seed 31,
eps 1e-7): rotation count, SHA-256 of the whole pivot log (int32 pairs) and of the sorted
final diagonal (float64), and every 4096th pivot.  The GPU test compares the HIP path
with these without re-running the oracle.  Calls only the oracle and the input generators."""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2607_23187_amd import inputs as I  # noqa: E402

N, SEED, EPS = 1024, 31, 1e-7


def threshold(a):
    n = a.shape[0]
    return 10 * n * 2.0 ** -53 * float(np.max(np.abs(np.diag(a)))) / (2.0 * n * (n - 1))


def main():
    p = I.nearly_diagonal(N, SEED, EPS)
    thr = threshold(p.a)
    out = {"input": f"inputs.nearly_diagonal({N}, {SEED}, {EPS})", "thr": thr, "runs": {}}
    for name, pivot in (("gap", O.GAP), ("greedy", O.GREEDY)):
        t = time.time()
        r = O.jacobi(p.a, pivot=pivot, stop=O.STOP_CERT, thr=thr, scan=1, want_vj=False)
        piv = np.ascontiguousarray(r.pivots.astype(np.int32))
        d = np.sort(np.diag(r.a))
        out["runs"][name] = {
            "rotations": int(r.rotations),
            "pivots_sha256": hashlib.sha256(piv.tobytes()).hexdigest(),
            "diag_sorted_sha256": hashlib.sha256(d.astype(np.float64).tobytes()).hexdigest(),
            "pivot_samples": {str(k): piv[k].tolist() for k in range(0, len(piv), 4096)},
            "seconds_here": time.time() - t,
        }
        print(name, out["runs"][name]["rotations"], time.time() - t, flush=True)
    with open(os.path.join(HERE, "full_size_parity.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
