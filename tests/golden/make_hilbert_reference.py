"""Writes hilbert_cholesky_sv.json: the singular values of the closed-form Cholesky factor
C_n of the Hilbert matrix (Sec. 4.2) for n = 20, 40, 100, as 30-digit decimal strings, and
the oracle's one-sided Jacobi SVD of fl64(C_100) under the relative score (Sec. 4.2, no
preconditioning): its rotation count and the SHA-256 of its pivot log and singular values.

The singular values are the square roots of the eigenvalues of H_n = C_n C_n^T, computed by
``oracle.hilbert_singular_values`` in multiprecision.  Each is computed at two working
precisions, and the script stops unless the two agree to 40 significant digits.  It calls
only the oracle and the input generators."""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import mpmath as mp  # noqa: E402

import oracle as O  # noqa: E402
from paper_2607_23187_amd import inputs as I  # noqa: E402


def main():
    out = {"source": "sqrt(eig(H_n)), H_n = (1/(i+j-1)), mpmath eigsy; see the docstring of "
                     "make_hilbert_reference.py", "sv": {}}
    for n in (20, 40, 100):
        dps = 60 + 2 * n
        a = O.hilbert_singular_values(n, dps)
        b = O.hilbert_singular_values(n, dps + 40)
        with mp.workdps(dps + 40):
            worst = max(abs(x - y) / y for x, y in zip(a, b))
        assert worst < mp.mpf(10) ** -40, (n, worst)
        out["sv"][str(n)] = [mp.nstr(x, 30, min_fixed=1, max_fixed=0) for x in b]
        print(n, "agree to", mp.nstr(worst, 3), flush=True)
    c = I.hilbert_cholesky(100)
    r = O.svd(c, 2.0 ** -53, pivot=O.RELATIVE, maxrot=400000, logcap=400000)
    out["c100_relative"] = {
        "tol": 2.0 ** -53, "rotations": r.rotations, "status": r.status, "thr": r.thr,
        "pivots_sha256": hashlib.sha256(np.ascontiguousarray(r.pivots, dtype=np.int32)
                                        .tobytes()).hexdigest(),
        "sv_sha256": hashlib.sha256(np.ascontiguousarray(r.s).tobytes()).hexdigest(),
    }
    print("c100 relative:", r.rotations, "rotations", flush=True)
    with open(os.path.join(HERE, "hilbert_cholesky_sv.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
