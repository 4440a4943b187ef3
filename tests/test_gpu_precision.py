"""Precision variant of the contraction Q^T A Q: three-slice BF16 products on the matrix
cores with FP32 accumulation flushed into FP64 every 128 terms (opts.split_gemm = 1),
against the FP64 MFMA products.

The variant's A_hat carries FP32-level error, so its eigenvalues are FP32-accurate (error
about 2^-24 ||A|| sqrt(n)), not FP64-accurate; the FP64 path on the same input stays within
10 n u ||A||_2.  Both are reported by the precision benchmark."""
import sys

import numpy as np
import pytest
import torch

from paper_2607_23187_amd import inputs as I
from paper_2607_23187_amd import jacobi as J

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.mark.parametrize("n", [100, 512, 1000])
def test_split_contraction_error(n):
    p = I.clustered(n, seed=9100 + n, size=8, offset=1e-10)
    lam2 = float(np.max(np.abs(p.lam)))
    tol = 10 * n * U * lam2 / np.linalg.norm(p.a)
    a = torch.from_numpy(p.a).cuda()
    print("precision variant", n, flush=True)
    r64 = J.eigh(a, tol=tol, pivot="gap", precond="fp32")
    rsp = J.eigh(a, tol=tol, pivot="gap", precond="fp32", split_gemm=True)
    assert r64.status == J.OK and rsp.status == J.OK
    e64 = np.max(np.abs(r64.w.cpu().numpy() - p.lam))
    esp = np.max(np.abs(rsp.w.cpu().numpy() - p.lam))
    assert e64 <= 10 * n * U * lam2
    # FP32-level: within a small multiple of u_32 ||A||_F, and clearly worse than FP64
    assert esp <= 4 * U32 * np.linalg.norm(p.a)
    assert esp > e64
    v = rsp.v.cpu().numpy()
    assert np.linalg.norm(v.T @ v - np.eye(n)) <= 10 * n * U
