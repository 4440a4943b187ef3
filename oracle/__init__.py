"""CPU oracle for the preconditioned Jacobi eigensolver with gap-aware pivoting.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product.  It shares no code with the HIP
path; the only thing both sides consume is the seeded input module.

Pipeline (Shao & Nakatsukasa, Sec. 2.1 and Algorithm 1):

1. read the upper triangle of A and mirror it (Algorithm 1 input: a symmetric matrix);
2. ``precond='fp32'``: cyclic FP32 Jacobi -> V_l (Sec. 2.1, low-precision spectral
   decomposition), re-orthogonalised in FP64 by Householder QR with diag(R) > 0 (the
   experiments of Sec. 4 use Householder QR).  With ``passes=2`` (default) the FP32
   decomposition is refined once: FP32 Jacobi again on fl32(Q^T A Q), Q <- QR(Q V_2).
   Then A_hat = Q^T (A Q), symmetrised.  The FP32 Jacobi skips pairs that FP32 cannot
   separate (a_pq and a_pp - a_qq both at the rounding level of the diagonal) and leaves
   them to the FP64 phase;
3. FP64 Jacobi on A_hat with greedy or gap-aware pivots (eq. (1)) until the chosen stop
   rule holds (Theorem 1 certificate by default);
4. V = Q V_J, optionally polished by one Newton-Schulz step; eigenvalues =
   diag(A_final), sorted ascending with V's columns permuted.

The Jacobi loop itself is C (``jacobi_oracle.cpp``), compiled without FMA contraction.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

GREEDY, GAP, RELATIVE = 0, 1, 2
STOP_CERT, STOP_OFF, STOP_SCORE = 0, 1, 2
OK, MAXROT, STALL, NONFINITE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle's C++ into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [("rotations", ctypes.c_longlong), ("rescans", ctypes.c_longlong),
                ("final_sel", ctypes.c_double), ("final_cert", ctypes.c_double),
                ("final_off", ctypes.c_double), ("status", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp, ip, fp = (ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                      ctypes.POINTER(ctypes.c_float))
        L.orc_score_gap.restype = ctypes.c_double
        L.orc_score_gap.argtypes = [ctypes.c_double] * 3
        L.orc_rotation.restype = None
        L.orc_rotation.argtypes = [ctypes.c_double] * 3 + [dp] * 3
        L.orc_jacobi.restype = ctypes.c_int
        L.orc_jacobi.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_longlong, ctypes.c_int, dp, ip, dp, ctypes.c_longlong,
                                 ctypes.POINTER(_Stats)]
        L.orc_score_rel.restype = ctypes.c_double
        L.orc_score_rel.argtypes = [ctypes.c_double] * 3
        L.orc_svd1.restype = ctypes.c_int
        L.orc_svd1.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_longlong, ctypes.c_int, dp, dp, ip, dp,
                               ctypes.c_longlong, ctypes.POINTER(_Stats)]
        L.orc_jacobi_f32.restype = ctypes.c_int
        L.orc_jacobi_f32.argtypes = [fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


# ----------------------------------------------------------------- primitives
def score_gap(aii: float, ajj: float, aij: float) -> float:
    """eq. (1) for one pair (0 when a_ij == 0)."""
    return lib().orc_score_gap(aii, ajj, aij)


def score_rel(aii: float, ajj: float, aij: float) -> float:
    """Relative score of Sec. 4.2, (1/a_ii + 1/a_jj) L_ij, for an SPD 2 x 2 block."""
    return lib().orc_score_rel(aii, ajj, aij)


def rotation(app: float, aqq: float, apq: float):
    """(t, c, s) of the Jacobi rotation that diagonalises [[app, apq], [apq, aqq]]."""
    t, c, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_rotation(app, aqq, apq, ctypes.byref(t), ctypes.byref(c), ctypes.byref(s))
    return t.value, c.value, s.value


@dataclass
class JacobiResult:
    a: np.ndarray              # final matrix
    vj: np.ndarray | None      # product of the rotations
    pivots: np.ndarray         # (rotations, 2) int32
    cs: np.ndarray             # (rotations, 2) float64
    rotations: int
    rescans: int
    final_sel: float
    final_cert: float
    final_off: float
    status: int


def jacobi(a: np.ndarray, pivot: int = GAP, stop: int = STOP_CERT, thr: float = 0.0,
           maxrot: int | None = None, scan: int = 1, want_vj: bool = True,
           logcap: int | None = None) -> JacobiResult:
    """FP64 Jacobi (Algorithm 1) on a full symmetric matrix, absolute threshold ``thr``."""
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    if maxrot is None:
        maxrot = max(64, 40 * n * n)
    if logcap is None:
        logcap = min(maxrot, 40 * n * n + 64)
    vj = np.empty((n, n)) if want_vj else None
    plog = np.empty((logcap, 2), dtype=np.int32)
    cslog = np.empty((logcap, 2), dtype=np.float64)
    st = _Stats()
    lib().orc_jacobi(_dp(a), n, pivot, stop, float(thr), int(maxrot), scan, _dp(vj),
                     plog.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(cslog),
                     int(logcap), ctypes.byref(st))
    r = int(st.rotations)
    k = min(r, logcap)
    return JacobiResult(a, vj, plog[:k].copy(), cslog[:k].copy(), r, int(st.rescans),
                        st.final_sel, st.final_cert, st.final_off, int(st.status))


F32_TOL1, F32_RHO1 = 2.0 ** -22, 1.0   # single pass: FP32 floor of off(fl32(A)), or no progress
# first of two passes: the refinement restarts from fl32(Q^T A Q), whose off-norm is at the
# FP32 level whatever the first pass reached, so the first pass stops earlier
F32_TOL1_REFINED = 2.0 ** -18
# refinement passes: until a sweep fails to halve off, or off <= 2^-30 ||A32||_F (below
# that what remains is the FP32-level coupling inside clusters that the pass skips)
F32_TOL2, F32_RHO2 = 2.0 ** -30, 0.5


def jacobi_f32(a: np.ndarray, max_sweeps: int = 20, tol: float = F32_TOL1,
               rho: float = F32_RHO1, verbose: bool = False):
    """Cyclic FP32 Jacobi: returns (A32_final, V32, sweeps).  Pairs whose a_pq and
    a_pp - a_qq are both at FP32 rounding level of the diagonal are skipped; sweeps stop at
    off <= tol ||A32||_F, when a sweep leaves off >= rho times its previous value, or after
    ``max_sweeps``."""
    a32 = np.array(a, dtype=np.float32, order="C", copy=True)
    n = a32.shape[0]
    v32 = np.empty((n, n), dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    sweeps = lib().orc_jacobi_f32(a32.ctypes.data_as(fp), n, v32.ctypes.data_as(fp),
                                  max_sweeps, tol, rho, 1 if verbose else 0)
    return a32, v32, sweeps


def householder_q(x: np.ndarray) -> np.ndarray:
    """Orthogonal factor of a Householder QR (LAPACK geqrf/orgqr) with diag(R) > 0."""
    q, r = np.linalg.qr(np.asarray(x, dtype=np.float64))
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


@dataclass
class EighResult:
    w: np.ndarray
    v: np.ndarray | None
    rotations: int
    pivots: np.ndarray
    status: int
    normF: float
    thr: float
    a_hat: np.ndarray
    q: np.ndarray | None
    sweeps32: int = 0
    extra: dict = field(default_factory=dict)


def polish(v: np.ndarray) -> np.ndarray:
    """One Newton-Schulz step toward the nearest orthogonal matrix, written as a small
    correction: R = I - V^T V, V <- V + V R / 2 (Sec. 2.1 names Newton-Schulz as one way
    to orthogonalise in working precision)."""
    r = np.eye(v.shape[1]) - v.T @ v
    return v + 0.5 * (v @ r)


def symmetric_from_upper(a: np.ndarray) -> np.ndarray:
    """Algorithm 1 input: take the upper triangle (i <= j) and mirror it."""
    a = np.asarray(a, dtype=np.float64)
    u = np.triu(a)
    return u + np.triu(a, 1).T


def threshold(stop: int, tol: float, n: int, normF: float) -> float:
    """Absolute threshold from a relative tolerance.  Certificate: Theorem 1 asks for
    max L_ij <= tau / (2 n (n-1)) to guarantee |lambda_k - a_kk| <= tau, tau = tol ||A||_F."""
    if stop == STOP_CERT:
        return tol * normF / (2.0 * n * (n - 1)) if n > 1 else 0.0
    return tol * normF


def eigh(a: np.ndarray, tol: float, pivot: int = GAP, precond: str = "fp32",
         stop: int = STOP_CERT, abs_thr: float | None = None, want_v: bool = True,
         maxrot: int | None = None, scan: int = 1, sweeps32: int = 20,
         polish_v: bool = True, passes: int = 2, verbose: bool = False) -> EighResult:
    """Whole preconditioned solve: returns ascending eigenvalues and eigenvectors.
    ``verbose`` prints the progress of the FP32 sweeps on stderr."""
    a = symmetric_from_upper(a)
    n = a.shape[0]
    if not np.all(np.isfinite(a)):
        return EighResult(np.full(n, np.nan), None, 0, np.empty((0, 2), np.int32), NONFINITE,
                          float("nan"), float("nan"), a, None)
    normF = float(np.sqrt(np.sum(a * a)))
    thr = abs_thr if abs_thr is not None else threshold(stop, tol, n, normF)
    q = None
    sw = 0
    if precond == "fp32" and n > 1:
        _, v32, sw = jacobi_f32(a, max_sweeps=sweeps32,
                                 tol=F32_TOL1 if passes == 1 else F32_TOL1_REFINED,
                                 verbose=verbose)
        q = householder_q(v32.astype(np.float64))
        for _ in range(passes - 1):
            a1 = q.T @ (a @ q)
            a1 = 0.5 * (a1 + a1.T)
            _, v2, sw2 = jacobi_f32(a1, max_sweeps=sweeps32, tol=F32_TOL2, rho=F32_RHO2,
                                    verbose=verbose)
            sw += sw2
            q = householder_q(q @ v2.astype(np.float64))
        a_hat = q.T @ (a @ q)
        a_hat = 0.5 * (a_hat + a_hat.T)
    else:
        a_hat = a.copy()
    res = jacobi(a_hat, pivot=pivot, stop=stop, thr=thr, maxrot=maxrot, scan=scan,
                 want_vj=want_v)
    d = np.diag(res.a).copy()
    order = np.argsort(d, kind="stable")
    w = d[order]
    v = None
    if want_v:
        v = res.vj if q is None else q @ res.vj
        if polish_v:
            v = polish(v)
        v = np.ascontiguousarray(v[:, order])
    return EighResult(w, v, res.rotations, res.pivots, res.status, normF, thr, a_hat, q, sw,
                      {"final_cert": res.final_cert, "final_off": res.final_off,
                       "rescans": res.rescans})


def total_relative_error(lam_exact: np.ndarray, lam: np.ndarray) -> float:
    """Sec. 4 error measure: sum_i |lambda_i - lambda_hat_i| / ||A||_2 (both sorted)."""
    lam_exact = np.sort(lam_exact)
    return float(np.sum(np.abs(lam_exact - np.sort(lam))) / np.max(np.abs(lam_exact)))


# ----------------------------------------------------------------- one-sided SVD (Alg. 2)
@dataclass
class SvdResult:
    s: np.ndarray              # singular values, descending
    u: np.ndarray | None       # m x n, columns b_k / s_k (0 where s_k == 0)
    v: np.ndarray | None       # n x n right factor
    x: np.ndarray              # final columns of B (as rows, n x m), unsorted
    g: np.ndarray              # Gram matrix of the final columns, unsorted
    rotations: int
    rescans: int
    pivots: np.ndarray
    cs: np.ndarray
    status: int
    normF: float               # ||B^T B||_F of the input
    thr: float
    final_sel: float
    sweeps32: int = 0


def gram_rows(x: np.ndarray) -> np.ndarray:
    """x x^T with every entry a dot product summed in index order (as the C loop does)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    g = np.empty((n, n))
    for i in range(n):
        for j in range(i, n):
            s = 0.0
            for a, b in zip(x[i], x[j]):
                s += a * b
            g[i, j] = g[j, i] = s
    return g


def svd_threshold(pivot: int, tol: float, n: int, normF: float) -> float:
    """Stop threshold of the one-sided method.  Greedy and gap: Theorem 1 on A = B^T B,
    tol ||A||_F / (2 n (n-1)) (|a_ij| >= L_ij, so the greedy rule implies the certificate).
    Relative: tol / (2 n (n-1)); Lhat is scale-free and bounds the relative shifts of the
    2 x 2 eigenvalues, so tol plays the part of a relative error."""
    if n < 2:
        return 0.0
    if pivot == RELATIVE:
        return tol / (2.0 * n * (n - 1))
    return tol * normF / (2.0 * n * (n - 1))


def svd(b: np.ndarray, tol: float, pivot: int = GAP, precond: str = "none",
        abs_thr: float | None = None, maxrot: int | None = None, scan: int = 1,
        sweeps32: int = 20, passes: int = 2, logcap: int | None = None,
        want_uv: bool = True) -> SvdResult:
    """One-sided Jacobi SVD of B (m x n, m >= n), Algorithm 2.

    ``precond='fp32'`` (Sec. 2.1): right singular vectors in FP32 as the eigenvectors of
    fl32(B^T B) from the cyclic FP32 Jacobi (refined ``passes - 1`` times as in ``eigh``),
    re-orthogonalised by Householder QR -> V; the one-sided method then runs on B V with
    its Gram matrix (B V)^T B V as the pivoting matrix.  ``'none'``: B itself (the setting
    of Sec. 4.2, where global transformations would spoil relative accuracy)."""
    b = np.asarray(b, dtype=np.float64)
    m, n = b.shape
    x = np.ascontiguousarray(b.T)
    if not np.all(np.isfinite(x)):
        return SvdResult(np.full(n, np.nan), None, None, x, np.full((n, n), np.nan), 0, 0,
                         np.empty((0, 2), np.int32), np.empty((0, 2)), NONFINITE,
                         float("nan"), float("nan"), float("nan"))
    g0 = x @ x.T
    normF = float(np.sqrt(np.sum(g0 * g0)))
    thr = abs_thr if abs_thr is not None else svd_threshold(pivot, tol, n, normF)
    vt = np.eye(n)
    sw = 0
    if precond == "fp32" and n > 1:
        g0 = 0.5 * (g0 + g0.T)
        _, v32, sw = jacobi_f32(g0, max_sweeps=sweeps32,
                                 tol=F32_TOL1 if passes == 1 else F32_TOL1_REFINED)
        q = householder_q(v32.astype(np.float64))
        for _ in range(passes - 1):
            a1 = q.T @ (g0 @ q)
            a1 = 0.5 * (a1 + a1.T)
            # refinement without the off-norm floor: a graded B puts eigenvalues of B^T B
            # far below 2^-30 ||B^T B||, and their vectors need the longer refinement
            _, v2, sw2 = jacobi_f32(a1, max_sweeps=sweeps32, tol=0.0, rho=F32_RHO2)
            sw += sw2
            q = householder_q(q @ v2.astype(np.float64))
        x = np.ascontiguousarray(q.T @ x)
        vt = np.ascontiguousarray(q.T)
    if maxrot is None:
        maxrot = max(64, 40 * n * n)
    if logcap is None:
        logcap = min(maxrot, 40 * n * n + 64)
    g = np.empty((n, n))
    plog = np.empty((logcap, 2), dtype=np.int32)
    cslog = np.empty((logcap, 2), dtype=np.float64)
    st = _Stats()
    lib().orc_svd1(_dp(x), m, n, pivot, float(thr), int(maxrot), scan, _dp(vt), _dp(g),
                   plog.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(cslog), int(logcap),
                   ctypes.byref(st))
    r = int(st.rotations)
    k = min(r, logcap)
    sig = np.sqrt(np.diag(g))
    order = np.argsort(-sig, kind="stable")
    u = v = None
    if want_uv:
        safe = np.where(sig > 0, sig, 1.0)
        u = np.where(sig[None, :] > 0, x.T / safe[None, :], 0.0)[:, order]
        v = vt.T[:, order].copy()
    return SvdResult(sig[order], u, v, x, g, r, int(st.rescans), plog[:k].copy(),
                     cslog[:k].copy(), int(st.status), normF, thr, st.final_sel, sw)


def hilbert_singular_values(n: int, dps: int):
    """Singular values of the Cholesky factor C_n of the Hilbert matrix H_n (Sec. 4.2), as
    mpmath numbers of ``dps`` digits, descending.  H_n = C_n C_n^T, so they are the square
    roots of the eigenvalues of H_n = (1/(i+j-1)), computed by mpmath's symmetric eigensolver
    in ``dps``-digit arithmetic (the entries of H_n are its only input)."""
    import mpmath as mp
    with mp.workdps(dps):
        h = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                h[i, j] = mp.mpf(1) / (i + j + 1)
        ev = mp.eigsy(h, eigvals_only=True)
        vals = sorted((ev[i] for i in range(n)), reverse=True)
        return [mp.sqrt(v) for v in vals]
