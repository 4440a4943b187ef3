"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *constructs* test matrices: it draws spectra and a Haar-distributed
orthogonal factor and multiplies them out.  It contains none of the eigensolver's
arithmetic (no pivot scores, no rotations, no preconditioner), so both the CPU oracle
and the HIP path can consume its output without sharing any method code.

Spectra follow the paper's experiments:

* the 4x4 block-diagonal worked example of the introduction (Sec. 1);
* the clustered n=1000 spectrum of Sec. 4.1 (cluster ``1+exp(-alpha k)`` next to an
  equispaced block on ``[2,3]``);
* clustered spectra of the same kind at other sizes (tight clusters of a few
  eigenvalues with tiny offsets, mixed with well separated eigenvalues), which stand in
  for the paper's synthetic matrices at the sizes the benchmarks use.

Every matrix is ``A = Q diag(lam) Q^T`` with ``Q`` the orthogonal factor of a QR
factorisation of a seeded N(0,1) matrix, signs fixed so that ``diag(R) > 0``, then
symmetrised exactly as ``(A + A^T)/2``.  All arrays are float64, C-contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_C1 = 20261201  # single 64x64, 8 clusters of 8
SEED_C2 = 20261202  # single 1024x1024, half clustered, half log-uniform
SEED_C3 = 20261203  # single 4096x4096, clusters of 8
SEED_C4 = 20261204  # 2048 matrices, n log-uniform in [32, 512]
SEED_C5 = 20261205  # request stream, n log-uniform in [16, 2048]
SEED_P41 = 20261206  # Sec. 4.1 replication, n = 1000


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Orthogonal factor of QR(G), G ~ N(0,1)^{n x n}, with diag(R) made positive."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return np.ascontiguousarray(q * d[None, :])


def from_spectrum(lam: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """A = Q diag(lam) Q^T with a Haar Q, symmetrised exactly."""
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    q = haar_orthogonal(n, rng)
    a = (q * lam[None, :]) @ q.T
    a = 0.5 * (a + a.T)
    return np.ascontiguousarray(a)


# ---------------------------------------------------------------- spectra
def spectrum_clusters(n: int, size: int, rng: np.random.Generator,
                      lo: float = 1.0, hi: float = 2.0, offset: float = 1e-10) -> np.ndarray:
    """Clusters of ``size`` eigenvalues: centre U[lo,hi], members centre + U[0,offset]."""
    nclu = (n + size - 1) // size
    centres = rng.uniform(lo, hi, size=nclu)
    lam = np.repeat(centres, size)[:n] + rng.uniform(0.0, offset, size=nclu * size)[:n]
    return lam


def spectrum_c2(n: int, rng: np.random.Generator) -> np.ndarray:
    """Half: clusters of 16 with centres U[1,10], relative spread 1e-8; half log-uniform [1e-3,1e3]."""
    h = n // 2
    nclu = (h + 15) // 16
    centres = rng.uniform(1.0, 10.0, size=nclu)
    clustered = np.repeat(centres, 16)[:h] * (1.0 + rng.uniform(0.0, 1e-8, size=nclu * 16)[:h])
    spread = np.exp(rng.uniform(math.log(1e-3), math.log(1e3), size=n - h))
    return np.concatenate([clustered, spread])


def spectrum_mixed(n: int, rng: np.random.Generator) -> np.ndarray:
    """Batched-workload spectrum: with probability 1/2 clustered (cluster size U{4..16},
    spread log-uniform in [1e-10, 1e-6], centres U[1,2], last cluster truncated),
    otherwise uniform in [1,2]."""
    if rng.uniform() < 0.5:
        m = int(rng.integers(4, 17))
        sigma = math.exp(rng.uniform(math.log(1e-10), math.log(1e-6)))
        nclu = (n + m - 1) // m
        centres = rng.uniform(1.0, 2.0, size=nclu)
        return np.repeat(centres, m)[:n] + rng.uniform(0.0, sigma, size=nclu * m)[:n]
    return rng.uniform(1.0, 2.0, size=n)


def spectrum_sec41(n: int, alpha: float) -> np.ndarray:
    """Sec. 4.1: first half 1 + exp(-alpha k), second half 2 + (k-1)/(h-1), k = 1..h."""
    h = n // 2
    k = np.arange(1, h + 1, dtype=np.float64)
    return np.concatenate([1.0 + np.exp(-alpha * k), 2.0 + (k - 1.0) / (h - 1.0)])


# ---------------------------------------------------------------- workloads
@dataclass
class Problem:
    a: np.ndarray          # (n, n) float64 symmetric
    lam: np.ndarray        # exact spectrum used in the construction, ascending
    name: str


def worked_example() -> Problem:
    """The 4x4 block-diagonal matrix of the introduction (Sec. 1)."""
    a = np.zeros((4, 4))
    a[0, 0], a[0, 1], a[1, 0], a[1, 1] = 1.0, 1e-8, 1e-8, 2.0
    a[2, 2], a[2, 3], a[3, 2], a[3, 3] = 1.0, 1e-9, 1e-9, 1.0 + 1e-10
    return Problem(a, np.array([]), "worked_example")


def clustered(n: int, seed: int, size: int = 8, offset: float = 1e-10) -> Problem:
    """Clusters of ``size`` with centres U[1,2] and offsets U[0,offset] (64x64 and 4096x4096 recipe)."""
    rng = rng_for(seed)
    lam = spectrum_clusters(n, size, rng, offset=offset)
    return Problem(from_spectrum(lam, rng), np.sort(lam), f"clustered{size}_n{n}")


def config_c1() -> Problem:
    return clustered(64, SEED_C1, 8)


def config_c2(n: int = 1024, seed: int = SEED_C2) -> Problem:
    rng = rng_for(seed)
    lam = spectrum_c2(n, rng)
    return Problem(from_spectrum(lam, rng), np.sort(lam), f"c2_n{n}")


def config_c3(n: int = 4096) -> Problem:
    return clustered(n, SEED_C3, 8)


def sec41(n: int = 1000, alpha: float = 1.0, seed: int = SEED_P41) -> Problem:
    rng = rng_for(seed)
    lam = spectrum_sec41(n, alpha)
    return Problem(from_spectrum(lam, rng), np.sort(lam), f"sec41_n{n}_a{alpha}")


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = rng_for(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def config_c4(count: int = 2048, lo: int = 32, hi: int = 512, seed: int = SEED_C4):
    """Batch of independent matrices, n log-uniform in [lo, hi]; spectra by ``spectrum_mixed``."""
    sizes = batch_sizes(count, lo, hi, seed)
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for i, n in enumerate(sizes):
        rng = np.random.Generator(np.random.PCG64(children[i]))
        lam = spectrum_mixed(int(n), rng)
        out.append(Problem(from_spectrum(lam, rng), np.sort(lam), f"c4_{i}_n{n}"))
    return out


def config_c5_stream(count: int = 20000, lo: int = 16, hi: int = 2048, rate: float = 1.0,
                     seed: int = SEED_C5):
    """Request stream: Poisson arrival times at ``rate`` per second and sizes log-uniform in
    [lo, hi].  Matrices are built lazily by ``c5_problem`` (clusters of 8, offsets 1e-10)."""
    rng = rng_for(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    return arrivals, sizes


def c5_problem(i: int, n: int, seed: int = SEED_C5) -> Problem:
    child = np.random.SeedSequence([seed, i])
    rng = np.random.Generator(np.random.PCG64(child))
    lam = spectrum_clusters(n, 8, rng)
    return Problem(from_spectrum(lam, rng), np.sort(lam), f"c5_{i}_n{n}")


def nearly_diagonal(n: int, seed: int, eps: float = 1e-7, spectrum: str = "c2") -> Problem:
    """A matrix shaped like the output of a low-precision preconditioner: the diagonal is a
    spectrum (the recipe of the 1024-size benchmark by default, clusters of 8 otherwise) and
    the off-diagonal entries are symmetric N(0, (eps * ||lam||_inf)^2).  ``lam`` is the
    diagonal, not the exact spectrum."""
    rng = rng_for(seed)
    lam = spectrum_c2(n, rng) if spectrum == "c2" else spectrum_clusters(n, 8, rng)
    e = rng.standard_normal((n, n)) * (eps * float(np.max(np.abs(lam))))
    a = 0.5 * (e + e.T)
    a[np.diag_indices(n)] = lam
    return Problem(np.ascontiguousarray(a), np.sort(lam), f"nearly_diagonal_{spectrum}_n{n}")


def random_symmetric(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Dense symmetric matrix with N(0, scale^2) entries (no special spectrum)."""
    rng = rng_for(seed)
    g = rng.standard_normal((n, n)) * scale
    return np.ascontiguousarray(0.5 * (g + g.T))


# ----------------------------------------------------------------- SVD inputs
SEED_SVD = 20261207  # rectangular matrices of prescribed singular values


def hilbert_cholesky(n: int) -> np.ndarray:
    """Closed-form lower-triangular Cholesky factor C_n of the Hilbert matrix (Sec. 4.2):
    c_ij = sqrt(2j-1) ((i-1)!)^2 / ((i+j-1)! (i-j)!) for i >= j (1-based), 0 above the
    diagonal.  The factorial ratio is formed exactly as a rational number and rounded once;
    the square root is rounded once and the product once (about 1.5 ulp per entry)."""
    from fractions import Fraction
    c = np.zeros((n, n))
    f = [math.factorial(k) for k in range(2 * n)]
    for i in range(1, n + 1):
        for j in range(1, i + 1):
            ratio = Fraction(f[i - 1] ** 2, f[i + j - 1] * f[i - j])
            c[i - 1, j - 1] = math.sqrt(2 * j - 1) * float(ratio)
    return c


def with_singular_values(m: int, sv: np.ndarray, seed: int) -> np.ndarray:
    """B = U diag(sv) V^T (m x n, n = len(sv)) with Haar-distributed U (first n columns of
    an m x m factor) and V."""
    rng = rng_for(seed)
    n = len(sv)
    u = haar_orthogonal(m, rng)[:, :n]
    v = haar_orthogonal(n, rng)
    return np.ascontiguousarray((u * np.asarray(sv, dtype=np.float64)[None, :]) @ v.T)


def svd_graded(m: int, n: int, seed: int, decades: float = 12.0) -> np.ndarray:
    """Rectangular test matrix with singular values spread log-uniformly over `decades`
    decades, plus a pair of close singular values (the gap score's case)."""
    rng = rng_for(seed + 1)
    sv = np.sort(10.0 ** (-decades * rng.random(n)))[::-1].copy()
    if n >= 4:
        sv[n // 2] = sv[n // 2 - 1] * (1.0 - 1e-9)
    return with_singular_values(m, sv, seed)
