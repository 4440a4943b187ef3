"""Pins of the oracle's one-sided Jacobi SVD (Algorithm 2) and relative score (Sec. 4.2).

Each test compares the oracle with something independent of it: the exact eigenvalues of
2x2 blocks in multiprecision (what the scores measure), LAPACK, the defining identities
B V = U diag(S) and V^T V = I, brute-force argmax over all pairs, the multiprecision
singular values of the Hilbert Cholesky factor (themselves pinned by trace and determinant
closed forms), and the paper's statements about C_100.
"""
import hashlib
import json
import math
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle as O
from paper_2607_23187_amd import inputs as I

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def setup_module(_):
    O.build(force=False)


def golden():
    with open(os.path.join(GOLDEN, "hilbert_cholesky_sv.json")) as f:
        return json.load(f)


def ref_sv(n):
    return np.array([float(x) for x in golden()["sv"][str(n)]])


# ----------------------------------------------------------------- the relative score
def shifts_2x2(a, b, c):
    """Exact eigenvalue shifts of [[a, c], [c, b]] (multiprecision): (lam_hi - max(a, b),
    min(a, b) - lam_lo); both equal L of eq. (1)."""
    with mp.workprec(400):
        a, b, c = mp.mpf(a), mp.mpf(b), mp.mpf(c)
        mid, rad = (a + b) / 2, mp.sqrt(((a - b) / 2) ** 2 + c * c)
        return mid + rad - max(a, b), min(a, b) - (mid - rad), a, b


@pytest.mark.parametrize("a,b,c", [
    (1.0, 1.0, 1e-3), (2.0, 1.0, 0.3), (1.0, 1e-8, 1e-6), (1e-160, 3e-161, 1e-170),
    (7.5e-120, 7.5e-120 * (1 + 2 ** -40), 1e-140), (3.0, 0.5, -0.9), (1e30, 1e-30, 1e-5),
])
def test_rel_score_is_sum_of_relative_eigenvalue_shifts(a, b, c):
    # Sec. 4.2: (1/a_ii + 1/a_jj) L_ij with L_ij the shift of each eigenvalue of the block
    up, down, A, B = shifts_2x2(a, b, c)
    with mp.workprec(400):
        expect = up / max(A, B) + down / min(A, B)
    got = O.score_rel(a, b, c)
    assert abs(mp.mpf(got) - expect) <= 8 * U * abs(expect), (got, expect)


def test_rel_score_scale_invariant_and_zero():
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, b = 10.0 ** rng.uniform(-100, 100, 2)
        c = rng.uniform(-1, 1) * math.sqrt(a * b)
        s = O.score_rel(a, b, c)
        for k in (-300, -77, 1, 64, 200):
            if 0 < abs(math.ldexp(max(a, b), k)) < 1e300 and math.ldexp(min(a, b), k) > 1e-290:
                assert O.score_rel(math.ldexp(a, k), math.ldexp(b, k), math.ldexp(c, k)) == s
    assert O.score_rel(1.0, 2.0, 0.0) == 0.0
    assert O.score_rel(0.0, 0.0, 0.0) == 0.0


# ----------------------------------------------------------------- the one-sided method
def check_factorisation(b, r, tol_rel):
    m, n = b.shape
    bn = np.linalg.norm(b)
    # B V = U diag(S): the columns were rotated with the same G as V
    assert np.linalg.norm(b @ r.v - r.u * r.s[None, :]) <= 30 * n * U * bn
    assert np.linalg.norm(r.v.T @ r.v - np.eye(n)) <= 30 * n * U
    assert np.all(np.diff(r.s) <= 0)
    ls = np.linalg.svd(b, compute_uv=False)
    assert np.max(np.abs(r.s - ls)) <= tol_rel * ls[0]


@pytest.mark.parametrize("pivot,tol", [(O.GAP, U), (O.RELATIVE, U), (O.GREEDY, 1e-11)])
@pytest.mark.parametrize("m,n", [(40, 25), (33, 33), (70, 9)])
def test_svd_matches_lapack(pivot, tol, m, n):
    b = I.svd_graded(m, n, seed=m * 100 + n, decades=6.0)
    r = O.svd(b, tol, pivot=pivot)
    assert r.status == O.OK
    check_factorisation(b, r, 50 * m * U)


def test_relative_score_leaves_columns_orthogonal_to_its_bound():
    # at exit every Lhat_ij <= thr, and cos^2(b_i, b_j) <= 1.5 Lhat_ij for the 2x2 block
    b = I.svd_graded(50, 30, seed=77, decades=10.0)
    r = O.svd(b, U, pivot=O.RELATIVE)
    x = r.x
    with mp.workprec(200):
        worst = 0.0
        for i in range(30):
            for j in range(i + 1, 30):
                dij = mp.fsum(mp.mpf(p) * mp.mpf(q) for p, q in zip(x[i], x[j]))
                ni = mp.sqrt(mp.fsum(mp.mpf(p) ** 2 for p in x[i]))
                nj = mp.sqrt(mp.fsum(mp.mpf(p) ** 2 for p in x[j]))
                worst = max(worst, float(abs(dij) / (ni * nj)))
    assert worst <= math.sqrt(1.5 * r.thr) + 50 * 50 * U


@pytest.mark.parametrize("pivot,tol", [(O.GREEDY, 1e-12), (O.GAP, U), (O.RELATIVE, U)])
def test_row_cache_equals_full_scan(pivot, tol):
    b = I.svd_graded(36, 24, seed=3, decades=8.0)
    a = O.svd(b, tol, pivot=pivot, scan=0)
    c = O.svd(b, tol, pivot=pivot, scan=1)
    assert a.rotations == c.rotations > 0
    assert np.array_equal(a.pivots, c.pivots)
    assert np.array_equal(a.s, c.s)


@pytest.mark.parametrize("pivot", [O.GAP, O.RELATIVE])
def test_each_pivot_is_the_argmax_of_the_exact_block_shifts(pivot):
    # replay the logged rotations on B and check every pivot against the scores defined
    # through the exact eigenvalues of each 2x2 block of the exact Gram matrix
    b = I.svd_graded(12, 7, seed=11, decades=5.0)
    r = O.svd(b, U, pivot=pivot, maxrot=25)
    x = np.ascontiguousarray(b.T).copy()
    n = x.shape[0]
    for (p, q), (c, s) in zip(r.pivots, r.cs):
        with mp.workprec(300):
            g = [[mp.fsum(mp.mpf(u) * mp.mpf(w) for u, w in zip(x[i], x[j])) for j in range(n)]
                 for i in range(n)]
            scores = {}
            for i in range(n):
                for j in range(i + 1, n):
                    up, _, A, B = shifts_2x2(g[i][i], g[j][j], g[i][j])
                    scores[(i, j)] = up * (1 / A + 1 / B) if pivot == O.RELATIVE else up
            top = max(scores.values())
        assert scores[(int(p), int(q))] >= top * (1 - 1e-9), (p, q)
        xp, xq = x[p].copy(), x[q].copy()
        x[p] = c * xp + s * xq
        x[q] = c * xq - s * xp


def test_preconditioning_cuts_rotations():
    # Sec. 2.1: B V has columns orthogonal to O(u_32), so far fewer FP64 rotations remain
    b = I.svd_graded(80, 60, seed=21, decades=4.0)
    plain = O.svd(b, U, pivot=O.GAP)
    pre = O.svd(b, U, pivot=O.GAP, precond="fp32", passes=1)
    assert pre.status == O.OK and plain.status == O.OK
    assert pre.rotations < plain.rotations / 3
    check_factorisation(b, pre, 50 * 80 * U)


def test_edge_cases():
    b = np.arange(1.0, 6.0)[:, None]
    r = O.svd(b, U)
    assert r.rotations == 0 and r.s[0] == np.sqrt(np.sum(b * b))
    assert np.array_equal(r.v, [[1.0]])
    z = I.svd_graded(10, 4, seed=1)
    z[:, 2] = 0.0
    r = O.svd(z, U, pivot=O.RELATIVE)
    assert r.status == O.OK and r.s[-1] == 0.0 and np.all(r.u[:, -1] == 0.0)
    nan = z.copy()
    nan[3, 1] = np.nan
    assert O.svd(nan, U).status == O.NONFINITE


# ----------------------------------------------------------------- Sec. 4.2: Hilbert
def test_hilbert_reference_trace_and_determinant():
    # sum sigma^2 = trace(H_n) = sum 1/(2i-1); prod sigma^2 = det(H_n) = c_n^4 / c_2n with
    # c_n = prod_{i<n} i! (Cauchy determinant)
    for n in (20, 40, 100):
        with mp.workdps(60):
            sv = [mp.mpf(x) for x in golden()["sv"][str(n)]]
            tr = mp.fsum(mp.mpf(1) / (2 * i - 1) for i in range(1, n + 1))
            assert abs(mp.fsum(s * s for s in sv) - tr) <= mp.mpf(10) ** -27 * tr
            cn = mp.mpf(math.prod(math.factorial(i) for i in range(1, n)))
            c2n = mp.mpf(math.prod(math.factorial(i) for i in range(1, 2 * n)))
            det = cn ** 4 / c2n
            prod = mp.fprod(s * s for s in sv)
            assert abs(prod / det - 1) <= mp.mpf(10) ** -25


def test_hilbert_cholesky_closed_form():
    # the closed form of Sec. 4.2 is the Cholesky factor: C C^T = H exactly (rational
    # arithmetic), and the float64 generator rounds each entry three times (<= 3u relative)
    n = 12
    f = math.factorial
    c = [[Fraction(0)] * n for _ in range(n)]
    for i in range(1, n + 1):
        for j in range(1, i + 1):
            c[i - 1][j - 1] = Fraction(f(i - 1) ** 2, f(i + j - 1) * f(i - j))  # / sqrt(2j-1)
    for i in range(n):
        for k in range(n):
            s = sum(c[i][j] * c[k][j] * (2 * j + 1) for j in range(n))
            assert s == Fraction(1, i + k + 1)
    g = I.hilbert_cholesky(40)
    with mp.workdps(50):
        for i in range(40):
            for j in range(i + 1):
                ex = mp.sqrt(2 * j + 1) * mp.mpf(f(i) ** 2) / (mp.mpf(f(i + j + 1)) * f(i - j))
                assert abs(mp.mpf(g[i, j]) - ex) <= 3.001 * U * ex  # three roundings


def test_hilbert_relative_score_accurate_where_gap_is_not():
    # Sec. 4.2: absolute pivot rules leave the tiny singular values of C_n inaccurate; the
    # relative score reaches them
    ref = ref_sv(20)
    c = I.hilbert_cholesky(20)
    rel = O.svd(c, U, pivot=O.RELATIVE)
    gap = O.svd(c, U, pivot=O.GAP)
    assert rel.status == gap.status == O.OK
    assert np.max(np.abs(rel.s - ref) / ref) <= 1e-11
    assert np.max(np.abs(gap.s - ref) / ref) >= 1e-3


def test_hilbert_c100_rotation_count_and_tail():
    # Sec. 4.2: with the relative score the method converges after about 1e5 rotations; the
    # smallest singular values are far closer to the reference than under the gap score
    ref = ref_sv(100)
    c = I.hilbert_cholesky(100)
    rel = O.svd(c, U, pivot=O.RELATIVE, maxrot=400000, logcap=400000)
    assert rel.status == O.OK
    assert 5e4 <= rel.rotations <= 2e5
    g = golden()["c100_relative"]
    assert rel.rotations == g["rotations"]
    assert hashlib.sha256(np.ascontiguousarray(rel.pivots, dtype=np.int32).tobytes()
                          ).hexdigest() == g["pivots_sha256"]
    assert hashlib.sha256(np.ascontiguousarray(rel.s).tobytes()).hexdigest() == g["sv_sha256"]
    gap = O.svd(c, U, pivot=O.GAP)
    e_rel = np.log10(np.abs(rel.s - ref) / ref + 1e-17)
    e_gap = np.log10(np.abs(gap.s - ref) / ref + 1e-17)
    assert np.median(e_rel[50:]) < np.median(e_gap[50:]) - 10
    assert np.max(np.abs(rel.s[:10] - ref[:10]) / ref[:10]) <= 1e-13
