"""Eigenvector and large-n parity of the HIP path (through the C ABI) with the CPU oracle.

Algorithm 1 with eq. (1) and the rotation of Sec. 2 fix every floating-point operation of
the FP64 phase, and Sec. 2.1 defines the eigenvectors as the preconditioner times the
accumulated rotations.  Without the preconditioner (V_J starts at I) and without the
polish, both sides therefore perform the same IEEE operations in the same order:

* V must equal the oracle's column-permuted V_J bit for bit, and W its sorted diagonal,
  for every kernel variant (LDS-resident, HBM-resident with 1, 2, 4 and 8 rows per
  thread, 512 and 1024 threads), single and batched, across rotation-log drains;
* at n = 1500 (512 threads x 4 rows), 4096 (512 x 8) and 6000 (1024 x 8) the pivot
  sequence and the diagonal bytes after a common rotation cap equal the oracle's, and at
  n = 2048 to 7800 (every layout of the log drain) so does V.

Large cases stop both sides at the same rotation cap (status MAXROT), which keeps the
oracle's cost to seconds while every rotation is still compared.
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def cert_thr(lam_max, n):
    return 10 * n * U * lam_max / (2.0 * n * (n - 1))


def oracle_sorted(a, pivot, thr, maxrot=None, want_vj=True):
    """The oracle's FP64 phase on the same bytes: sorted diagonal, V_J's columns permuted
    to match (stable ascending order, as the library sorts)."""
    ref = O.jacobi(a, pivot=pivot, stop=O.STOP_CERT, thr=thr, maxrot=maxrot, scan=1,
                   want_vj=want_vj, logcap=maxrot)
    d = np.diag(ref.a).copy()
    order = np.argsort(d, kind="stable")
    v = np.ascontiguousarray(ref.vj[:, order]) if want_vj else None
    return ref, d[order], v


def dense_case(n):
    p = I.clustered(n, seed=5000 + n, size=4, offset=1e-9)
    return p.a, float(np.max(np.abs(p.lam)))


def nearly_diag_case(n):
    p = I.nearly_diagonal(n, 5100 + n, 1e-7, spectrum="clusters")
    return p.a, 2.0


@pytest.mark.parametrize("n", [17, 64, 129])
@pytest.mark.parametrize("pivot", [J.GREEDY, J.GAP])
def test_eigenvectors_bitwise_full_solve(n, pivot):
    a, lam2 = dense_case(n)
    thr = cert_thr(lam2, n)
    say("V parity full", n, pivot)
    r = J.eigh(gpu(a), precond="none", pivot=pivot, stop="cert", abs_thr=thr, polish_v=False)
    ref, w, v = oracle_sorted(a, pivot, thr)
    assert r.status == J.OK and ref.status == O.OK
    assert r.stats["rotations"] == ref.rotations
    assert np.array_equal(r.w.cpu().numpy(), w)
    assert np.array_equal(r.v.cpu().numpy(), v)


@pytest.mark.parametrize("n,pivot,cap", [(520, J.GAP, None), (520, J.GREEDY, 20000),
                                         (1024, J.GAP, 20000), (1024, J.GREEDY, 20000)])
def test_eigenvectors_bitwise_nearly_diagonal(n, pivot, cap):
    """The input shape the preconditioner leaves; a full solve at n = 520 (gap), the first
    20000 rotations otherwise."""
    a, lam2 = nearly_diag_case(n)
    thr = cert_thr(lam2, n)
    say("V parity nearly diagonal", n, pivot, cap)
    r = J.eigh(gpu(a), precond="none", pivot=pivot, stop="cert", abs_thr=thr, polish_v=False,
               max_rotations=cap or 0)
    ref, w, v = oracle_sorted(a, pivot, thr, maxrot=cap)
    assert r.stats["rotations"] == ref.rotations
    assert r.status == (J.WARN_MAXROT if cap else J.OK)
    assert np.array_equal(r.w.cpu().numpy(), w)
    assert np.array_equal(r.v.cpu().numpy(), v)


@pytest.mark.parametrize("pivot", ["greedy", "gap"])
def test_batched_eigenvectors_bitwise_across_log_drains(pivot):
    """Batched solves without the preconditioner: W and V equal the oracle's bit for bit.
    The 520-row member needs more rotations than one batched log holds (2^16), so its V is
    assembled over several drains."""
    sizes = [3, 40, 100, 129, 520]
    cases = [dense_case(n) if n < 520 else nearly_diag_case(n) for n in sizes]
    mats = [gpu(a) for a, _ in cases]
    # one absolute threshold for the batch, as the oracle takes it
    thr = min(cert_thr(l2, a.shape[0]) for a, l2 in cases)
    say("batched V parity", pivot, sizes)
    status, res = J.eigh_batched(mats, tol=1.0, pivot=pivot, precond="none", polish_v=False,
                                 abs_thr=thr)
    assert status == J.OK
    for (a, _), r in zip(cases, res):
        piv = J.GREEDY if pivot == "greedy" else J.GAP
        ref, w, v = oracle_sorted(a, piv, thr)
        assert r.stats["rotations"] == ref.rotations, a.shape[0]
        assert np.array_equal(r.w.cpu().numpy(), w), a.shape[0]
        assert np.array_equal(r.v.cpu().numpy(), v), a.shape[0]


@pytest.mark.parametrize("n,pivot", [(1500, J.GAP), (1500, J.GREEDY), (4096, J.GAP),
                                     (6000, J.GAP)])
def test_large_n_pivot_sequence_matches_oracle(n, pivot):
    """Kernel variants beyond n = 1024: 512 threads x 4 rows (n <= 2048), 512 x 8
    (n <= 4096) and 1024 x 8 (n <= 8192).  The first 20000 rotations of a dense random
    symmetric matrix: identical pivot log and diagonal bytes."""
    cap = 20000
    a = I.random_symmetric(n, seed=6000 + n)
    say("large-n parity", n, pivot)
    r = J.eigh(gpu(a), precond="none", pivot=pivot, stop="cert", abs_thr=1e-300,
               max_rotations=cap, pivot_log_cap=cap, want_v=False)
    ref = O.jacobi(a, pivot=pivot, stop=O.STOP_CERT, thr=1e-300, maxrot=cap, scan=1,
                   want_vj=False, logcap=cap)
    assert r.status == J.WARN_MAXROT and ref.status == O.MAXROT
    assert r.stats["rotations"] == ref.rotations == cap
    assert np.array_equal(r.pivots.cpu().numpy(), ref.pivots)
    assert np.array_equal(r.w.cpu().numpy(), np.sort(np.diag(ref.a)))


@pytest.mark.parametrize("sizes", [[1500, 300], [4100, 64]])
def test_batched_large_members_match_oracle(sizes):
    """The batched persistent launch for members above n = 1024 (512 x 4 up to 2048,
    1024 x 8 above 4096): every row of a large member is owned by a thread, so the
    diagonal after a common rotation cap equals the oracle's bit for bit."""
    cap = 6000
    mats_np = [I.random_symmetric(n, seed=6500 + n) for n in sizes]
    say("batched large members", sizes)
    status, res = J.eigh_batched([gpu(a) for a in mats_np], tol=1.0, pivot="gap",
                                 precond="none", abs_thr=1e-300, max_rotations=cap,
                                 want_v=False)
    assert status == J.WARN_MAXROT
    for a, r in zip(mats_np, res):
        ref = O.jacobi(a, pivot=O.GAP, stop=O.STOP_CERT, thr=1e-300, maxrot=cap, scan=1,
                       want_vj=False, logcap=cap)
        assert r.status == J.WARN_MAXROT
        assert r.stats["rotations"] == ref.rotations == cap
        assert np.array_equal(r.w.cpu().numpy(), np.sort(np.diag(ref.a))), a.shape[0]


@pytest.mark.parametrize("n,batched", [(2048, False), (4100, False), (7800, False),
                                       (2100, True)])
def test_large_n_eigenvectors_bitwise(n, batched):
    """The log drain's layouts beyond n = 1024: 3 rows of V per wave in 21 lane groups
    (n = 2048, 2100), one row in 32 lane groups (n = 4100), one row and one rotation per
    step (n = 7800, where the row alone fills the LDS).  The first 5000 rotations of a
    dense random symmetric matrix, single and batched: V equals the oracle's V_J bit for
    bit (columns in the sorted order of the diagonal)."""
    cap = 5000
    a = I.random_symmetric(n, seed=6700 + n)
    say("large-n V parity", n, "batched" if batched else "single")
    if batched:
        small = I.random_symmetric(300, seed=6701)
        st, res = J.eigh_batched([gpu(a), gpu(small)], tol=1.0, pivot="gap", precond="none",
                                 polish_v=False, abs_thr=1e-300, max_rotations=cap)
        r = res[0]
    else:
        r = J.eigh(gpu(a), precond="none", pivot=J.GAP, stop="cert", abs_thr=1e-300,
                   polish_v=False, max_rotations=cap)
    ref, w, v = oracle_sorted(a, J.GAP, 1e-300, maxrot=cap)
    assert r.status == J.WARN_MAXROT and ref.status == O.MAXROT
    assert r.stats["rotations"] == ref.rotations == cap
    assert np.array_equal(r.w.cpu().numpy(), w)
    assert np.array_equal(r.v.cpu().numpy(), v)


def test_device_array_batched_form_equals_host_form():
    """jacobi_eigh_batched (pointer, size and status arrays in device memory) gives the same
    bits and statuses as the host-array form."""
    sizes = [5, 64, 130, 257]
    cases = [dense_case(n) for n in sizes]
    mats = [gpu(a) for a, _ in cases]
    tol = 1e-13
    st_h, rh = J.eigh_batched(mats, tol=tol, pivot="gap", precond="fp32")
    st_d, rd = J.eigh_batched_device(mats, tol=tol, pivot="gap", precond="fp32")
    assert st_h == st_d == J.OK
    for x, (w, v, info) in zip(rh, rd):
        assert info == J.OK
        assert torch.equal(x.w, w)
        assert torch.equal(x.v, v)


@pytest.mark.parametrize("e", [600, -600, 130, -130])
def test_out_of_range_inputs_are_scaled_exactly(e):
    """Entries far outside the FP32 range (or whose squares leave FP64's): the library
    solves 2^k A for the k that brings max |a_ij| into [1/2, 1) and scales W back, so the
    result is 2^e times the result on A -- the same bits, by the scale invariance of
    eq. (1), the rotation and Theorem 1's threshold -- and matches the oracle on A."""
    n = 150
    a, lam2 = dense_case(n)
    a = a / np.max(np.abs(a)) * 0.75  # max |a_ij| in [1/2, 1): solved as given
    lam = np.linalg.eigvalsh(a)
    lam2 = float(np.max(np.abs(lam)))
    thr = cert_thr(lam2, n)
    say("scaled input", e)
    r0 = J.eigh(gpu(a), pivot="gap", precond="none", polish_v=False, abs_thr=thr)
    r1 = J.eigh(gpu(np.ldexp(a, e)), pivot="gap", precond="none", polish_v=False,
                abs_thr=np.ldexp(thr, e))
    assert r0.status == r1.status == J.OK
    assert r0.stats["scale_exp"] == 0 and r1.stats["scale_exp"] == -e
    assert r1.stats["rotations"] == r0.stats["rotations"]
    assert np.array_equal(r1.w.cpu().numpy(), np.ldexp(r0.w.cpu().numpy(), e))
    assert torch.equal(r1.v, r0.v)
    ref, w, v = oracle_sorted(a, O.GAP, thr)
    assert np.array_equal(r0.w.cpu().numpy(), w)
    assert np.array_equal(r0.v.cpu().numpy(), v)
    # the preconditioned path on the scaled input: FP64-accurate against the spectrum
    tol = 10 * n * U * lam2 / np.linalg.norm(a)
    rp = J.eigh(gpu(np.ldexp(a, e)), tol=tol, pivot="gap", precond="fp32")
    assert rp.status == J.OK
    assert np.max(np.abs(np.ldexp(rp.w.cpu().numpy(), -e) - lam)) <= 10 * n * U * lam2
    # batched members are scaled one by one (relative tolerance: each member's threshold
    # follows its own norm)
    st, rb = J.eigh_batched([gpu(np.ldexp(a, e)), gpu(a)], tol=tol, pivot="gap",
                            precond="none", polish_v=False)
    assert st == J.OK
    assert rb[0].stats["scale_exp"] == -e and rb[1].stats["scale_exp"] == 0
    assert rb[0].stats["rotations"] == rb[1].stats["rotations"]
    assert np.array_equal(rb[0].w.cpu().numpy(), np.ldexp(rb[1].w.cpu().numpy(), e))
    assert torch.equal(rb[0].v, rb[1].v)


def test_unsorted_output_keeps_diagonal_order():
    """opts.sort = 0: W in the order of the final diagonal and V unpermuted."""
    n = 64
    a, lam2 = dense_case(n)
    thr = cert_thr(lam2, n)
    r = J.eigh(gpu(a), precond="none", pivot="gap", abs_thr=thr, polish_v=False, sort=False)
    ref = O.jacobi(a, pivot=O.GAP, stop=O.STOP_CERT, thr=thr, scan=1, want_vj=True)
    assert np.array_equal(r.w.cpu().numpy(), np.diag(ref.a))
    assert np.array_equal(r.v.cpu().numpy(), ref.vj)


@pytest.mark.parametrize("n,pivot", [(512, J.GAP), (700, J.GREEDY), (1024, J.GAP),
                                     (2049, J.GAP), (4097, J.GREEDY)])
def test_multi_workgroup_kernel_equals_one_workgroup(n, pivot):
    """The FP64 phase on several workgroups (one wave each, candidates exchanged through L2
    every rotation) performs the same arithmetic as the one-workgroup kernel: same pivots,
    rotation count, diagonal and eigenvectors, for 1, 2 and 4 rows per thread, with row
    rescans."""
    cap = 3000
    a = I.random_symmetric(n, seed=7000 + n)
    say("multi-workgroup vs one", n, pivot)
    kw = dict(precond="none", pivot=pivot, stop="cert", abs_thr=1e-300, max_rotations=cap,
              pivot_log_cap=cap, polish_v=False)
    r1 = J.eigh(gpu(a), jacobi_wgs="one", **kw)
    rm = J.eigh(gpu(a), jacobi_wgs="many", **kw)
    assert r1.stats["jacobi_wgs"] == 1 and rm.stats["jacobi_wgs"] > 1
    assert r1.status == rm.status == J.WARN_MAXROT
    assert rm.stats["rotations"] == r1.stats["rotations"] == cap
    # (the rescan counts may differ: a stale row's cached bound is widened by one float ulp
    # per reduction level and the two kernels group the maximum differently; a rescan only
    # makes a row exact, so the pivots do not depend on it)
    assert torch.equal(rm.pivots, r1.pivots)
    assert torch.equal(rm.w, r1.w)
    assert torch.equal(rm.v, r1.v)


@pytest.mark.parametrize("stop", ["cert", "score", "off"])
def test_multi_workgroup_full_solve_matches_oracle(stop):
    """A whole FP64 phase on several workgroups against the oracle (n = 600, nearly diagonal
    input, both pivot rules through the certificate stop with greedy's L cache): pivots,
    rotation count and bits of W and V.  The off-norm stop sums its per-row parts in another
    order than the oracle, so there the pivots agree up to the common length."""
    n = 600
    a, lam2 = nearly_diag_case(n)
    for pivot in (J.GAP, J.GREEDY):
        thr = cert_thr(lam2, n) if stop == "cert" else 1e-13
        say("multi-workgroup full", stop, pivot)
        cap = 40 * n * n
        r = J.eigh(gpu(a), precond="none", pivot=pivot, stop=stop, abs_thr=thr, polish_v=False,
                   pivot_log_cap=cap, jacobi_wgs="many")
        so = {"cert": O.STOP_CERT, "off": O.STOP_OFF, "score": O.STOP_SCORE}[stop]
        ref = O.jacobi(a, pivot=pivot, stop=so, thr=thr, scan=1, want_vj=True)
        assert r.status == J.OK and r.stats["jacobi_wgs"] > 1
        piv = r.pivots.cpu().numpy()
        if stop == "off":
            m = min(len(piv), len(ref.pivots))
            assert abs(len(piv) - len(ref.pivots)) <= 1
            assert np.array_equal(piv[:m], ref.pivots[:m])
            continue
        assert r.stats["rotations"] == ref.rotations
        assert np.array_equal(piv, ref.pivots)
        d = np.diag(ref.a).copy()
        order = np.argsort(d, kind="stable")
        assert np.array_equal(r.w.cpu().numpy(), d[order])
        assert np.array_equal(r.v.cpu().numpy(), ref.vj[:, order])
