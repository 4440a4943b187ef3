"""CPU-side checks of the C ABI: the library loads, exports every function that
include/jacobi.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2607_23187_amd import jacobi as J

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jacobi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_header_declares_the_expected_entry_points():
    assert declared_functions() == sorted(J.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = J.load()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_defaults_and_strings():
    o = J.default_opts()
    assert (o.stop, o.polish_v, o.fp32_max_sweeps, o.fp32_passes, o.max_rotations, o.abs_thr,
            o.split_gemm) == (0, 1, 20, 2, 0, 0.0, 0)
    assert (o.sort, o.update_mode, o.tune, o.graph, o.profile, o.fp32_block,
            o.jacobi_wgs, o.batch_threads) == (1, 0, 1, 0, 0, 0, 0, 0)
    assert J.strerror(0) == "ok"
    assert "NaN" in J.strerror(J.ERR_NONFINITE)
    assert J.strerror(-3) == "invalid argument"
    assert J.workspace_size(0) == 0 and J.workspace_size(1) == 0
    assert J.workspace_size(1024, "fp32") > J.workspace_size(1024, "none") > 8 * 1024 * 1024


def _ex(A, n, lda, W, V, ldv, tol, pivot=1, precond=1, opts=None):
    L = J.load()
    return L.jacobi_eigh_ex(A, n, lda, W, V, ldv, tol, pivot, precond,
                            ctypes.byref(opts) if opts is not None else None, None, None)


def test_argument_errors_follow_lapack_info_convention():
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert _ex(None, 4, 4, fake, None, 4, 1e-12) == -1
    assert _ex(fake, -1, 4, fake, None, 4, 1e-12) == -2
    assert _ex(fake, 4, 3, fake, None, 4, 1e-12) == -3
    assert _ex(fake, 4, 4, None, None, 4, 1e-12) == -4
    assert _ex(fake, 4, 4, fake, fake, 2, 1e-12) == -6
    assert _ex(fake, 4, 4, fake, None, 4, 0.0) == -7
    assert _ex(fake, 4, 4, fake, None, 4, float("nan")) == -7
    assert _ex(fake, 4, 4, fake, None, 4, 1e-12, pivot=7) == -8
    assert _ex(fake, 4, 4, fake, None, 4, 1e-12, precond=5) == -9
    for field, bad in (("stop", 9), ("sort", 2), ("update_mode", 3), ("tune", -1),
                       ("graph", 2), ("profile", 5), ("fp32_block", 24), ("fp32_passes", 3),
                       ("jacobi_wgs", 3), ("batch_threads", 64)):
        o = J.default_opts()
        setattr(o, field, bad)
        assert _ex(fake, 4, 4, fake, None, 4, 1e-12, opts=o) == -10, field
    # n = 0 is a no-op that needs no device
    assert _ex(fake, 0, 1, fake, None, 1, 1e-12) == 0
    # too large
    assert _ex(fake, J.MAX_N + 1, J.MAX_N + 1, fake, None, J.MAX_N + 1, 1e-12) == J.ERR_TOO_LARGE
    L = J.load()
    assert L.jacobi_eigh_batched(-1, None, None, None, None, None, 1e-12, 1, 1, None,
                                 None, None) == -1
    assert L.jacobi_eigh_batched(0, None, None, None, None, None, 1e-12, 1, 1, None,
                                 None, None) == 0
    assert L.jacobi_eigh_batched(2, None, fake, fake, fake, None, 1e-12, 1, 1, None,
                                 fake, None) == -2
    assert L.jacobi_eigh_batched(2, fake, fake, fake, fake, None, 1e-12, 1, 1, None,
                                 None, None) == -11
    assert L.jacobi_eigh_batched_host(-1, None, None, None, None, None, None, 1e-12, 1, 1,
                                      None, None, None, None) == -1


def test_batched_host_form_argument_numbers():
    """The host-array batched form numbers its arguments A = 2 ... opts = 11 and rejects the
    whole batch before any device work."""
    L = J.load()
    VP, IA = ctypes.c_void_p * 2, ctypes.c_int * 2
    fake = 0x1000
    a, w = VP(fake, fake), VP(fake, fake)
    n, lda, info = IA(4, 4), IA(4, 4), IA(0, 0)

    def call(a=a, n=n, lda=lda, w=w, v=None, ldv=None, tol=1e-12, pivot=1, precond=1, opts=None):
        return L.jacobi_eigh_batched_host(2, a, n, lda, w, v, ldv, tol, pivot, precond,
                                          ctypes.byref(opts) if opts is not None else None,
                                          info, None, None)

    assert call(a=VP(fake, None)) == -2 and info[1] == -2
    assert call(n=IA(4, -3)) == -3
    assert call(lda=IA(4, 2)) == -4
    assert call(w=VP(None, fake)) == -5
    assert call(v=VP(fake, fake), ldv=IA(4, 3)) == -7
    assert call(tol=-1.0) == -8
    assert call(pivot=5) == -9
    assert call(precond=4) == -10
    o = J.default_opts()
    o.update_mode = 7
    assert call(opts=o) == -11
    assert call(n=IA(4, J.MAX_N + 1), lda=IA(4, J.MAX_N + 1)) == J.ERR_TOO_LARGE


def test_server_rejects_bad_arguments():
    """Argument checks of jacobi_server_create run before any device call."""
    L = J.load()
    o = J.default_opts()
    assert not L.jacobi_server_create(0, 1 << 20, 1e-12, 1, 1, ctypes.byref(o))
    assert not L.jacobi_server_create(2, 1 << 20, 1e-12, 7, 1, ctypes.byref(o))
    assert not L.jacobi_server_create(2, 1 << 20, -1.0, 1, 1, ctypes.byref(o))
    assert L.jacobi_server_poll(None, None, 0, 0) == -1
    assert L.jacobi_server_pending(None) == -1


def test_svd_argument_errors():
    """jacobi_svd validates its arguments before any device call."""
    L = J.load()
    fake = ctypes.c_void_p(0x1000)

    def svd(B, m, n, ldb, S, Up, ldu, V, ldv, tol, pivot=1, precond=0, opts=None):
        return L.jacobi_svd(B, m, n, ldb, S, Up, ldu, V, ldv, tol, pivot, precond,
                            ctypes.byref(opts) if opts is not None else None, None, None)

    assert svd(None, 5, 4, 5, fake, None, 5, None, 4, 1e-12) == -1
    assert svd(fake, 3, 4, 5, fake, None, 5, None, 4, 1e-12) == -2      # m < n
    assert svd(fake, 5, -1, 5, fake, None, 5, None, 4, 1e-12) == -3
    assert svd(fake, 5, 4, 4, fake, None, 5, None, 4, 1e-12) == -4
    assert svd(fake, 5, 4, 5, None, None, 5, None, 4, 1e-12) == -5
    assert svd(fake, 5, 4, 5, fake, fake, 4, None, 4, 1e-12) == -7
    assert svd(fake, 5, 4, 5, fake, None, 5, fake, 3, 1e-12) == -9
    assert svd(fake, 5, 4, 5, fake, None, 5, None, 4, 0.0) == -10
    assert svd(fake, 5, 4, 5, fake, None, 5, None, 4, 1e-12, pivot=3) == -11
    assert svd(fake, 5, 4, 5, fake, None, 5, None, 4, 1e-12, precond=2) == -12
    o = J.default_opts()
    o.fp32_passes = 3
    assert svd(fake, 5, 4, 5, fake, None, 5, None, 4, 1e-12, opts=o) == -13
    assert svd(fake, 5, 0, 5, fake, None, 5, None, 1, 1e-12) == 0
    big = J.MAX_N + 1
    assert svd(fake, big, big, big, fake, None, big, None, big, 1e-12) == J.ERR_TOO_LARGE
    # the relative score is defined for the Gram matrix of the SVD only
    assert _ex(fake, 4, 4, fake, None, 4, 1e-12, pivot=J.RELATIVE) == -8
