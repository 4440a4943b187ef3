"""ctypes binding of the C ABI in ``include/jacobi.h`` (argument marshalling only).

Device memory and streams come from torch; every step of the solve runs in the HIP
library.  There is no fallback: without the built library or without a GPU every call
raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjacobi.so")

GREEDY, GAP, RELATIVE = 0, 1, 2
PRECOND_NONE, PRECOND_FP32 = 0, 1
STOP_CERT, STOP_OFF, STOP_SCORE = 0, 1, 2
OK, WARN_MAXROT, WARN_STALL, ERR_NONFINITE, ERR_NOMEM, ERR_DEVICE, ERR_TOO_LARGE = range(7)
MAX_N = 8192
NOALLOC_MAX_N = 512

_PIVOTS = {"greedy": GREEDY, "gap": GAP, "relative": RELATIVE, GREEDY: GREEDY, GAP: GAP,
           RELATIVE: RELATIVE}
_PRECONDS = {"none": PRECOND_NONE, "fp32": PRECOND_FP32, None: PRECOND_NONE,
             PRECOND_NONE: PRECOND_NONE, PRECOND_FP32: PRECOND_FP32}
_STOPS = {"cert": STOP_CERT, "off": STOP_OFF, "score": STOP_SCORE,
          STOP_CERT: STOP_CERT, STOP_OFF: STOP_OFF, STOP_SCORE: STOP_SCORE}


class Opts(ctypes.Structure):
    _fields_ = [("stop", ctypes.c_int), ("polish_v", ctypes.c_int),
                ("fp32_max_sweeps", ctypes.c_int), ("fp32_passes", ctypes.c_int),
                ("max_rotations", ctypes.c_longlong),
                ("abs_thr", ctypes.c_double), ("pivot_log", ctypes.c_void_p),
                ("pivot_log_cap", ctypes.c_longlong), ("split_gemm", ctypes.c_int),
                ("sort", ctypes.c_int), ("update_mode", ctypes.c_int), ("tune", ctypes.c_int),
                ("graph", ctypes.c_int), ("profile", ctypes.c_int),
                ("fp32_block", ctypes.c_int), ("jacobi_wgs", ctypes.c_int),
                ("batch_threads", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("rotations", ctypes.c_longlong), ("rescans", ctypes.c_longlong),
                ("final_max_score", ctypes.c_double), ("final_off", ctypes.c_double),
                ("normF", ctypes.c_double), ("thr", ctypes.c_double),
                ("sweeps32", ctypes.c_int), ("status", ctypes.c_int),
                ("ms_precond", ctypes.c_float), ("ms_gemm", ctypes.c_float),
                ("ms_jacobi", ctypes.c_float), ("ms_finalize", ctypes.c_float),
                ("ms_jacobi_kernel", ctypes.c_float), ("a_hat_off", ctypes.c_double),
                ("prof_ns", ctypes.c_double * 6), ("ms_apply_log", ctypes.c_float),
                ("scale_exp", ctypes.c_int), ("jacobi_wgs", ctypes.c_int)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["prof_ns"] = list(self.prof_ns)
        return d


EXPORTS = ["je_opts_default", "jacobi_eigh", "jacobi_eigh_ex", "jacobi_eigh_batched",
           "jacobi_eigh_batched_host", "jacobi_eigh_noalloc", "jacobi_svd",
           "jacobi_workspace_size", "jacobi_strerror", "jacobi_release",
           "jacobi_server_create", "jacobi_server_submit", "jacobi_server_poll",
           "jacobi_server_pending", "jacobi_server_clock", "jacobi_server_destroy"]


class Done(ctypes.Structure):
    """Mirror of je_done (completion record of a served request)."""
    _fields_ = [("tag", ctypes.c_longlong), ("status", ctypes.c_int), ("n", ctypes.c_int),
                ("batch", ctypes.c_int), ("pad", ctypes.c_int), ("rotations", ctypes.c_longlong),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]

_lib = None


def load(path: str = LIB_PATH):
    """Load libjacobi.so and declare the C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2607_23187_amd.build`")
    L = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.je_opts_default.argtypes = [ctypes.POINTER(Opts)]
    L.je_opts_default.restype = None
    L.jacobi_eigh.argtypes = [vp, ip, ip, vp, vp, dp, ip, ip]
    L.jacobi_eigh.restype = ctypes.c_int
    L.jacobi_eigh_ex.argtypes = [vp, ip, ip, vp, vp, ip, dp, ip, ip, ctypes.POINTER(Opts),
                                 ctypes.POINTER(Stats), vp]
    L.jacobi_eigh_ex.restype = ctypes.c_int
    L.jacobi_eigh_noalloc.argtypes = L.jacobi_eigh_ex.argtypes
    L.jacobi_eigh_noalloc.restype = ctypes.c_int
    L.jacobi_eigh_batched.argtypes = [ip, vp, vp, vp, vp, vp, dp, ip, ip,
                                      ctypes.POINTER(Opts), vp, vp]
    L.jacobi_eigh_batched.restype = ctypes.c_int
    L.jacobi_eigh_batched_host.argtypes = [ip, ctypes.POINTER(vp), ctypes.POINTER(ip),
                                           ctypes.POINTER(ip), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), ctypes.POINTER(ip), dp, ip, ip,
                                           ctypes.POINTER(Opts), ctypes.POINTER(ip),
                                           ctypes.POINTER(Stats), vp]
    L.jacobi_eigh_batched_host.restype = ctypes.c_int
    L.jacobi_svd.argtypes = [vp, ip, ip, ip, vp, vp, ip, vp, ip, dp, ip, ip,
                             ctypes.POINTER(Opts), ctypes.POINTER(Stats), vp]
    L.jacobi_svd.restype = ctypes.c_int
    L.jacobi_workspace_size.argtypes = [ip, ip]
    L.jacobi_workspace_size.restype = ctypes.c_size_t
    L.jacobi_strerror.argtypes = [ip]
    L.jacobi_strerror.restype = ctypes.c_char_p
    L.jacobi_release.argtypes = []
    L.jacobi_release.restype = None
    L.jacobi_server_create.argtypes = [ip, ctypes.c_size_t, dp, ip, ip, ctypes.POINTER(Opts)]
    L.jacobi_server_create.restype = vp
    L.jacobi_server_submit.argtypes = [vp, vp, ip, ip, vp, vp, ip, ctypes.c_longlong]
    L.jacobi_server_submit.restype = ctypes.c_int
    L.jacobi_server_poll.argtypes = [vp, ctypes.POINTER(Done), ip, ip]
    L.jacobi_server_poll.restype = ctypes.c_int
    L.jacobi_server_pending.argtypes = [vp]
    L.jacobi_server_pending.restype = ctypes.c_longlong
    L.jacobi_server_clock.argtypes = [vp]
    L.jacobi_server_clock.restype = ctypes.c_double
    L.jacobi_server_destroy.argtypes = [vp]
    L.jacobi_server_destroy.restype = None
    _lib = L
    return L


def strerror(status: int) -> str:
    return load().jacobi_strerror(int(status)).decode()


def default_opts() -> Opts:
    o = Opts()
    load().je_opts_default(ctypes.byref(o))
    return o


@dataclass
class Result:
    w: torch.Tensor                  # (n,) ascending eigenvalues, float64, device
    v: torch.Tensor | None           # (n, n): v[:, k] is the eigenvector of w[k]
    status: int
    stats: dict
    pivots: torch.Tensor | None      # (rotations, 2) int32 pivot log, 0-based


def _check_device_tensor(a: torch.Tensor):
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise TypeError("A must be a torch CUDA (HIP) tensor")
    if a.dtype != torch.float64:
        raise TypeError("A must be float64")
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("A must be square")


_UPDATE_MODES = {"auto": 0, "mirror": 1, "timestamp": 2, 0: 0, 1: 1, 2: 2}


_WGS = {"auto": 0, "one": 1, "many": 2, 0: 0, 1: 1, 2: 2}


def _opts(stop="cert", polish_v=True, fp32_max_sweeps=20, fp32_passes=2, split_gemm=False,
          max_rotations=0, abs_thr=0.0, sort=True, update_mode="auto", tune=True, graph=False,
          profile=False, fp32_block=0, jacobi_wgs="auto", batch_threads=0) -> Opts:
    o = default_opts()
    o.stop = _STOPS[stop]
    o.polish_v = 1 if polish_v else 0
    o.fp32_max_sweeps = int(fp32_max_sweeps)
    o.fp32_passes = int(fp32_passes)
    o.split_gemm = int(split_gemm)
    o.max_rotations = int(max_rotations)
    o.abs_thr = float(abs_thr)
    o.sort = 1 if sort else 0
    o.update_mode = _UPDATE_MODES[update_mode]
    o.tune = 1 if tune else 0
    o.graph = 1 if graph else 0
    o.profile = 1 if profile else 0
    o.fp32_block = int(fp32_block)
    o.jacobi_wgs = _WGS[jacobi_wgs]
    o.batch_threads = int(batch_threads)
    return o


def eigh(a: torch.Tensor, tol: float = 1e-14, pivot="gap", precond="fp32", stop="cert",
         want_v: bool = True, abs_thr: float = 0.0, max_rotations: int = 0,
         polish_v: bool = True, fp32_max_sweeps: int = 20, fp32_passes: int = 2,
         pivot_log_cap: int = 0, split_gemm: bool = False, sort: bool = True,
         update_mode="auto", graph: bool = False, profile: bool = False, fp32_block: int = 0,
         jacobi_wgs="auto", stream: torch.cuda.Stream | None = None, check: bool = True,
         noalloc: bool = False) -> Result:
    """Eigen-decomposition of the symmetric float64 CUDA tensor ``a``.

    The library reads the upper triangle of ``a`` in column-major terms (``a[j, i]`` for
    i <= j of the row-major tensor); for a symmetric tensor this is the whole matrix.
    ``noalloc`` calls jacobi_eigh_noalloc (the library's fixed device workspace; the output
    tensors are still allocated here by torch).
    """
    _check_device_tensor(a)
    L = load()
    n = a.shape[0]
    a = a.contiguous()
    w = torch.empty(n, dtype=torch.float64, device=a.device)
    vt = torch.empty((n, n), dtype=torch.float64, device=a.device) if want_v else None
    o = _opts(stop, polish_v, fp32_max_sweeps, fp32_passes, split_gemm, max_rotations, abs_thr,
              sort, update_mode, True, graph, profile, fp32_block, jacobi_wgs)
    plog = None
    if pivot_log_cap > 0:
        plog = torch.full((pivot_log_cap, 2), -1, dtype=torch.int32, device=a.device)
        o.pivot_log = plog.data_ptr()
        o.pivot_log_cap = int(pivot_log_cap)
    st = Stats()
    s = stream if stream is not None else torch.cuda.current_stream(a.device)
    with torch.cuda.device(a.device):
        fn = L.jacobi_eigh_noalloc if noalloc else L.jacobi_eigh_ex
        status = fn(a.data_ptr(), n, max(1, n), w.data_ptr(),
                    vt.data_ptr() if vt is not None else None, max(1, n), float(tol),
                    _PIVOTS[pivot], _PRECONDS[precond], ctypes.byref(o), ctypes.byref(st),
                    ctypes.c_void_p(s.cuda_stream))
    if check and (status < 0 or status >= ERR_NONFINITE):
        raise RuntimeError(f"jacobi_eigh failed: {status} ({strerror(status)})")
    if plog is not None:
        plog = plog[: min(st.rotations, pivot_log_cap)]
    return Result(w, vt.t() if vt is not None else None, status, st.as_dict(), plog)


@dataclass
class SvdResult:
    s: torch.Tensor                  # (n,) singular values, descending, float64, device
    u: torch.Tensor | None           # (m, n)
    v: torch.Tensor | None           # (n, n): b @ v == u * s
    status: int
    stats: dict
    pivots: torch.Tensor | None      # (rotations, 2) int32 pivot log, 0-based


def svd(b: torch.Tensor, tol: float = 2.0 ** -53, pivot="gap", precond="none",
        want_u: bool = True, want_v: bool = True, abs_thr: float = 0.0, max_rotations: int = 0,
        fp32_max_sweeps: int = 20, fp32_passes: int = 2, pivot_log_cap: int = 0,
        stream: torch.cuda.Stream | None = None, check: bool = True) -> SvdResult:
    """One-sided Jacobi SVD (Algorithm 2) of the float64 CUDA tensor ``b`` (m x n, m >= n)."""
    if not isinstance(b, torch.Tensor) or not b.is_cuda:
        raise TypeError("B must be a torch CUDA (HIP) tensor")
    if b.dtype != torch.float64 or b.dim() != 2:
        raise TypeError("B must be a 2-D float64 tensor")
    L = load()
    m, n = b.shape
    bt = b.t().contiguous()          # column-major B, ldb = m
    sv = torch.empty(n, dtype=torch.float64, device=b.device)
    ut = torch.empty((n, m), dtype=torch.float64, device=b.device) if want_u else None
    vt = torch.empty((n, n), dtype=torch.float64, device=b.device) if want_v else None
    o = default_opts()
    o.fp32_max_sweeps = int(fp32_max_sweeps)
    o.fp32_passes = int(fp32_passes)
    o.max_rotations = int(max_rotations)
    o.abs_thr = float(abs_thr)
    plog = None
    if pivot_log_cap > 0:
        plog = torch.full((pivot_log_cap, 2), -1, dtype=torch.int32, device=b.device)
        o.pivot_log = plog.data_ptr()
        o.pivot_log_cap = int(pivot_log_cap)
    st = Stats()
    s = stream if stream is not None else torch.cuda.current_stream(b.device)
    with torch.cuda.device(b.device):
        status = L.jacobi_svd(bt.data_ptr(), m, n, max(1, m), sv.data_ptr(),
                              ut.data_ptr() if ut is not None else None, max(1, m),
                              vt.data_ptr() if vt is not None else None, max(1, n), float(tol),
                              _PIVOTS[pivot], _PRECONDS[precond], ctypes.byref(o),
                              ctypes.byref(st), ctypes.c_void_p(s.cuda_stream))
    if check and (status < 0 or status >= ERR_NONFINITE):
        raise RuntimeError(f"jacobi_svd failed: {status} ({strerror(status)})")
    if plog is not None:
        plog = plog[: min(st.rotations, pivot_log_cap)]
    return SvdResult(sv, ut.t() if ut is not None else None, vt.t() if vt is not None else None,
                     status, st.as_dict(), plog)


def eigh_batched(mats: list[torch.Tensor], tol: float = 1e-14, pivot="gap", precond="fp32",
                 stop="cert", want_v: bool = True, max_rotations: int = 0,
                 polish_v: bool = True, abs_thr: float = 0.0, sort: bool = True,
                 update_mode="auto", tune: bool = True, fp32_passes: int = 2,
                 graph: bool = False, fp32_block: int = 0, batch_threads: int = 0,
                 stream: torch.cuda.Stream | None = None):
    """Batch of independent problems of possibly different sizes (host-array form, with
    per-problem statistics).  ``graph`` replays the repeated step sequences from captured
    HIP graphs (same results)."""
    L = load()
    b = len(mats)
    for m in mats:
        _check_device_tensor(m)
    mats = [m.contiguous() for m in mats]
    ws = [torch.empty(m.shape[0], dtype=torch.float64, device=m.device) for m in mats]
    vs = [torch.empty_like(m) for m in mats] if want_v else None
    VP = ctypes.c_void_p * b
    IA = ctypes.c_int * b
    a_p = VP(*[m.data_ptr() for m in mats])
    w_p = VP(*[x.data_ptr() for x in ws])
    v_p = VP(*[x.data_ptr() for x in vs]) if vs is not None else None
    ns = IA(*[m.shape[0] for m in mats])
    info = IA()
    stats = (Stats * b)()
    o = _opts(stop, polish_v, 20, fp32_passes, False, max_rotations, abs_thr, sort,
              update_mode, tune, graph, fp32_block=fp32_block, batch_threads=batch_threads)
    s = stream if stream is not None else torch.cuda.current_stream()
    status = L.jacobi_eigh_batched_host(b, a_p, ns, ns, w_p, v_p, ns, float(tol),
                                        _PIVOTS[pivot], _PRECONDS[precond], ctypes.byref(o),
                                        info, stats, ctypes.c_void_p(s.cuda_stream))
    if status < 0:
        raise RuntimeError(f"jacobi_eigh_batched_host: argument {-status} invalid")
    out = []
    for i in range(b):
        out.append(Result(ws[i], vs[i].t() if vs is not None else None, int(info[i]),
                          stats[i].as_dict(), None))
    return status, out


def eigh_batched_device(mats: list[torch.Tensor], tol: float = 1e-14, pivot="gap",
                        precond="fp32", stop="cert", want_v: bool = True,
                        max_rotations: int = 0, stream: torch.cuda.Stream | None = None):
    """The same through the device-array form (jacobi_eigh_batched): pointer, size and
    status arrays live in device memory.  Returns (status, [(w, v, info)])."""
    L = load()
    b = len(mats)
    for m in mats:
        _check_device_tensor(m)
    mats = [m.contiguous() for m in mats]
    dev = mats[0].device
    ws = [torch.empty(m.shape[0], dtype=torch.float64, device=dev) for m in mats]
    vs = [torch.empty_like(m) for m in mats] if want_v else None
    a_p = torch.tensor([m.data_ptr() for m in mats], dtype=torch.int64, device=dev)
    w_p = torch.tensor([x.data_ptr() for x in ws], dtype=torch.int64, device=dev)
    v_p = (torch.tensor([x.data_ptr() for x in vs], dtype=torch.int64, device=dev)
           if vs is not None else None)
    ns = torch.tensor([m.shape[0] for m in mats], dtype=torch.int32, device=dev)
    info = torch.full((b,), -99, dtype=torch.int32, device=dev)
    o = _opts(stop, True, 20, 2, False, max_rotations)
    s = stream if stream is not None else torch.cuda.current_stream()
    torch.cuda.synchronize()
    status = L.jacobi_eigh_batched(b, a_p.data_ptr(), ns.data_ptr(), ns.data_ptr(),
                                   w_p.data_ptr(), v_p.data_ptr() if v_p is not None else None,
                                   float(tol), _PIVOTS[pivot], _PRECONDS[precond],
                                   ctypes.byref(o), info.data_ptr(),
                                   ctypes.c_void_p(s.cuda_stream))
    infos = info.cpu().tolist()
    return status, [(ws[i], vs[i].t() if vs is not None else None, infos[i]) for i in range(b)]


class Server:
    """Request server of the library (jacobi_server_*): submit(A, tag) queues a problem,
    poll() returns completion records.  Keeps each request's tensors alive until its record
    has been polled; the solve itself runs in the library's lane threads (continuous
    batching within an HBM budget)."""

    def __init__(self, workers: int = 2, hbm_budget: int = 1 << 30, tol: float = 1e-14,
                 pivot="gap", precond="fp32", stop="cert", want_v: bool = True,
                 polish_v: bool = True, graph: bool = False):
        L = load()
        o = _opts(stop, polish_v, graph=graph)
        self._want_v = want_v
        self._h = L.jacobi_server_create(int(workers), int(hbm_budget), float(tol),
                                         _PIVOTS[pivot], _PRECONDS[precond], ctypes.byref(o))
        if not self._h:
            raise RuntimeError("jacobi_server_create failed")
        self._live = {}

    def submit(self, a: torch.Tensor, tag: int):
        _check_device_tensor(a)
        a = a.contiguous()
        n = a.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=a.device)
        v = torch.empty_like(a) if self._want_v else None
        # A is written by the caller's stream and read by the server's lanes on their own
        # streams: wait for the caller's stream only (a device-wide synchronisation would
        # also wait for the solves in flight)
        torch.cuda.current_stream(a.device).synchronize()
        r = load().jacobi_server_submit(self._h, ctypes.c_void_p(a.data_ptr()), n, max(1, n),
                                        ctypes.c_void_p(w.data_ptr()),
                                        ctypes.c_void_p(v.data_ptr()) if v is not None else None,
                                        max(1, n), int(tag))
        if r != 0:
            raise RuntimeError(f"jacobi_server_submit: status {r}")
        self._live[int(tag)] = (a, w, v)

    def poll(self, wait: bool = False, max_records: int = 1024):
        buf = (Done * max_records)()
        k = load().jacobi_server_poll(self._h, buf, max_records, 1 if wait else 0)
        out = []
        for i in range(k):
            d = buf[i]
            a, w, v = self._live.pop(int(d.tag))
            out.append({"tag": int(d.tag), "status": int(d.status), "n": int(d.n),
                        "batch": int(d.batch), "rotations": int(d.rotations),
                        "t_submit": d.t_submit, "t_start": d.t_start, "t_done": d.t_done,
                        "w": w, "v": v.t() if v is not None else None})
        return out

    def pending(self) -> int:
        return int(load().jacobi_server_pending(self._h))

    def clock(self) -> float:
        return float(load().jacobi_server_clock(self._h))

    def close(self):
        if self._h:
            load().jacobi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size(n: int, precond="fp32") -> int:
    return int(load().jacobi_workspace_size(int(n), _PRECONDS[precond]))


def release():
    load().jacobi_release()
