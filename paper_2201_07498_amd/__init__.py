"""Python binding of liblanczos_topk.so, the gfx950 Top-K sparse symmetric
eigensolver (Lanczos with full reorthogonalisation + Jacobi + Ritz vectors).

Argument marshalling only: every step of the solve runs in the HIP library.
Device arrays are torch tensors on a ROCm device; streams are torch streams.
There is no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblanczos_topk.so")

LZ_FP64, LZ_FP32, LZ_BF16 = 0, 1, 2
PRECISION = {"fp64": LZ_FP64, "fp32": LZ_FP32, "bf16": LZ_BF16}
REORTH = {"none": 0, "once": 1, "twice": 2, "selective": 3}
REORDER = {"off": 0, "hubs": 1, "auto": 2}
ARITH = {"mixed": 0, "fp32": 1}
MAX_STEPS = 64
STATUS = {0: "LZ_OK", -1: "LZ_ERR_INVALID_ARG", -2: "LZ_ERR_OUT_OF_MEMORY", -3: "LZ_ERR_HIP",
          -4: "LZ_ERR_WORKSPACE_TOO_SMALL", -5: "LZ_ERR_TOO_LARGE", -6: "LZ_ERR_NOT_CONVERGED",
          -7: "LZ_ERR_NONFINITE", -8: "LZ_ERR_BREAKDOWN", -9: "LZ_ERR_RESTART_BUDGET", 1: "LZ_PENDING"}


class LanczosError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)}")


class Options(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("reorth", ctypes.c_int32), ("report", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("profile", ctypes.c_int32), ("reorder", ctypes.c_int32), ("arith", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("sweep", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("m_eff", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("jacobi_sweeps", ctypes.c_int32), ("beta_last", ctypes.c_double),
                ("resid", ctypes.c_double * MAX_STEPS), ("abs_resid", ctypes.c_double * MAX_STEPS),
                ("ortho_loss", ctypes.c_double), ("ritz_ortho_loss", ctypes.c_double),
                ("mean_angle_deg", ctypes.c_double), ("alpha", ctypes.c_double * MAX_STEPS),
                ("beta", ctypes.c_double * (MAX_STEPS + 1)), ("theta", ctypes.c_double * MAX_STEPS),
                ("t_setup_ms", ctypes.c_double), ("t_lanczos_ms", ctypes.c_double),
                ("t_spmv_ms", ctypes.c_double), ("t_orth_ms", ctypes.c_double),
                ("t_finish_ms", ctypes.c_double), ("reordered", ctypes.c_int32), ("spmv_layout", ctypes.c_int32),
                ("bytes_streamed", ctypes.c_int64)]

    def to_dict(self, K: int, m: int) -> dict:
        return dict(status=self.status, m_eff=self.m_eff, restarts=self.restarts,
                    jacobi_sweeps=self.jacobi_sweeps, beta_last=self.beta_last,
                    resid=np.array(self.resid[:K]), abs_resid=np.array(self.abs_resid[:K]),
                    ortho_loss=self.ortho_loss, ritz_ortho_loss=self.ritz_ortho_loss,
                    mean_angle_deg=self.mean_angle_deg, alpha=np.array(self.alpha[:m]),
                    beta=np.array(self.beta[:m + 1]), theta=np.array(self.theta[:m]),
                    t_setup_ms=self.t_setup_ms, t_lanczos_ms=self.t_lanczos_ms,
                    t_spmv_ms=self.t_spmv_ms, t_orth_ms=self.t_orth_ms, t_finish_ms=self.t_finish_ms,
                    reordered=bool(self.reordered), spmv_layout=int(self.spmv_layout),
                    bytes_streamed=int(self.bytes_streamed))


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        L.lz_options_init.restype = None
        L.lz_options_init.argtypes = [ctypes.POINTER(Options)]
        L.lz_status_string.restype = ctypes.c_char_p
        L.lz_status_string.argtypes = [ctypes.c_int]
        L.lanczos_topk.restype = ctypes.c_int
        L.lanczos_topk.argtypes = [P, P, P, i64, i32, i32, i32, P, P, P]
        L.lanczos_topk_workspace_size.restype = ctypes.c_size_t
        L.lanczos_topk_workspace_size.argtypes = [i64, i64, i32, i32, i32]
        L.lanczos_topk_workspace_size_opt.restype = ctypes.c_size_t
        L.lanczos_topk_workspace_size_opt.argtypes = [i64, i64, i32, i32, i32, ctypes.POINTER(Options)]
        L.lanczos_topk_ex.restype = ctypes.c_int
        L.lanczos_topk_ex.argtypes = [P, P, P, i64, i64, i32, i32, i32, P, P, P,
                                      ctypes.POINTER(Options), ctypes.POINTER(Report)]
        L.lanczos_topk_async.restype = ctypes.c_int
        L.lanczos_topk_async.argtypes = [P, P, P, i64, i64, i32, i32, i32, P, P, P, ctypes.POINTER(Options), P]
        L.lanczos_topk_noalloc.restype = ctypes.c_int
        L.lanczos_topk_noalloc.argtypes = [P, P, P, i64, i64, i32, i32, i32, P, P, P, ctypes.POINTER(Options), P]
        L.lanczos_topk_noalloc_max_bytes.restype = ctypes.c_size_t
        L.lanczos_topk_noalloc_max_bytes.argtypes = []
        L.lz_check_symmetric.restype = ctypes.c_int
        L.lz_check_symmetric.argtypes = [P, P, P, i64, i32, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]
        L.lanczos_topk_host.restype = ctypes.c_int
        L.lanczos_topk_host.argtypes = [P, P, P, i64, i32, i32, i32, i64, i64, P, P, P,
                                        ctypes.POINTER(Options), ctypes.POINTER(Report)]
        L.lanczos_topk_host_workspace_size.restype = ctypes.c_size_t
        L.lanczos_topk_host_workspace_size.argtypes = [i64, i64, i32, i32, i32]
        L.lz_spmv.restype = ctypes.c_int
        L.lz_spmv.argtypes = [P, P, P, i64, i64, i32, P, P, P]
        L.lz_ortho_loss.restype = ctypes.c_int
        L.lz_ortho_loss.argtypes = [P, i64, i64, i32, i32, P, ctypes.POINTER(ctypes.c_double)]
        L.lz_tridiag_eig.restype = ctypes.c_int
        L.lz_tridiag_eig.argtypes = [P, P, i32, P, P, ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


def _prec(precision) -> int:
    if isinstance(precision, str):
        return PRECISION[precision]
    return int(precision)


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_csr(rowptr, col, val, precision: int):
    import torch
    for t, dt, name in ((rowptr, torch.int64, "rowptr"), (col, torch.int32, "col")):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous {dt} device tensor")
    want = {LZ_FP64: torch.float64, LZ_FP32: torch.float32, LZ_BF16: torch.bfloat16}[precision]
    if not (val.is_cuda and val.dtype == want and val.is_contiguous()):
        raise TypeError(f"val must be a contiguous {want} device tensor")


def _check_outputs(out, workspace, K: int, n: int, dev):
    """The output and workspace tensors the library writes through raw
    pointers: contiguous float64 device tensors of the right size, and a
    device workspace, all on the matrix's device."""
    import torch
    if out is not None:
        vals, vecs = out
        for t, size, name in ((vals, K, "out[0]"), (vecs, K * n, "out[1]")):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device == dev and t.dtype == torch.float64
                    and t.is_contiguous() and t.numel() == size):
                raise TypeError(f"{name} must be a contiguous float64 tensor of {size} elements on {dev}")
    if workspace is not None:
        if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.device == dev
                and workspace.is_contiguous()):
            raise TypeError(f"workspace must be a contiguous tensor on {dev}")


def workspace_size(n: int, nnz: int, K: int, m: int, precision="fp64", sweep=None, reorder="auto") -> int:
    """Workspace bytes of a device-resident solve (default options, or the
    given sweep / reorder choice)."""
    if sweep is None and reorder == "auto":
        return int(lib().lanczos_topk_workspace_size(n, nnz, K, m, _prec(precision)))
    opt = _options(0, "twice", True, False, reorder, "mixed", None, sweep=sweep)
    return int(lib().lanczos_topk_workspace_size_opt(n, nnz, K, m, _prec(precision), ctypes.byref(opt)))


def topk(rowptr, col, val, K: int, m: int, precision="fp64", seed: int = 0, reorth="twice",
         report: bool = True, stream=None, workspace=None, nnz: int | None = None,
         profile: bool = False, out=None, reorder="auto", arith="mixed", sweep=None):
    """Top-K eigenpairs.  Returns (vals[K], vecs[n, K] view of the column-major
    output, report dict)."""
    import torch
    p = _prec(precision)
    _check_csr(rowptr, col, val, p)
    n = rowptr.numel() - 1
    if nnz is None:
        nnz = col.numel()
    dev = rowptr.device
    _check_outputs(out, workspace, K, n, dev)
    if out is None:
        vals = torch.empty(K, dtype=torch.float64, device=dev)
        vecs = torch.empty(K, n, dtype=torch.float64, device=dev)
    else:
        vals, vecs = out
    opt = _options(seed, reorth, report, profile, reorder, arith, workspace, sweep=sweep)
    rep = Report()
    rc = lib().lanczos_topk_ex(rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), n, nnz, K, m, p,
                               _stream_ptr(stream), vals.data_ptr(), vecs.data_ptr(),
                               ctypes.byref(opt), ctypes.byref(rep))
    if rc != 0:
        raise LanczosError(rc, "lanczos_topk_ex")
    return vals, vecs.T, rep.to_dict(K, m)


SWEEP = {None: -1, "auto": -1, False: 0, "off": 0, True: 1, "on": 1}


def _options(seed, reorth, report, profile, reorder, arith, workspace, max_restarts=-1, sweep=None) -> Options:
    opt = Options()
    lib().lz_options_init(ctypes.byref(opt))
    opt.seed = seed & (2 ** 64 - 1)
    opt.reorth = REORTH[reorth] if isinstance(reorth, str) else int(reorth)
    opt.report = 1 if report else 0
    opt.profile = 1 if profile else 0
    opt.reorder = REORDER[reorder] if isinstance(reorder, str) else int(reorder)
    opt.arith = ARITH[arith] if isinstance(arith, str) else int(arith)
    opt.max_restarts = int(max_restarts)
    opt.sweep = SWEEP[sweep] if (sweep is None or isinstance(sweep, (str, bool))) else int(sweep)
    if workspace is not None:
        opt.workspace = ctypes.c_void_p(workspace.data_ptr())
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
    return opt


REPORT_BYTES = ctypes.sizeof(Report)


def topk_async(rowptr, col, val, K: int, m: int, precision="fp64", seed: int = 0, reorth="twice",
               report: bool = True, stream=None, workspace=None, nnz: int | None = None, out=None,
               reorder="auto", arith="mixed", max_restarts: int = -1, d_report=None, sweep=None,
               _entry="lanczos_topk_async"):
    """Stream-ordered Top-K (lanczos_topk_async): enqueues the solve on
    `stream` and returns at once.  Returns (vals, vecs view, d_report), where
    d_report is a uint8 device tensor holding the lz_report (read it with
    report_from_device after the stream has finished)."""
    import torch
    p = _prec(precision)
    _check_csr(rowptr, col, val, p)
    n = rowptr.numel() - 1
    if nnz is None:
        nnz = col.numel()
    dev = rowptr.device
    _check_outputs(out, workspace, K, n, dev)
    if out is None:
        vals = torch.empty(K, dtype=torch.float64, device=dev)
        vecs = torch.empty(K, n, dtype=torch.float64, device=dev)
    else:
        vals, vecs = out
    if d_report is None:
        d_report = torch.empty(REPORT_BYTES, dtype=torch.uint8, device=dev)
    elif not (d_report.is_cuda and d_report.device == dev and d_report.dtype == torch.uint8
              and d_report.is_contiguous() and d_report.numel() >= REPORT_BYTES):
        raise TypeError(f"d_report must be a contiguous uint8 tensor of {REPORT_BYTES} bytes on {dev}")
    opt = _options(seed, reorth, report, False, reorder, arith, workspace, max_restarts, sweep)
    rc = getattr(lib(), _entry)(rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), n, nnz, K, m, p,
                                _stream_ptr(stream), vals.data_ptr(), vecs.data_ptr(), ctypes.byref(opt),
                                ctypes.c_void_p(d_report.data_ptr()))
    if rc != 0:
        raise LanczosError(rc, _entry)
    return vals, vecs.T, d_report


def topk_noalloc(rowptr, col, val, K: int, m: int, precision="fp64", **kw):
    """lanczos_topk_noalloc: topk_async with the library's fixed device
    scratch array as the workspace (no device allocation; calls overlapping
    on one device race).  Same arguments as topk_async except workspace."""
    if kw.get("workspace") is not None:
        raise TypeError("topk_noalloc takes no workspace")
    return topk_async(rowptr, col, val, K, m, precision, _entry="lanczos_topk_noalloc", **kw)


def noalloc_max_bytes() -> int:
    return int(lib().lanczos_topk_noalloc_max_bytes())


def report_from_device(d_report, K: int, m: int) -> dict:
    """Decodes an lz_report written to device memory (synchronises)."""
    raw = bytes(d_report[:REPORT_BYTES].cpu().numpy().tobytes())
    return Report.from_buffer_copy(raw).to_dict(K, m)


def check_symmetric(rowptr, col, val, precision="fp64", rtol: float = 0.0):
    """lz_check_symmetric on host numpy arrays (values in the storage type of
    `precision`, bf16 as uint16 bits).  Returns (symmetric, bad_row)."""
    p = _prec(precision)
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, {LZ_FP64: np.float64, LZ_FP32: np.float32, LZ_BF16: np.uint16}[p])
    bad = ctypes.c_int64(-1)
    rc = lib().lz_check_symmetric(rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, rowptr.size - 1, p,
                                  float(rtol), ctypes.byref(bad))
    if rc < 0:
        raise LanczosError(rc, "lz_check_symmetric")
    return rc == 1, int(bad.value)


def host_workspace_size(n: int, nnz: int, K: int, m: int, precision="fp64") -> int:
    return int(lib().lanczos_topk_host_workspace_size(n, nnz, K, m, _prec(precision)))


def topk_host(rowptr, col, val, K: int, m: int, precision="fp64", slab_nnz: int = 0, resident_nnz: int = 0,
              seed: int = 0, reorth="twice", report: bool = True, stream=None, workspace=None,
              profile: bool = False, out=None, arith="mixed", device="cuda:0"):
    """Top-K eigenpairs of a matrix whose entries stay in host memory
    (lanczos_topk_host).  rowptr: contiguous int64 CPU tensor; col, val:
    contiguous pinned CPU tensors (int32, and the storage dtype).  Results are
    device tensors as in topk()."""
    import torch
    p = _prec(precision)
    want = {LZ_FP64: torch.float64, LZ_FP32: torch.float32, LZ_BF16: torch.bfloat16}[p]
    for t, dt, name in ((rowptr, torch.int64, "rowptr"), (col, torch.int32, "col"), (val, want, "val")):
        if t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {dt} host tensor")
    n = rowptr.numel() - 1
    _check_outputs(out, workspace, K, n, torch.device(device))
    if out is None:
        vals = torch.empty(K, dtype=torch.float64, device=device)
        vecs = torch.empty(K, n, dtype=torch.float64, device=device)
    else:
        vals, vecs = out
    opt = _options(seed, reorth, report, profile, "off", arith, workspace)
    rep = Report()
    rc = lib().lanczos_topk_host(rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), n, K, m, p, slab_nnz,
                                 resident_nnz, _stream_ptr(stream), vals.data_ptr(), vecs.data_ptr(),
                                 ctypes.byref(opt), ctypes.byref(rep))
    if rc != 0:
        raise LanczosError(rc, "lanczos_topk_host")
    return vals, vecs.T, rep.to_dict(K, m)


def topk_plain(rowptr, col, val, K: int, m: int, precision="fp64", stream=None):
    """The minimal entry point lanczos_topk (default options, no report)."""
    import torch
    p = _prec(precision)
    _check_csr(rowptr, col, val, p)
    n = rowptr.numel() - 1
    vals = torch.empty(K, dtype=torch.float64, device=rowptr.device)
    vecs = torch.empty(K, n, dtype=torch.float64, device=rowptr.device)
    rc = lib().lanczos_topk(rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), n, K, m, p,
                            _stream_ptr(stream), vals.data_ptr(), vecs.data_ptr())
    if rc != 0:
        raise LanczosError(rc, "lanczos_topk")
    return vals, vecs.T


def spmv(rowptr, col, val, x, precision="fp64", stream=None):
    """y = A x with the solver's SpMV kernels (y is float64 for fp64, else float32)."""
    import torch
    p = _prec(precision)
    _check_csr(rowptr, col, val, p)
    n = rowptr.numel() - 1
    y = torch.empty(n, dtype=torch.float64 if p == LZ_FP64 else torch.float32, device=rowptr.device)
    rc = lib().lz_spmv(rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), n, col.numel(), p,
                       x.data_ptr(), y.data_ptr(), _stream_ptr(stream))
    if rc != 0:
        raise LanczosError(rc, "lz_spmv")
    return y


def tridiag_eig(alpha, offdiag):
    """Jacobi eigensolve of one symmetric tridiagonal matrix on the GPU."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    m = a.size
    o = np.ascontiguousarray(offdiag if m > 1 else np.zeros(1), dtype=np.float64)
    theta = np.zeros(m)
    S = np.zeros((m, m))
    sw = ctypes.c_int32(0)
    rc = lib().lz_tridiag_eig(a.ctypes.data, o.ctypes.data, m, theta.ctypes.data, S.ctypes.data,
                              ctypes.byref(sw))
    if rc != 0:
        raise LanczosError(rc, "lz_tridiag_eig")
    return theta, S, sw.value


def ortho_loss(X, precision="fp64", stream=None) -> float:
    """max |X^T X - I| of the columns of a device matrix X (n x c, column-major
    storage: pass the transpose view of a contiguous (c, n) tensor)."""
    import torch
    p = _prec(precision)
    n, c = X.shape
    if X.stride(0) != 1:
        raise TypeError("X must be column-major (stride 1 along rows)")
    out = ctypes.c_double(0.0)
    rc = lib().lz_ortho_loss(X.data_ptr(), X.stride(1), n, c, p, _stream_ptr(stream), ctypes.byref(out))
    if rc != 0:
        raise LanczosError(rc, "lz_ortho_loss")
    return out.value


# ------------------------------------------------------------------ serving
class Request(ctypes.Structure):
    _fields_ = [("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("K", ctypes.c_int32), ("m", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reorth", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("out_vals", ctypes.c_void_p), ("out_vecs", ctypes.c_void_p), ("out_resid", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("m_eff", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("slot", ctypes.c_int32), ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("device_ms", ctypes.c_double), ("resid_max", ctypes.c_double),
                ("ortho_loss", ctypes.c_double)]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("active", ctypes.c_uint64), ("queued", ctypes.c_uint64), ("arena_bytes", ctypes.c_size_t),
                ("arena_in_use", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
                ("worker_enqueue_ms", ctypes.c_double)]


def _server_lib():
    L = lib()
    if not hasattr(L, "_server_ready"):
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.lz_request_footprint.restype = ctypes.c_size_t
        L.lz_request_footprint.argtypes = [i64, i64, i32, i32, i32]
        L.lz_server_create.restype = ctypes.c_int
        L.lz_server_create.argtypes = [ctypes.c_int, ctypes.c_size_t, i32, i32, ctypes.POINTER(P)]
        L.lz_server_submit.restype = ctypes.c_int
        L.lz_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.lz_server_poll.restype = ctypes.c_int
        L.lz_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
        L.lz_server_wait.restype = ctypes.c_int
        L.lz_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
        L.lz_server_get_stats.restype = ctypes.c_int
        L.lz_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
        L.lz_server_destroy.restype = ctypes.c_int
        L.lz_server_destroy.argtypes = [P]
        L._server_ready = True
    return L


def request_footprint(n: int, nnz: int, K: int, m: int, precision="fp64") -> int:
    return int(_server_lib().lz_request_footprint(n, nnz, K, m, _prec(precision)))


def _host_ptr(a):
    """Address of a contiguous host array (numpy array or CPU torch tensor)."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise TypeError("host arrays must be contiguous")
        return a.ctypes.data
    if a.is_cuda or not a.is_contiguous():
        raise TypeError("host arrays must be contiguous CPU tensors")
    return a.data_ptr()


class Server:
    """Continuous-batching request loop of the C library (lz_server_*).

    submit() takes host CSR arrays (numpy or pinned CPU tensors); they and
    the output buffers are kept alive here until the request completes."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 8, use_graphs: bool = True, device: int = 0):
        L = _server_lib()
        h = ctypes.c_void_p()
        rc = L.lz_server_create(device, int(hbm_budget_bytes), max_slots, 1 if use_graphs else 0, ctypes.byref(h))
        if rc != 0:
            raise LanczosError(rc, "lz_server_create")
        self._h = h
        self._keep = {}

    def submit(self, rowptr, col, val, K: int, m: int, precision="fp64", seed: int = 0, reorth="twice",
               want_vectors: bool = False) -> int:
        n = len(rowptr) - 1
        nnz = len(col)
        vals = np.zeros(K, dtype=np.float64)
        resid = np.zeros(K, dtype=np.float64)
        vecs = np.zeros((K, n), dtype=np.float64) if want_vectors else None
        req = Request(rowptr=_host_ptr(rowptr), col=_host_ptr(col), val=_host_ptr(val), n=n, nnz=nnz, K=K, m=m,
                      precision=_prec(precision), reorth=REORTH[reorth] if isinstance(reorth, str) else int(reorth),
                      seed=seed & (2 ** 64 - 1), out_vals=vals.ctypes.data,
                      out_vecs=vecs.ctypes.data if vecs is not None else None, out_resid=resid.ctypes.data)
        t = ctypes.c_uint64(0)
        rc = _server_lib().lz_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if rc != 0:
            raise LanczosError(rc, "lz_server_submit")
        self._keep[t.value] = (rowptr, col, val, vals, vecs, resid)
        return t.value

    def poll(self, ticket: int):
        """None while running, else (vals, vecs or None, result dict).  The
        dict holds the lz_result fields and "resid", the relative residual of
        each returned pair in the order of vals (zeros unless status is 0)."""
        res = Result()
        rc = _server_lib().lz_server_poll(self._h, ticket, ctypes.byref(res))
        if rc == 1:
            return None
        return self._finish(ticket, rc, res)

    def wait(self, ticket: int):
        res = Result()
        rc = _server_lib().lz_server_wait(self._h, ticket, ctypes.byref(res))
        return self._finish(ticket, rc, res)

    def _finish(self, ticket, rc, res):
        keep = self._keep.get(ticket)
        if rc < 0 and keep is None:
            raise LanczosError(rc, "lz_server_poll")
        d = res.to_dict()
        d["status"] = rc
        d["resid"] = keep[5] if keep else None
        vals, vecs = (keep[3], keep[4]) if keep else (None, None)
        return vals, (vecs.T if vecs is not None else None), d

    def release(self, ticket: int):
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        st = ServerStats()
        _server_lib().lz_server_get_stats(self._h, ctypes.byref(st))
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if self._h:
            _server_lib().lz_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
