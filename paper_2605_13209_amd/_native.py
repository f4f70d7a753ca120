"""ctypes binding of ``libchol_mi355x.so`` (declared in ``include/chol.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
torch tensors supply device memory and streams.  There is no fallback: if
the library is not built, every call raises.

Matrices are column-major.  A column-major n x m torch tensor is one whose
stride is (1, ld); ``colmajor_empty`` makes one.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libchol_mi355x.so")

CHOL_FP64, CHOL_FP32, CHOL_FP16_SCALED = 0, 1, 2
PRECISIONS = {"fp64": CHOL_FP64, "fp32": CHOL_FP32, "fp16_scaled": CHOL_FP16_SCALED}
CHOL_REFINE_IR, CHOL_REFINE_PCG = 0, 1
METHODS = {"ir": CHOL_REFINE_IR, "pcg": CHOL_REFINE_PCG}
CHOL_ERR_WORKSPACE = -101
CHOL_ERR_NOT_CONVERGED = -102
CHOL_ERR_NOT_SPD = -103

_lib = None
_vp, _i64, _int, _dbl, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t


class CholError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: status {status} ({chol_status_string(status)})")


class FactorOpts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("panel_width", ctypes.c_int32), ("lookahead", ctypes.c_int32),
                ("super_tile", ctypes.c_int32), ("graph", ctypes.c_int32)]


class RefineReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("cert", ctypes.c_double),
                ("resid_norm", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("fallback_used", ctypes.c_int32), ("reserved", ctypes.c_int32)]


CHOL_FALLBACK_PCG, CHOL_FALLBACK_SHIFT, CHOL_FALLBACK_FP32 = 1, 2, 4


EXPORTS = {
    # name: (restype, argtypes)
    "gp_assemble": (_int, [_vp, _i64, _i64, _i64, _dbl, _dbl, _dbl, _vp, _i64, _int, _vp]),
    "chol_factor_bytes": (_sz, [_i64, _int, _int]),
    "chol_tile_default": (_int, [_i64, _int]),
    "chol_factor": (_int, [_vp, _i64, _i64, _int, _int, _vp, _sz, ctypes.POINTER(_vp),
                           ctypes.POINTER(_i64), _vp]),
    "chol_factor_ex": (_int, [_vp, _i64, _i64, _int, ctypes.POINTER(FactorOpts), _vp, _sz, ctypes.POINTER(_vp),
                              ctypes.POINTER(_i64), _vp]),
    "chol_get_info": (_int, [_vp, ctypes.POINTER(_i64)]),
    "chol_solve": (_int, [_vp, _vp, _i64, _i64, _vp]),
    "chol_refine_bytes": (_sz, [_i64, _i64, _int]),
    "chol_refine_solve": (_int, [_vp, _vp, _i64, _vp, _i64, _i64, _dbl, _dbl, _dbl, _vp, _i64, _vp,
                                 _i64, _i64, _dbl, _int, _int, _vp, _sz, ctypes.POINTER(RefineReport),
                                 _vp]),
    "chol_refine_noalloc_max_bytes": (_sz, []),
    "chol_refine_solve_noalloc": (_int, [_vp, _vp, _i64, _vp, _i64, _i64, _dbl, _dbl, _dbl, _vp, _i64, _vp,
                                         _i64, _i64, _dbl, _int, _int, ctypes.POINTER(RefineReport), _vp]),
    "chol_residual": (_int, [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _i64, _vp]),
    "chol_factor_to_dense": (_int, [_vp, _vp, _i64, _vp]),
    "chol_factor_n": (_i64, [_vp]),
    "chol_factor_tile": (_int, [_vp]),
    "chol_factor_precision": (_int, [_vp]),
    "chol_factor_fallback": (_int, [_vp]),
    "chol_factor_free": (None, [_vp]),
    "chol_status_string": (ctypes.c_char_p, [_int]),
    "chol_set_option": (_int, [ctypes.c_char_p, _i64]),
    "chol_get_option": (_i64, [ctypes.c_char_p]),
    "chol_profile_read": (_int, [ctypes.POINTER(_dbl), ctypes.POINTER(_i64), ctypes.POINTER(_dbl)]),
    "chol_profile_reset": (None, []),
    "chol_hetero_host_bytes": (_sz, [_i64]),
    "chol_factor_hetero": (_int, [_vp, _i64, _i64, _dbl, _int, _vp, _sz, _vp, _sz, ctypes.POINTER(_vp),
                                  ctypes.POINTER(_i64), _vp, _vp]),
    "cg_hetero_workspace_bytes": (_sz, [_i64]),
    "cg_hetero_host_bytes": (_sz, [_i64, _dbl]),
    "cg_solve_hetero": (_int, [_vp, _i64, _i64, _vp, _vp, _dbl, _i64, _i64, _dbl, _vp, _sz, _vp, _sz,
                               ctypes.POINTER(_i64), ctypes.POINTER(_dbl), _vp, _vp]),
    "chol_batch_desc_bytes": (_sz, [_int]),
    "chol_batch_create": (_int, [_int, _vp, _sz, _int, _vp, ctypes.POINTER(_vp)]),
    "chol_batch_destroy": (None, [_vp]),
    "chol_batch_add": (_int, [_vp, _vp, _i64, _i64, _vp, _sz, ctypes.POINTER(_i64)]),
    "chol_batch_step": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int)]),
    "chol_batch_status": (_int, [_vp, _i64, ctypes.POINTER(_int)]),
    "chol_batch_take": (_int, [_vp, _i64, ctypes.POINTER(_vp)]),
    "chol_host_potrf_tile": (_int, [_vp]),
    "chol_host_trsm_tile": (None, [_vp, _vp]),
    "chol_host_gemm_nt_tiles": (None, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _int, _int]),
    "cg_workspace_bytes": (_sz, [_i64, _int, _i64]),
    "cg_solve": (_int, [_vp, _i64, _i64, _int, _vp, _i64, _vp, _i64, _i64, _dbl, _i64, _i64, _vp, _sz,
                        ctypes.POINTER(_i64), ctypes.POINTER(_dbl), _vp]),
}
CG_MAX_RHS = 16


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run `python -m paper_2605_13209_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def chol_status_string(status: int) -> str:
    return lib().chol_status_string(int(status)).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise CholError(rc, what)


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def colmajor_empty(rows: int, cols: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    """An uninitialised rows x cols tensor with column-major strides (1, rows)."""
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def to_colmajor(t: torch.Tensor, device="cuda") -> torch.Tensor:
    """Column-major FP64 copy (or view, if already so) of a 1-D or 2-D tensor on ``device``."""
    if t.dim() == 1:
        t = t[:, None]
    t = t.to(device=device, dtype=torch.float64)
    if t.stride(0) == 1 and t.stride(1) >= max(1, t.shape[0]):
        return t
    out = colmajor_empty(t.shape[0], t.shape[1], device=t.device)
    out.copy_(t)
    return out


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("expected a column-major 2-D tensor (stride (1, ld))")
    return max(1, t.stride(1), t.shape[0])


def _need_device(t: torch.Tensor, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{what} must be float64")


def set_option(key: str, value: int):
    _check(lib().chol_set_option(key.encode(), int(value)), f"chol_set_option({key})")


def get_option(key: str) -> int:
    return int(lib().chol_get_option(key.encode()))


def chol_profile_read():
    """(kernel ms, launches, algorithmic flops) of the trailing-update launches recorded so far."""
    ms, n, fl = _dbl(0), _i64(0), _dbl(0)
    _check(lib().chol_profile_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)), "chol_profile_read")
    return float(ms.value), int(n.value), float(fl.value)


def chol_profile_reset():
    lib().chol_profile_reset()


def gp_assemble(X: torch.Tensor, lengthscale: float, variance: float, noise: float, *, full: bool = True,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Squared-exponential covariance plus noise, column-major n x n FP64 on X's device."""
    _need_device(X, "X")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a row-major n x d tensor")
    n, d = X.shape
    A = colmajor_empty(n, n, device=X.device) if out is None else out
    _check(lib().gp_assemble(X.data_ptr(), n, d, max(d, X.stride(0)), float(lengthscale), float(variance),
                             float(noise), A.data_ptr(), _ld(A), 1 if full else 0, _stream(stream)),
           "gp_assemble")
    return A


def chol_factor_bytes(n: int, precision: str | int = "fp64", tile: int = 0) -> int:
    p = PRECISIONS.get(precision, precision)
    return int(lib().chol_factor_bytes(int(n), int(p), int(tile)))


def chol_tile_default(n: int, precision: str | int = "fp64") -> int:
    return int(lib().chol_tile_default(int(n), int(PRECISIONS.get(precision, precision))))


def chol_refine_bytes(n: int, nrhs: int, method: str | int = "ir") -> int:
    return int(lib().chol_refine_bytes(int(n), int(nrhs), int(METHODS.get(method, method))))


@dataclass
class RefineResult:
    X: torch.Tensor
    iters: int
    converged: bool
    cert: float
    resid_norm: float
    time_ms: float
    status: int
    fallback_used: int = 0


class Factor:
    """Host handle of a factor living in a caller-owned workspace tensor."""

    def __init__(self, handle, workspace: torch.Tensor, stream):
        self._h = handle
        self.workspace = workspace
        self.stream = stream
        self.n = int(lib().chol_factor_n(handle))
        self.tile = int(lib().chol_factor_tile(handle))
        self.precision = int(lib().chol_factor_precision(handle))
        self.fallback = int(lib().chol_factor_fallback(handle))

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("factor freed")
        return self._h

    def info(self) -> int:
        v = _i64(0)
        _check(lib().chol_get_info(self.handle, ctypes.byref(v)), "chol_get_info")
        return int(v.value)

    def free(self):
        if self._h is not None:
            lib().chol_factor_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def chol_factor(A: torch.Tensor, precision: str | int = "fp64", tile: int = 0, *,
                workspace: torch.Tensor | None = None, sync: bool = True, stream=None,
                panel_width: int = 0, lookahead: int = -1, super_tile: int = 0, graph: int = -1) -> Factor:
    """Factor A = L L^T on the GPU (chol_factor_ex).  With sync=True, raises
    CholError(CHOL_ERR_NOT_SPD) if info > 0.  panel_width / lookahead /
    super_tile override the process-wide schedule options for this call."""
    _need_device(A, "A")
    n = A.shape[0]
    p = int(PRECISIONS.get(precision, precision))
    need = chol_factor_bytes(n, p, tile)
    if need == 0:
        raise ValueError("invalid n / precision / tile")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
    h = _vp()
    info = _i64(0)
    st = _stream(stream)
    opts = FactorOpts(int(tile), int(panel_width), int(lookahead), int(super_tile), int(graph))
    rc = lib().chol_factor_ex(A.data_ptr(), n, _ld(A), p, ctypes.byref(opts), workspace.data_ptr(),
                              workspace.numel() * workspace.element_size(), ctypes.byref(h),
                              ctypes.byref(info) if sync else None, st)
    _check(rc, "chol_factor")
    F = Factor(h, workspace, st)
    if sync and info.value != 0:
        F.free()
        e = CholError(CHOL_ERR_NOT_SPD, "chol_factor")
        e.info = int(info.value)
        raise e
    return F


def chol_solve(F: Factor, B: torch.Tensor, stream=None) -> torch.Tensor:
    """In place: B <- A^{-1} B (column-major FP64, n x nrhs)."""
    _need_device(B, "B")
    _check(lib().chol_solve(F.handle, B.data_ptr(), B.shape[1], _ld(B), _stream(stream)), "chol_solve")
    return B


def chol_refine_solve(F: Factor, B: torch.Tensor, *, A: torch.Tensor | None = None,
                      X_feat: torch.Tensor | None = None, lengthscale: float = 1.0, variance: float = 1.0,
                      noise: float = 0.0, tol: float = 1e-10, max_iter: int = 30, method: str | int = "ir",
                      out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                      raise_on_fail: bool = True, stream=None) -> RefineResult:
    """FP64-accurate solve of A X = B with a (low-precision) factor F, by IR or PCG."""
    _need_device(B, "B")
    n, k = B.shape
    m = int(METHODS.get(method, method))
    X = colmajor_empty(n, k, device=B.device) if out is None else out
    need = chol_refine_bytes(n, k, m)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=B.device)
    rep = RefineReport()
    a_ptr, lda = (A.data_ptr(), _ld(A)) if A is not None else (None, max(1, n))
    if X_feat is not None:
        xf_ptr, d, ldxf = X_feat.data_ptr(), X_feat.shape[1], max(X_feat.shape[1], X_feat.stride(0))
    else:
        xf_ptr, d, ldxf = None, 0, 0
    rc = lib().chol_refine_solve(F.handle, a_ptr, lda, xf_ptr, d, ldxf, float(lengthscale), float(variance),
                                 float(noise), B.data_ptr(), _ld(B), X.data_ptr(), _ld(X), k, float(tol),
                                 int(max_iter), m, workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), ctypes.byref(rep), _stream(stream))
    if rc not in (0, CHOL_ERR_NOT_CONVERGED) or (rc != 0 and raise_on_fail):
        _check(rc, "chol_refine_solve")
    return RefineResult(X, rep.iters, bool(rep.converged), rep.cert, rep.resid_norm, rep.time_ms, rc,
                        rep.fallback_used)


def chol_refine_solve_noalloc(F: Factor, B: torch.Tensor, out: torch.Tensor, *, A: torch.Tensor | None = None,
                              X_feat: torch.Tensor | None = None, lengthscale: float = 1.0,
                              variance: float = 1.0, noise: float = 0.0, tol: float = 1e-10, max_iter: int = 30,
                              method: str | int = "ir", raise_on_fail: bool = True, stream=None) -> RefineResult:
    """chol_refine_solve with the library's static device scratch array instead
    of a workspace (no device allocation by the library; ``out`` is required,
    so the binding allocates nothing either)."""
    _need_device(B, "B")
    _need_device(out, "out")
    n, k = B.shape
    m = int(METHODS.get(method, method))
    rep = RefineReport()
    a_ptr, lda = (A.data_ptr(), _ld(A)) if A is not None else (None, max(1, n))
    if X_feat is not None:
        xf_ptr, d, ldxf = X_feat.data_ptr(), X_feat.shape[1], max(X_feat.shape[1], X_feat.stride(0))
    else:
        xf_ptr, d, ldxf = None, 0, 0
    rc = lib().chol_refine_solve_noalloc(F.handle, a_ptr, lda, xf_ptr, d, ldxf, float(lengthscale),
                                         float(variance), float(noise), B.data_ptr(), _ld(B), out.data_ptr(),
                                         _ld(out), k, float(tol), int(max_iter), m, ctypes.byref(rep),
                                         _stream(stream))
    if rc not in (0, CHOL_ERR_NOT_CONVERGED) or (rc != 0 and raise_on_fail):
        _check(rc, "chol_refine_solve_noalloc")
    return RefineResult(out, rep.iters, bool(rep.converged), rep.cert, rep.resid_norm, rep.time_ms, rc,
                        rep.fallback_used)


def chol_refine_noalloc_max_bytes() -> int:
    return int(lib().chol_refine_noalloc_max_bytes())


class BatchEngine:
    """The continuous-batching factorisation engine (chol_batch_*): FP32
    factors, tile 128, one tile column per step for every active job."""

    def __init__(self, max_jobs: int = 64, stream=None, use_graph: bool = True, device=None):
        self.max_jobs = int(max_jobs)
        nb = int(lib().chol_batch_desc_bytes(self.max_jobs))
        if nb == 0:
            raise ValueError("max_jobs out of range")
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self.desc = torch.empty(nb, dtype=torch.uint8, device=dev)
        h = _vp()
        _check(lib().chol_batch_create(self.max_jobs, self.desc.data_ptr(), nb, 1 if use_graph else 0,
                                       _stream(self.stream), ctypes.byref(h)), "chol_batch_create")
        self._h = h
        self._ws = {}

    def add(self, A: torch.Tensor, workspace: torch.Tensor | None = None) -> int:
        _need_device(A, "A")
        n = A.shape[0]
        need = chol_factor_bytes(n, CHOL_FP32, 128)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
        job = _i64(0)
        _check(lib().chol_batch_add(self._h, A.data_ptr(), n, _ld(A), workspace.data_ptr(),
                                    workspace.numel() * workspace.element_size(), ctypes.byref(job)),
               "chol_batch_add")
        self._ws[int(job.value)] = workspace
        return int(job.value)

    def step(self) -> tuple[int, int]:
        a, f = _int(0), _int(0)
        _check(lib().chol_batch_step(self._h, ctypes.byref(a), ctypes.byref(f)), "chol_batch_step")
        return int(a.value), int(f.value)

    def done(self, job: int) -> bool:
        d = _int(0)
        _check(lib().chol_batch_status(self._h, int(job), ctypes.byref(d)), "chol_batch_status")
        return bool(d.value)

    def take(self, job: int) -> "Factor":
        h = _vp()
        _check(lib().chol_batch_take(self._h, int(job), ctypes.byref(h)), "chol_batch_take")
        return Factor(h, self._ws.pop(int(job)), _stream(self.stream))

    def close(self):
        if self._h is not None:
            torch.cuda.synchronize()
            lib().chol_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HeteroReport(ctypes.Structure):
    _fields_ = [("gpu_share_target", ctypes.c_double), ("gpu_share_tiles", ctypes.c_double),
                ("gpu_tile_updates", ctypes.c_double), ("cpu_tile_updates", ctypes.c_double),
                ("bytes_h2d", ctypes.c_double), ("bytes_d2h", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_cpu", ctypes.c_double), ("ms_wait_gpu", ctypes.c_double),
                ("border_shifts", ctypes.c_int32), ("handover_column", ctypes.c_int32),
                ("cpu_threads", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def chol_hetero_host_bytes(n: int) -> int:
    return int(lib().chol_hetero_host_bytes(int(n)))


def chol_factor_hetero(A: torch.Tensor, gpu_share: float, *, panel_width: int = 0,
                       workspace: torch.Tensor | None = None, host_ws: torch.Tensor | None = None,
                       stream=None, raise_not_spd: bool = True):
    """Heterogeneous CPU + GPU FP64 factorisation (tile 128); returns (Factor,
    report dict).  host_ws: a host uint8/float64 tensor of at least
    chol_hetero_host_bytes(n) bytes (pinned for asynchronous copies)."""
    _need_device(A, "A")
    n = A.shape[0]
    need = chol_factor_bytes(n, CHOL_FP64, 128)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
    hb = chol_hetero_host_bytes(n)
    if host_ws is None:
        host_ws = torch.empty(max(hb, 8), dtype=torch.uint8, pin_memory=True)
    if host_ws.is_cuda:
        raise ValueError("host_ws must be host memory")
    h = _vp()
    info = _i64(0)
    rep = HeteroReport()
    st = _stream(stream)
    rc = lib().chol_factor_hetero(A.data_ptr(), n, _ld(A), float(gpu_share), int(panel_width),
                                  workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                  host_ws.data_ptr(), host_ws.numel() * host_ws.element_size(), ctypes.byref(h),
                                  ctypes.byref(info), ctypes.byref(rep), st)
    _check(rc, "chol_factor_hetero")
    F = Factor(h, workspace, st)
    if raise_not_spd and info.value != 0:
        F.free()
        e = CholError(CHOL_ERR_NOT_SPD, "chol_factor_hetero")
        e.info = int(info.value)
        raise e
    return F, rep.as_dict()


class CgHeteroReport(ctypes.Structure):
    _fields_ = [("gpu_share_target", ctypes.c_double), ("gpu_share_tiles", ctypes.c_double),
                ("bytes_h2d", ctypes.c_double), ("bytes_d2h", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_cpu", ctypes.c_double), ("ms_wait_gpu", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("recomputations", ctypes.c_int32), ("gpu_rows", ctypes.c_int32), ("cpu_threads", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def cg_solve_hetero(A: torch.Tensor, b: torch.Tensor, gpu_share: float, *, X: torch.Tensor | None = None,
                    eps: float = 1e-6, max_iter: int = 100000, recompute: int = 50,
                    workspace: torch.Tensor | None = None, host_ws: torch.Tensor | None = None, stream=None):
    """Heterogeneous CPU + GPU CG for one right-hand side b (device, n or n x 1).
    Returns (X, iterations, relres, converged, report dict)."""
    _need_device(A, "A")
    _need_device(b, "b")
    n = A.shape[0]
    if X is None:
        X = torch.zeros(n, dtype=torch.float64, device=A.device)
    need = int(lib().cg_hetero_workspace_bytes(n))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    hb = int(lib().cg_hetero_host_bytes(n, float(gpu_share)))
    if host_ws is None:
        host_ws = torch.empty(max(hb, 8), dtype=torch.uint8, pin_memory=True)
    if host_ws.is_cuda:
        raise ValueError("host_ws must be host memory")
    it = _i64(0)
    rr = ctypes.c_double(0.0)
    rep = CgHeteroReport()
    rc = lib().cg_solve_hetero(A.data_ptr(), n, _ld(A), b.data_ptr(), X.data_ptr(), float(eps), int(max_iter),
                               int(recompute), float(gpu_share), workspace.data_ptr(),
                               workspace.numel() * workspace.element_size(), host_ws.data_ptr(),
                               host_ws.numel() * host_ws.element_size(), ctypes.byref(it), ctypes.byref(rr),
                               ctypes.byref(rep), _stream(stream))
    if rc not in (0, CHOL_ERR_NOT_CONVERGED):
        _check(rc, "cg_solve_hetero")
    return X, int(it.value), float(rr.value), rc == 0, rep.as_dict()


def chol_residual(A: torch.Tensor, X: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """R = B - A X (A symmetric, lower triangle read), FP64 with double-double accumulation."""
    n, k = B.shape
    R = colmajor_empty(n, k, device=B.device) if out is None else out
    _check(lib().chol_residual(A.data_ptr(), _ld(A), n, X.data_ptr(), _ld(X), B.data_ptr(), _ld(B),
                               R.data_ptr(), _ld(R), k, _stream(stream)), "chol_residual")
    return R


def chol_factor_to_dense(F: Factor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Dense column-major FP64 L (upper triangle zero)."""
    L = colmajor_empty(F.n, F.n, device=F.workspace.device) if out is None else out
    _check(lib().chol_factor_to_dense(F.handle, L.data_ptr(), _ld(L), _stream(stream)), "chol_factor_to_dense")
    return L


def cg_workspace_bytes(n: int, nrhs: int = 1, tile: int = 0) -> int:
    return int(lib().cg_workspace_bytes(int(n), int(tile), int(nrhs)))


@dataclass
class CgResult:
    X: torch.Tensor
    iters: list
    relres: list
    converged: bool
    status: int


def cg_solve(A: torch.Tensor, B: torch.Tensor, X: torch.Tensor | None = None, *, eps: float = 1e-6,
             max_iter: int = 100000, recompute: int = 50, tile: int = 0, workspace: torch.Tensor | None = None,
             raise_on_fail: bool = False, stream=None) -> CgResult:
    """The paper's CG on the GPU (cg_solve): X holds the starting guess (zeros
    if None) and receives the iterate; synchronous."""
    _need_device(A, "A")
    _need_device(B, "B")
    n, k = B.shape
    if X is None:
        X = colmajor_empty(n, k, device=B.device)
        X.zero_()
    need = cg_workspace_bytes(n, k, tile)
    if need == 0:
        raise ValueError("invalid n / nrhs / tile")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=B.device)
    its = (_i64 * k)()
    rr = (_dbl * k)()
    rc = lib().cg_solve(A.data_ptr(), n, _ld(A), int(tile), B.data_ptr(), _ld(B), X.data_ptr(), _ld(X), k,
                        float(eps), int(max_iter), int(recompute), workspace.data_ptr(),
                        workspace.numel() * workspace.element_size(), its, rr, _stream(stream))
    if rc not in (0, CHOL_ERR_NOT_CONVERGED) or (rc != 0 and raise_on_fail):
        _check(rc, "cg_solve")
    return CgResult(X, [int(v) for v in its], [float(v) for v in rr], rc == 0, rc)
