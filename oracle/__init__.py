"""Plain CPU FP64 oracle for the GP Cholesky solver path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2605_13209_amd``) never imports, links or calls it, and it
imports nothing from the product library.

The arithmetic lives in ``chol_oracle.c`` (plain loops, FP64, sums in index
order), compiled with gcc into ``liboracle.so``; this module only marshals
numpy arrays to it.  Each function cites the passage it follows:

* ``gp_assemble``  - squared-exponential covariance, the stand-in for the
  paper's GP kernel matrices (Experimental Setup).
* ``cholesky``     - L L^T = A, L lower (Fundamentals, "The Cholesky
  decomposition"), computed by its defining equations.
* ``forward`` / ``backward`` / ``solve`` - forward and back substitution with L
  (same section).
* ``residual`` / ``gp_residual`` - b - A x with long-double accumulation.
* ``refine``       - iterative refinement with a low-precision factor (the
  paper lists mixed precision as future work; textbook IR).
* ``cg``           - the paper's conjugate gradient method (Fundamentals, "The
  Conjugate Gradient method"), with its periodic true-residual recomputation.
* ``pcg``          - CG (paper's CG algorithm) preconditioned with M = F F^T.
* ``backward_error`` / ``backward_error_estimate`` / ``certificate`` -
  checkers (the estimate is Hutchinson's, for orders the exact one cannot reach).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chol_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int64
_IP = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, IEEE semantics, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_gp_assemble.argtypes = [_D, _I, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        lib.oracle_gp_entry.argtypes = [_D, _I, _I, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.oracle_gp_entry.restype = ctypes.c_double
        lib.oracle_cholesky.argtypes = [_D, _I, _I, _D, _I]
        lib.oracle_cholesky.restype = ctypes.c_int64
        for f in (lib.oracle_forward, lib.oracle_backward, lib.oracle_solve):
            f.argtypes = [_D, _I, _I, _D, _I, _I]
        lib.oracle_residual.argtypes = [_D, _I, _I, _D, _D, _I, _D]
        lib.oracle_gp_residual.argtypes = [_D, _I, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           _D, _D, _I, _D]
        lib.oracle_refine.argtypes = [_D, _I, _D, _I, _I, _D, _D, _I, ctypes.c_double, ctypes.c_double,
                                      _I, _IP, _D]
        lib.oracle_refine.restype = ctypes.c_int64
        lib.oracle_pcg.argtypes = [_D, _I, _D, _I, _I, _D, _D, _I, ctypes.c_double, ctypes.c_double,
                                   _I, _I, _IP, _D]
        lib.oracle_pcg.restype = ctypes.c_int64
        lib.oracle_cg.argtypes = [_D, _I, _I, _D, _D, _I, ctypes.c_double, _I, _I, _IP, _D]
        lib.oracle_cg.restype = ctypes.c_int64
        lib.oracle_backward_error_probes.argtypes = [_D, _I, _D, _I, ctypes.c_double, ctypes.c_double,
                                                     ctypes.c_double, _D, _I, _I, _D, _I, _D, _D]
        lib.oracle_backward_error.argtypes = [_D, _I, _D, _I, _I]
        lib.oracle_backward_error.restype = ctypes.c_double
        lib.oracle_certificate.argtypes = [_D, _D, _I, ctypes.c_double]
        lib.oracle_certificate.restype = ctypes.c_double
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _colmajor(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return np.array(a, dtype=np.float64, order="F", copy=True)


def num_threads() -> int:
    """Threads used by the oracle's OpenMP loops."""
    return int(_load().oracle_num_threads())


def gp_assemble(X, lengthscale: float, variance: float, noise: float) -> np.ndarray:
    """Full n x n SE covariance + noise on the diagonal (column-major)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, d = X.shape
    A = np.empty((n, n), dtype=np.float64, order="F")
    _load().oracle_gp_assemble(_p(X), n, d, lengthscale, variance, noise, _p(A))
    return A


def gp_entry(X, i: int, j: int, lengthscale: float, variance: float, noise: float) -> float:
    X = np.ascontiguousarray(X, dtype=np.float64)
    return _load().oracle_gp_entry(_p(X), X.shape[1], int(i), int(j), lengthscale, variance, noise)


def cholesky(A):
    """Returns (L, info).  L full n x n column-major with zero upper triangle."""
    A = np.asfortranarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.empty((n, n), dtype=np.float64, order="F")
    info = _load().oracle_cholesky(_p(A), n, max(n, 1), _p(L), max(n, 1))
    if info < 0:
        raise MemoryError("oracle_cholesky: allocation failed")
    return L, int(info)


def _tri(fn, L, B):
    L = np.asfortranarray(L, dtype=np.float64)
    vec = np.ndim(B) == 1
    X = _colmajor(B)
    n, k = X.shape
    getattr(_load(), fn)(_p(L), n, max(n, 1), _p(X), k, max(n, 1))
    return X[:, 0] if vec else X


def forward(L, B):
    return _tri("oracle_forward", L, B)


def backward(L, B):
    return _tri("oracle_backward", L, B)


def solve(L, B):
    return _tri("oracle_solve", L, B)


def residual(A, X, B):
    A = np.asfortranarray(A, dtype=np.float64)
    vec = np.ndim(B) == 1
    Xc, Bc = _colmajor(X), _colmajor(B)
    n, k = Bc.shape
    R = np.empty((n, k), dtype=np.float64, order="F")
    _load().oracle_residual(_p(A), n, n, _p(Xc), _p(Bc), k, _p(R))
    return R[:, 0] if vec else R


def gp_residual(Xfeat, lengthscale, variance, noise, X, B):
    F = np.ascontiguousarray(Xfeat, dtype=np.float64)
    vec = np.ndim(B) == 1
    Xc, Bc = _colmajor(X), _colmajor(B)
    n, k = Bc.shape
    R = np.empty((n, k), dtype=np.float64, order="F")
    _load().oracle_gp_residual(_p(F), n, F.shape[1], lengthscale, variance, noise, _p(Xc), _p(Bc), k, _p(R))
    return R[:, 0] if vec else R


def refine(F, A, B, lam: float, tol: float = 1e-10, max_iter: int = 30):
    """Returns (X, iters[k], cert[k], n_failed)."""
    F = np.asfortranarray(F, dtype=np.float64)
    A = np.asfortranarray(A, dtype=np.float64)
    Bc = _colmajor(B)
    n, k = Bc.shape
    X = np.empty((n, k), dtype=np.float64, order="F")
    it = np.zeros(k, dtype=np.int64)
    ce = np.zeros(k, dtype=np.float64)
    failed = _load().oracle_refine(_p(F), n, _p(A), n, n, _p(Bc), _p(X), k, lam, tol, max_iter,
                                   it.ctypes.data_as(_IP), _p(ce))
    return X, it, ce, int(failed)


def pcg(F, A, B, lam: float, tol: float = 1e-10, max_iter: int = 200, recompute: int = 50):
    """Returns (X, iters[k], cert[k], n_failed)."""
    F = np.asfortranarray(F, dtype=np.float64)
    A = np.asfortranarray(A, dtype=np.float64)
    Bc = _colmajor(B)
    n, k = Bc.shape
    X = np.empty((n, k), dtype=np.float64, order="F")
    it = np.zeros(k, dtype=np.int64)
    ce = np.zeros(k, dtype=np.float64)
    failed = _load().oracle_pcg(_p(F), n, _p(A), n, n, _p(Bc), _p(X), k, lam, tol, max_iter, recompute,
                                it.ctypes.data_as(_IP), _p(ce))
    return X, it, ce, int(failed)


def cg(A, B, X0=None, eps: float = 1e-6, max_iter: int = 10000, recompute: int = 50):
    """The paper's CG per column.  Returns (X, iters[k], relres[k], n_stopped)."""
    A = np.asfortranarray(A, dtype=np.float64)
    Bc = _colmajor(B)
    n, k = Bc.shape
    X = np.zeros((n, k), dtype=np.float64, order="F") if X0 is None else _colmajor(X0)
    it = np.zeros(k, dtype=np.int64)
    rr = np.zeros(k, dtype=np.float64)
    stopped = _load().oracle_cg(_p(A), n, n, _p(Bc), _p(X), k, eps, max_iter, recompute,
                                it.ctypes.data_as(_IP), _p(rr))
    return X, it, rr, int(stopped)


def backward_error(A, L) -> float:
    A = np.asfortranarray(A, dtype=np.float64)
    L = np.asfortranarray(L, dtype=np.float64)
    n = A.shape[0]
    return _load().oracle_backward_error(_p(A), n, _p(L), n, n)


def backward_error_estimate(L, Z, A=None, Xfeat=None, lengthscale=1.0, variance=1.0, noise=0.0):
    """Hutchinson estimate of ||A - L L^T||_F / ||A||_F from the probe columns
    Z; A dense, or (A None) the GP matrix of the features Xfeat, matrix-free.
    Returns (estimate, num, den)."""
    L = np.asfortranarray(L, dtype=np.float64)
    n = L.shape[0]
    Zc = _colmajor(Z)
    k = Zc.shape[1]
    num, den = ctypes.c_double(0), ctypes.c_double(0)
    if A is not None:
        A = np.asfortranarray(A, dtype=np.float64)
        a_ptr, lda, f_ptr, d = _p(A), n, None, 0
    else:
        Xfeat = np.ascontiguousarray(Xfeat, dtype=np.float64)
        a_ptr, lda, f_ptr, d = None, 1, _p(Xfeat), Xfeat.shape[1]
    _load().oracle_backward_error_probes(a_ptr, lda, f_ptr, d, lengthscale, variance, noise, _p(L), L.shape[0],
                                         n, _p(Zc), k, ctypes.byref(num), ctypes.byref(den))
    return float(np.sqrt(num.value / den.value)), num.value, den.value


def certificate(r, x, lam: float) -> float:
    r = np.ascontiguousarray(r, dtype=np.float64).ravel()
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return _load().oracle_certificate(_p(r), _p(x), r.size, lam)
