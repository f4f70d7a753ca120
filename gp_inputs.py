"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds input recipes only: random draws and exact integer
constructions.  It contains none of the solver's arithmetic and imports
neither the oracle nor the HIP library.

Recipes
-------
* ``gp_problem``: the squared-exponential GP workload.  ``rng =
  numpy.random.default_rng(seed)``; features ``X = rng.uniform(-1, 1, (n, d))``
  drawn first, then right-hand sides ``B = rng.standard_normal((n, k))``,
  returned column-major.  The paper's own matrices come from a
  mass-spring-damper dataset that is not available here; this generator stands
  in for it at the same sizes.
* ``known_l0``: lower-triangular L0 with power-of-two diagonal and small
  integer off-diagonal entries, and A = L0 L0^T formed in exact integer
  arithmetic.  Every Cholesky algorithm that uses substitution (any blocking,
  any summation order, with or without fused multiply-add) must return L0
  bit-exactly, because every intermediate value is an integer below 2^53
  (2^24 for FP32 storage when n is small) and every division is by a power of
  two.
* ``serving_stream``: Poisson arrivals of GP solve requests of uneven size.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Hyper-parameters of the named workloads: (lengthscale, variance, noise).
SE_DEFAULT = (1.0, 1.0, 0.1)      # n = 1024 / 32768 / 65536 workloads
SE_WELL_COND = (0.5, 1.0, 1.0)    # n = 131072 FP16 workload


def gp_problem(n: int, d: int = 8, k: int = 1, seed: int = 0):
    """Features X (n x d, row-major FP64) and RHS B (n x k, column-major FP64)."""
    rng = np.random.default_rng(seed)
    X = np.ascontiguousarray(rng.uniform(-1.0, 1.0, (n, d)))
    B = np.asfortranarray(rng.standard_normal((n, k)))
    return X, B


def known_l0(n: int, family: str = "dense-int", seed: int = 0):
    """(L0, A) with A = L0 L0^T exact.  Both returned column-major FP64.

    dense-int : |L0_ij| <= 3 off the diagonal, diagonal in {1, 2, 4, 8}.
                Very ill-conditioned; only exact arithmetic reproduces L0.
    sparse-dd : diagonal 32, about 10% of the off-diagonal entries +-1.
                Well conditioned.
    small-int : |L0_ij| <= 1, diagonal in {1, 2}; entries of A stay below
                2^24 for n up to several thousand (exact in FP32 too).
    """
    rng = np.random.default_rng(seed)
    if family == "dense-int":
        L = rng.integers(-3, 4, size=(n, n)).astype(np.int64)
        diag = rng.choice(np.array([1, 2, 4, 8], dtype=np.int64), size=n)
    elif family == "sparse-dd":
        L = rng.integers(-1, 2, size=(n, n)).astype(np.int64)
        L *= (rng.random((n, n)) < 0.1)
        diag = np.full(n, 32, dtype=np.int64)
    elif family == "small-int":
        L = rng.integers(-1, 2, size=(n, n)).astype(np.int64)
        diag = rng.choice(np.array([1, 2], dtype=np.int64), size=n)
    else:
        raise ValueError(family)
    L = np.tril(L, -1)
    L[np.arange(n), np.arange(n)] = diag
    A = L @ L.T  # exact in int64
    if n and np.abs(A).max() >= 2**53:
        raise ValueError("entries too large for exact FP64")
    return np.asfortranarray(L.astype(np.float64)), np.asfortranarray(A.astype(np.float64))


@dataclass
class Request:
    """One GP solve request of the serving workload."""
    rid: int
    arrival: float          # seconds since the start of the stream
    n: int
    k: int
    lengthscale: float
    noise: float
    key: int                # matrix key; equal keys mean the same matrix
    seed: int               # seed of the features X (per key) ...
    rhs_seed: int           # ... and of the right-hand sides (per request)

    def features(self, d: int = 8) -> np.ndarray:
        rng = np.random.default_rng(self.seed)
        return np.ascontiguousarray(rng.uniform(-1.0, 1.0, (self.n, d)))

    def rhs(self) -> np.ndarray:
        rng = np.random.default_rng(self.rhs_seed)
        return np.asfortranarray(rng.standard_normal((self.n, self.k)))


def serving_stream(duration_s: float = 30.0, rate: float = 200.0, seed: int = 0,
                   n_min: int = 256, n_max: int = 8192, k_max: int = 64,
                   repeat_frac: float = 0.25, repeat_window: int = 64):
    """Poisson arrivals; n = round(exp(U[ln n_min, ln n_max])); lengthscale ~ U[0.3, 2];
    noise ~ U[0.01, 1]; k ~ U{1..k_max}; a fraction ``repeat_frac`` of the requests
    reuses the matrix of one of the last ``repeat_window`` distinct keys."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out: list[Request] = []
    keys: list[tuple] = []
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            break
        k = int(rng.integers(1, k_max + 1))
        if keys and rng.random() < repeat_frac:
            key, n, ls, noise, fseed = keys[int(rng.integers(max(0, len(keys) - repeat_window), len(keys)))]
        else:
            n = int(round(float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))))
            ls = float(rng.uniform(0.3, 2.0))
            noise = float(rng.uniform(0.01, 1.0))
            key = len(keys)
            fseed = int(rng.integers(0, 2**31 - 1))
            keys.append((key, n, ls, noise, fseed))
        out.append(Request(rid, t, n, k, ls, noise, key, fseed, int(rng.integers(0, 2**31 - 1))))
        rid += 1
    return out
