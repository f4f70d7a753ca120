"""The CPU tile kernels of the heterogeneous factorisation (host code in the
HIP library, called through its C ABI on host memory; no GPU needed),
checked against the oracle and exact-arithmetic cases."""
import ctypes

import numpy as np
import pytest

import gp_inputs
import oracle
from paper_2605_13209_amd import _native

B = 128
U = np.finfo(np.float64).eps / 2


def lib():
    return _native.lib()


def ptr(a):
    assert a.flags["F_CONTIGUOUS"] and a.dtype == np.float64
    return a.ctypes.data


def test_potrf_tile_matches_oracle():
    X, _ = gp_inputs.gp_problem(B, seed=3)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L = np.asfortranarray(A.copy())
    assert lib().chol_host_potrf_tile(ptr(L)) == 0
    assert np.all(np.triu(L, 1) == 0.0)
    Lref, info = oracle.cholesky(A)
    assert info == 0
    assert np.linalg.norm(L - Lref) / np.linalg.norm(Lref) <= 1e-13
    assert oracle.backward_error(A, L) <= 1e-15


def test_potrf_tile_exact_and_info():
    L0, A0 = gp_inputs.known_l0(B, "dense-int", seed=5)
    L = np.asfortranarray(A0.copy())
    assert lib().chol_host_potrf_tile(ptr(L)) == 0
    assert np.array_equal(L, L0)
    # a non-positive pivot at local column 41 (1-based: 42), as the oracle reports
    A = A0.copy()
    A[41, 41] = 0.0
    _, info_ref = oracle.cholesky(A)
    L = np.asfortranarray(A)
    assert lib().chol_host_potrf_tile(ptr(L)) == info_ref == 42


def test_trsm_tile_exact_and_residual():
    L0, _ = gp_inputs.known_l0(B, "sparse-dd", seed=6)
    Xi = np.asfortranarray(np.random.default_rng(1).integers(-4, 5, size=(B, B)).astype(np.float64))
    A = np.asfortranarray(Xi @ L0.T)  # exact: small integers
    Xs = A.copy(order="F")
    lib().chol_host_trsm_tile(ptr(L0), ptr(Xs))
    assert np.array_equal(Xs, Xi)
    # a general right-hand side: X L^T = A to rounding
    Xg, _ = gp_inputs.gp_problem(B, seed=7)
    G = oracle.gp_assemble(Xg, 1.0, 1.0, 0.1)
    Lg, _ = oracle.cholesky(G)
    R = np.asfortranarray(np.random.default_rng(2).standard_normal((B, B)))
    Xr = R.copy(order="F")
    lib().chol_host_trsm_tile(ptr(Lg), ptr(Xr))
    assert np.abs(Xr @ Lg.T - R).max() <= 64 * U * (np.abs(Xr) @ np.abs(Lg.T)).max()


@pytest.mark.parametrize("np_,lower", [(1, False), (3, False), (2, True)])
def test_gemm_nt_tiles(np_, lower):
    rng = np.random.default_rng(10 + np_)
    As = [np.asfortranarray(rng.integers(-8, 9, size=(B, B)).astype(np.float64)) for _ in range(np_)]
    Bs = [np.asfortranarray(rng.integers(-8, 9, size=(B, B)).astype(np.float64)) for _ in range(np_)]
    C0 = np.asfortranarray(rng.integers(-100, 101, size=(B, B)).astype(np.float64))
    C = C0.copy(order="F")
    pa = (ctypes.c_void_p * np_)(*[ptr(a) for a in As])
    pb = (ctypes.c_void_p * np_)(*[ptr(b) for b in Bs])
    lib().chol_host_gemm_nt_tiles(ptr(C), pa, pb, np_, 1 if lower else 0)
    ref = C0 - sum(a @ b.T for a, b in zip(As, Bs))  # exact in integers
    if lower:
        # the lower triangle is updated; the strict upper one is unspecified
        il = np.tril_indices(B)
        assert np.array_equal(C[il], ref[il])
    else:
        assert np.array_equal(C, ref)
