"""The refinement entry point that allocates nothing (chol_refine_solve_noalloc):
through the C ABI it gives the same results as chol_refine_solve with a
caller workspace (bitwise: same kernels, same order), which match the
oracle's refined FP64 solution within the 1e-10 bar; two calls in a row, the
second with a smaller problem (the static array keeps the first call's
contents); and a problem larger than the array is rejected before any device
work."""
import numpy as np
import pytest
import torch

import gp_inputs
import oracle
import paper_2605_13209_amd as P
from paper_2605_13209_amd import _native

pytestmark = pytest.mark.gpu


def dev(a):
    return P.to_colmajor(torch.from_numpy(np.asarray(a)))


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("method", ["ir", "pcg"])
def test_noalloc_matches_workspace_entry_point(method):
    cases = [(1500, 5, 11), (700, 2, 12)]  # second call smaller in n and k
    for n, k, seed in cases:
        X, B = gp_inputs.gp_problem(n, seed=seed, k=k)
        A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
        Ad = dev(A)
        F = P.chol_factor(Ad, "fp32", 128)
        Bd = dev(B)
        ref = P.chol_refine_solve(F, Bd, A=Ad, noise=0.1, tol=1e-10, method=method)
        out = P.colmajor_empty(n, k)
        got = _native.chol_refine_solve_noalloc(F, Bd, out, A=Ad, noise=0.1, tol=1e-10, method=method)
        assert got.converged and ref.converged
        assert got.iters == ref.iters and got.fallback_used == ref.fallback_used == 0
        x, xr = host(got.X), host(ref.X)
        assert np.array_equal(x, xr), (n, k, np.abs(x - xr).max())
        L, info = oracle.cholesky(A)
        xo, _, _, failed = oracle.refine(L, A, B, lam=0.1, tol=1e-13)
        assert info == 0 and failed == 0
        err = np.linalg.norm(x - xo, axis=0) / np.linalg.norm(xo, axis=0)
        assert err.max() <= 1e-10, (n, k, err.max())


def test_noalloc_matrix_free_and_size_limit():
    n, k = 900, 3
    X, B = gp_inputs.gp_problem(n, seed=13, k=k)
    Xd = torch.from_numpy(X).cuda()
    Ad = P.gp_assemble(Xd, 0.8, 1.0, 0.05)
    F = P.chol_factor(Ad, "fp32", 128)
    Bd = dev(B)
    ref = P.chol_refine_solve(F, Bd, X_feat=Xd, lengthscale=0.8, noise=0.05, tol=1e-10)
    out = P.colmajor_empty(n, k)
    got = _native.chol_refine_solve_noalloc(F, Bd, out, X_feat=Xd, lengthscale=0.8, noise=0.05, tol=1e-10)
    assert got.converged and np.array_equal(host(got.X), host(ref.X))
    # a problem whose refinement buffers exceed the static array: rejected, nothing enqueued
    cap = _native.chol_refine_noalloc_max_bytes()
    assert cap == 64 << 20
    big_k = cap // (40 * n) + 1
    assert _native.lib().chol_refine_bytes(n, big_k, 0) > cap
    rc = _native.lib().chol_refine_solve_noalloc(F.handle, Ad.data_ptr(), n, None, 0, 0, 1.0, 1.0, 0.05,
                                                 Bd.data_ptr(), n, out.data_ptr(), n, big_k, 1e-10, 30, 0,
                                                 None, None)
    assert rc == _native.CHOL_ERR_WORKSPACE
