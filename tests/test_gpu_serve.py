"""GPU serving: each result matches the oracle's refined FP64 solution, is
bitwise identical alone and in a concurrent mix, and factor reuse works."""
import numpy as np
import pytest

import gp_inputs
import oracle
from paper_2605_13209_amd.serve import HipExecutor, Server, SolveRequest

pytestmark = pytest.mark.gpu


def make_requests(seed=0, sizes=(256, 300, 511, 700, 1000, 1024, 384, 900), kmax=17):
    rng = np.random.default_rng(seed)
    reqs = []
    for i, n in enumerate(sizes):
        X, B = gp_inputs.gp_problem(n, d=8, k=int(rng.integers(1, kmax + 1)), seed=100 + i)
        ls = float(rng.uniform(0.3, 2.0))
        noise = float(rng.uniform(0.01, 1.0))
        reqs.append(SolveRequest(X=X, B=B, lengthscale=ls, variance=1.0, noise=noise, key=("m", i), rid=i))
    return reqs


def clone(r):
    return SolveRequest(X=r.X, B=r.B, lengthscale=r.lengthscale, variance=r.variance, noise=r.noise,
                        key=r.key, rid=r.rid, tol=r.tol)


def test_serving_matches_oracle():
    reqs = make_requests()
    with Server(HipExecutor(workers=4), hbm_budget=8e9, max_inflight=4) as s:
        futs = [s.submit(clone(r)) for r in reqs]
        out = [f.result(timeout=120) for f in futs]
    for r, res in zip(reqs, out):
        assert res.converged and res.cert <= 0.5e-10
        A = oracle.gp_assemble(r.X, r.lengthscale, r.variance, r.noise)
        L, info = oracle.cholesky(A)
        assert info == 0
        xref, _, _, failed = oracle.refine(L, A, r.B, lam=r.noise, tol=1e-13)
        assert failed == 0
        for c in range(r.k):
            err = np.linalg.norm(res.X[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c])
            assert err <= 1e-10, (r.n, c, err)


def test_alone_equals_mix_bitwise():
    reqs = make_requests(seed=1)
    ex = HipExecutor(workers=6)
    with Server(ex, hbm_budget=8e9, max_inflight=1, cache=False) as s:
        alone = [s.submit(clone(r)).result(timeout=120) for r in reqs]
    with Server(ex, hbm_budget=8e9, max_inflight=6, cache=False) as s:
        futs = [s.submit(clone(r)) for r in reqs]
        mixed = [f.result(timeout=120) for f in futs]
    for a, m in zip(alone, mixed):
        assert np.array_equal(a.X, m.X)
        assert a.iters == m.iters


def test_serving_large_sample_matches_oracle_and_mix():
    """The serving configuration's upper range (n up to 8192, up to 64
    right-hand sides): each result matches the oracle's refined solution, and
    is bitwise the same alone and in a concurrent mix."""
    reqs = make_requests(seed=3, sizes=(8192, 5000, 2900, 6144, 1500), kmax=64)
    reqs[0].B = gp_inputs.gp_problem(8192, d=8, k=64, seed=200)[1]  # the largest corner: n = 8192, k = 64
    ex = HipExecutor(workers=4)
    with Server(ex, hbm_budget=16e9, max_inflight=1, cache=False) as s:
        alone = [s.submit(clone(r)).result(timeout=300) for r in reqs]
    with Server(ex, hbm_budget=16e9, max_inflight=4, cache=False) as s:
        futs = [s.submit(clone(r)) for r in reqs]
        mixed = [f.result(timeout=300) for f in futs]
    for r, a, m in zip(reqs, alone, mixed):
        assert np.array_equal(a.X, m.X) and a.iters == m.iters
        assert a.converged and a.cert <= 0.5e-10
        A = oracle.gp_assemble(r.X, r.lengthscale, r.variance, r.noise)
        L, info = oracle.cholesky(A)
        assert info == 0
        xref, _, _, failed = oracle.refine(L, A, r.B, lam=r.noise, tol=1e-13)
        assert failed == 0
        err = np.linalg.norm(a.X - xref, axis=0) / np.linalg.norm(xref, axis=0)
        assert err.max() <= 1e-10, (r.n, r.k, err.max())


def test_factor_reuse():
    r = make_requests(seed=2, sizes=(800,))[0]
    with Server(HipExecutor(workers=2), hbm_budget=8e9, max_inflight=2) as s:
        first = s.submit(clone(r)).result(timeout=60)
        second = s.submit(clone(r)).result(timeout=60)
        assert not first.reused_factor and second.reused_factor
        assert np.array_equal(first.X, second.X)
        assert s.stats()["reused_factors"] == 1
