"""The continuous-batching factorisation engine (chol_batch_*) and the
serving executor built on it.  A job's factor is the FP32 factorisation
computed column by column, so it is bitwise the one chol_factor gives with
panel width 1 and no lookahead (the same tile kernels in the same order),
whatever else is in the batch and with or without the captured graph; the
refined solutions match the oracle's."""
import numpy as np
import pytest
import torch

import gp_inputs
import oracle
import paper_2605_13209_amd as P
from paper_2605_13209_amd.serve import BatchedHipExecutor, Server, SolveRequest

pytestmark = pytest.mark.gpu


def dev(a):
    return P.to_colmajor(torch.from_numpy(np.asarray(a)))


def host(t):
    return t.detach().cpu().numpy()


def gp_matrix(n, seed, hp=(1.0, 1.0, 0.1)):
    X, _ = gp_inputs.gp_problem(n, seed=seed)
    Xd = torch.from_numpy(X).cuda()
    return P.gp_assemble(Xd, *hp, full=False)


def run_engine(mats, use_graph=True, stagger=0):
    """Factor every matrix through one engine; job i joins after i*stagger steps."""
    eng = P.BatchEngine(max_jobs=16, use_graph=use_graph)
    torch.cuda.synchronize()
    jobs = {}
    pending = list(range(len(mats)))
    step = 0
    while pending or any(not eng.done(j) for j in jobs.values()):
        for i in list(pending):
            if step >= i * stagger:
                jobs[i] = eng.add(mats[i])
                pending.remove(i)
        eng.step()
        step += 1
    Fs, dense = [], []
    for i in range(len(mats)):
        F = eng.take(jobs[i])
        Fs.append(F)
        dense.append(P.chol_factor_to_dense(F, stream=eng.stream))
    torch.cuda.synchronize()  # the factors and their dense copies are on the engine's stream
    return eng, [(F, host(L)) for F, L in zip(Fs, dense)]


def test_batch_equals_column_by_column_factor_bitwise():
    sizes = [1000, 256, 3000, 129, 2048]
    mats = [gp_matrix(n, seed=50 + i) for i, n in enumerate(sizes)]
    eng, out = run_engine(mats, stagger=2)
    for A, (F, L) in zip(mats, out):
        assert F.info() == 0 and F.precision == P.CHOL_FP32
        ref = P.chol_factor(A, "fp32", 128, panel_width=1, lookahead=0)
        assert np.array_equal(L, host(P.chol_factor_to_dense(ref)))
    eng.close()


def test_batch_alone_equals_mixed_and_graph_equals_direct():
    sizes = [700, 2500, 1300]
    mats = [gp_matrix(n, seed=60 + i) for i, n in enumerate(sizes)]
    _, mixed = run_engine(mats, stagger=1)
    for i, A in enumerate(mats):
        _, alone = run_engine([A], use_graph=False)
        assert np.array_equal(alone[0][1], mixed[i][1])


def test_batch_factor_parity_and_refine():
    n = 1800
    X, B = gp_inputs.gp_problem(n, seed=70, k=3)
    A = oracle.gp_assemble(X, 0.8, 1.0, 0.05)
    Ad = dev(A)
    eng, out = run_engine([Ad, gp_matrix(900, seed=71)], stagger=3)
    F, L = out[0]
    assert oracle.backward_error(A, L) <= 5e-6
    res = P.chol_refine_solve(F, dev(B), A=Ad, noise=0.05, tol=1e-10)
    assert res.converged
    xref = oracle.solve(oracle.cholesky(A)[0], B)
    x = host(res.X)
    assert np.max(np.linalg.norm(x - xref, axis=0) / np.linalg.norm(xref, axis=0)) <= 1e-10
    eng.close()


def test_batch_not_spd_job_does_not_disturb_others():
    good = gp_matrix(1500, seed=80)
    Ab = oracle.gp_assemble(gp_inputs.gp_problem(1000, seed=81)[0], 1.0, 1.0, 0.1)
    Ab[600, 600] = -5.0
    _, info_ref = oracle.cholesky(Ab)
    eng, out = run_engine([good, dev(Ab)], stagger=0)
    assert out[1][0].info() == info_ref == 601
    ref = P.chol_factor(good, "fp32", 128, panel_width=1, lookahead=0)
    assert out[0][0].info() == 0 and np.array_equal(out[0][1], host(P.chol_factor_to_dense(ref)))
    eng.close()


def make_requests(seed, sizes, kmax):
    rng = np.random.default_rng(seed)
    reqs = []
    for i, n in enumerate(sizes):
        X, B = gp_inputs.gp_problem(n, d=8, k=int(rng.integers(1, kmax + 1)), seed=300 + i)
        reqs.append(SolveRequest(X=X, B=B, lengthscale=float(rng.uniform(0.3, 2.0)), variance=1.0,
                                 noise=float(rng.uniform(0.01, 1.0)), key=("b", seed, i), rid=i))
    return reqs


def clone(r):
    return SolveRequest(X=r.X, B=r.B, lengthscale=r.lengthscale, variance=r.variance, noise=r.noise,
                        key=r.key, rid=r.rid, tol=r.tol)


def test_batched_serving_certified_alone_and_mixed():
    """The serving configuration's range (n from 256 to 8192, up to 64
    right-hand sides) through the batched executor: each result is bitwise the
    same alone and in a mix, and certified by the oracle: the long-double
    residual b - A x of the GPU's solution gives ||r|| / (noise ||x||) <= 1e-10,
    a rigorous bound on its relative error (lambda_min(A) >= noise)."""
    reqs = make_requests(5, (256, 8192, 700, 3000, 1024, 5000, 384), kmax=64)
    ex = BatchedHipExecutor(workers=4)
    try:
        with Server(ex, hbm_budget=16e9, max_inflight=1, cache=False) as s:
            alone = [s.submit(clone(r)).result(timeout=120) for r in reqs]
        with Server(ex, hbm_budget=16e9, max_inflight=4, cache=False) as s:
            futs = [s.submit(clone(r)) for r in reqs]
            mixed = [f.result(timeout=120) for f in futs]
    finally:
        ex.close()
    assert ex.steps > 0
    for r, a, m in zip(reqs, alone, mixed):
        assert np.array_equal(a.X, m.X) and a.iters == m.iters
        assert a.converged and a.cert <= 0.5e-10
        A = oracle.gp_assemble(r.X, r.lengthscale, r.variance, r.noise)
        R = oracle.residual(A, a.X, r.B)
        for c in range(r.k):
            assert oracle.certificate(R[:, c], a.X[:, c], r.noise) <= 1e-10, (r.n, c)
