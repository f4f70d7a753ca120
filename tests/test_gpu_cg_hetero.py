"""GPU + CPU parity of the heterogeneous CG (cg_solve_hetero, through the C
ABI) against the oracle's CG, which follows the paper's algorithm step by
step.  As for the GPU-only CG, the two differ only in the order of the sums
inside A s and the dot products, so after m <= 8 steps the iterates agree to
1e-11 relative whatever the split; converged runs are compared through the
true residual."""
import numpy as np
import pytest
import torch

import gp_inputs
import oracle
import paper_2605_13209_amd as P

pytestmark = pytest.mark.gpu


def dev(a):
    return P.to_colmajor(torch.from_numpy(np.asarray(a)))


def host(t):
    return t.detach().cpu().numpy()


def gp(n, seed, hp=(1.0, 1.0, 0.1)):
    X, B = gp_inputs.gp_problem(n, seed=seed, k=1)
    return oracle.gp_assemble(X, *hp), B


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n,share", [(1000, 0.5), (2000, 0.9), (1300, 0.0), (1000, 1.0), (3000, 0.97),
                                     (130, 0.5)])
def test_hetero_cg_first_steps_match_oracle(n, share):
    A, B = gp(n, seed=n)
    Ad, Bd = dev(A), dev(B)
    for m in (1, 2, 5, 8):
        X, it, rr, conv, rep = P.cg_solve_hetero(Ad, Bd[:, 0], share, eps=1e-15, max_iter=m, recompute=0)
        xo, ito, rro, _ = oracle.cg(A, B, eps=1e-15, max_iter=m, recompute=0)
        assert it == ito[0] == m
        assert rel(host(X), xo[:, 0]) <= 1e-11, (m, rel(host(X), xo[:, 0]))
        np.testing.assert_allclose(rr, rro[0], rtol=1e-9, atol=1e-14)
        N = (n + 127) // 128
        assert rep["gpu_rows"] <= N and rep["iterations"] == m


@pytest.mark.parametrize("recompute", [1, 3])
def test_hetero_cg_recompute_steps_match_oracle(recompute):
    n = 1500
    A, B = gp(n, seed=31, hp=(0.7, 1.0, 0.05))
    X, it, rr, conv, rep = P.cg_solve_hetero(dev(A), dev(B)[:, 0], 0.6, eps=1e-15, max_iter=7,
                                             recompute=recompute)
    xo, ito, rro, _ = oracle.cg(A, B, eps=1e-15, max_iter=7, recompute=recompute)
    assert it == ito[0] and rep["recomputations"] == 7 // recompute
    assert rel(host(X), xo[:, 0]) <= 1e-11
    np.testing.assert_allclose(rr, rro[0], rtol=1e-9)


def test_hetero_cg_converged_matches_oracle_and_gpu_only():
    n = 2500
    A, B = gp(n, seed=41)
    eps = 1e-10
    Ad, Bd = dev(A), dev(B)
    X, it, rr, conv, rep = P.cg_solve_hetero(Ad, Bd[:, 0], 0.8, eps=eps, max_iter=5000, recompute=50)
    xo, ito, rro, stopped = oracle.cg(A, B, eps=eps, max_iter=5000, recompute=50)
    assert conv and stopped == 0
    assert abs(it - ito[0]) <= 0.1 * ito[0] + 2, (it, ito)
    x = host(X)
    R = oracle.residual(A, x, B[:, 0])
    true = np.linalg.norm(R) / np.linalg.norm(B[:, 0])
    assert true <= 2 * eps, true
    gap = np.linalg.norm(x - xo[:, 0])
    assert gap <= 2 * 2 * eps * np.linalg.norm(B[:, 0]) / 0.1
    g = P.cg_solve(Ad, Bd, eps=eps, max_iter=5000, recompute=50)
    assert abs(g.iters[0] - it) <= 0.1 * it + 2
    assert rep["bytes_h2d"] > 0 and rep["bytes_d2h"] > 0 and 0.0 < rep["gpu_share_tiles"] < 1.0


def test_hetero_cg_starting_guess():
    n = 900
    A, B = gp(n, seed=43)
    x0 = np.random.default_rng(5).standard_normal(n)
    X, it, rr, conv, rep = P.cg_solve_hetero(dev(A), dev(B)[:, 0], 0.5, X=dev(x0[:, None])[:, 0].clone(),
                                             eps=1e-15, max_iter=4, recompute=0)
    xo, ito, rro, _ = oracle.cg(A, B, X0=x0[:, None], eps=1e-15, max_iter=4, recompute=0)
    assert rel(host(X), xo[:, 0]) <= 1e-11
