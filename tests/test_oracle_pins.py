"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes one part of the oracle by something independent: exact
integer constructions, hand-worked closed forms, a high-precision library
factorisation (mpmath), LAPACK (numpy/scipy), scikit-learn's RBF kernel, and
rigorous bounds.  A dropped term, a sign error, a transposed operand or a
wrong index in any oracle routine fails at least one of them.
"""
import json
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import gp_inputs
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = np.finfo(np.float64).eps / 2


def _cases():
    with open(os.path.join(GOLDEN, "closed_form_cases.json")) as f:
        return json.load(f)


# --------------------------------------------------------------- Cholesky ---

@pytest.mark.parametrize("case", _cases()["cases"], ids=lambda c: c["name"])
def test_closed_form_factor_and_solve(case):
    A = np.array(case["A"], dtype=np.float64)
    L, info = oracle.cholesky(A)
    assert info == 0
    np.testing.assert_array_equal(L, np.array(case["L"], dtype=np.float64))
    y = oracle.forward(L, np.array(case["b"], dtype=np.float64))
    np.testing.assert_allclose(y, case["y"], rtol=0, atol=0)
    x = oracle.backward(L, y)
    np.testing.assert_allclose(x, case["x"], rtol=2 * U, atol=0)
    np.testing.assert_allclose(oracle.solve(L, np.array(case["b"], float)), case["x"], rtol=2 * U)


@pytest.mark.parametrize("case", _cases()["not_spd"], ids=lambda c: c["name"])
def test_not_spd_info(case):
    _, info = oracle.cholesky(np.array(case["A"], dtype=np.float64))
    assert info == case["info"]


def test_nan_and_negative_pivot_info():
    A = np.eye(7)
    A[4, 4] = -1.0
    assert oracle.cholesky(A)[1] == 5
    A = np.eye(7)
    A[2, 2] = np.nan
    assert oracle.cholesky(A)[1] == 3


def test_one_by_one():
    L, info = oracle.cholesky(np.array([[2.0]]))
    assert info == 0 and L[0, 0] == np.sqrt(2.0)


def test_identity_and_block_diagonal():
    L, info = oracle.cholesky(np.eye(9))
    assert info == 0
    np.testing.assert_array_equal(L, np.eye(9))
    _, A1 = gp_inputs.known_l0(5, "sparse-dd", seed=1)
    X, _ = gp_inputs.gp_problem(6, seed=2)
    A2 = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    A = sla.block_diag(A1, A2)
    L, info = oracle.cholesky(A)
    L1, _ = oracle.cholesky(A1)
    L2, _ = oracle.cholesky(A2)
    assert info == 0
    np.testing.assert_array_equal(L, sla.block_diag(L1, L2))


def test_identity_padding_invariant():
    """chol(diag(A, I)) = diag(chol(A), I) exactly; the padding rule for ragged tiles."""
    X, _ = gp_inputs.gp_problem(37, seed=3)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L, _ = oracle.cholesky(A)
    Lp, info = oracle.cholesky(sla.block_diag(A, np.eye(11)))
    assert info == 0
    np.testing.assert_array_equal(Lp, sla.block_diag(L, np.eye(11)))


@pytest.mark.parametrize("n,family", [(64, "dense-int"), (200, "dense-int"), (300, "sparse-dd"),
                                      (257, "small-int")])
def test_known_l0_exact_recovery(n, family):
    L0, A = gp_inputs.known_l0(n, family, seed=n)
    L, info = oracle.cholesky(A)
    assert info == 0
    np.testing.assert_array_equal(L, L0)


@pytest.mark.parametrize("n,family", [(120, "dense-int"), (300, "sparse-dd")])
def test_known_l0_exact_solve(n, family):
    L0, A = gp_inputs.known_l0(n, family, seed=7)
    rng = np.random.default_rng(5)
    x0 = rng.integers(-4, 5, size=(n, 3)).astype(np.int64)
    b = (A.astype(np.int64) @ x0).astype(np.float64)
    y = oracle.forward(L0, b)
    np.testing.assert_array_equal(y, (L0.T.astype(np.int64) @ x0).astype(np.float64))
    x = oracle.backward(L0, y)
    np.testing.assert_array_equal(x, x0.astype(np.float64))


@pytest.mark.parametrize("n", [3, 8, 15])
def test_mpmath_brute_force(n):
    """50-digit mpmath Cholesky and solve; FP64 oracle within c * kappa * u."""
    X, B = gp_inputs.gp_problem(n, seed=11 + n, k=1)
    A = oracle.gp_assemble(X, 0.8, 1.0, 0.05)
    mpmath.mp.dps = 50
    Am = mpmath.matrix(A.tolist())
    Lm = mpmath.cholesky(Am)
    xm = mpmath.cholesky_solve(Am, mpmath.matrix(B[:, 0].tolist()))
    L, info = oracle.cholesky(A)
    assert info == 0
    Lref = np.array(Lm.tolist(), dtype=np.float64)
    kappa = np.linalg.cond(A)
    np.testing.assert_allclose(L, Lref, rtol=0, atol=50 * n * kappa * U * np.abs(Lref).max())
    x = oracle.solve(L, B[:, 0])
    xref = np.array([float(v) for v in xm])
    assert np.linalg.norm(x - xref) / np.linalg.norm(xref) <= 10 * n * kappa * U


def test_against_lapack_on_gp_matrix():
    X, _ = gp_inputs.gp_problem(300, seed=4)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L, info = oracle.cholesky(A)
    assert info == 0
    Lnp = np.linalg.cholesky(A)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(L - Lnp) / np.linalg.norm(Lnp) <= 300 * kappa * U
    be = oracle.backward_error(A, L)
    assert be <= 1e-15


def test_triangular_solves_against_scipy():
    X, B = gp_inputs.gp_problem(150, seed=9, k=4)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L, _ = oracle.cholesky(A)
    y = oracle.forward(L, B)
    np.testing.assert_allclose(y, sla.solve_triangular(L, B, lower=True), rtol=1e-12, atol=1e-12)
    x = oracle.backward(L, y)
    np.testing.assert_allclose(x, sla.solve_triangular(L.T, y, lower=False), rtol=1e-12, atol=1e-12)
    xs = oracle.solve(L, B)
    xnp = np.linalg.solve(A, B)
    assert np.linalg.norm(xs - xnp) / np.linalg.norm(xnp) <= 1e-12


# -------------------------------------------------------------- assembly ---

def test_gp_assemble_against_sklearn_rbf():
    from sklearn.gaussian_process.kernels import RBF
    X, _ = gp_inputs.gp_problem(200, d=8, seed=1)
    for ls, var, noise in [(1.0, 1.0, 0.1), (0.5, 1.0, 1.0), (2.0, 3.0, 0.01)]:
        A = oracle.gp_assemble(X, ls, var, noise)
        K = var * RBF(length_scale=ls)(X) + noise * np.eye(200)
        np.testing.assert_allclose(A, K, rtol=1e-13, atol=0)
        assert np.array_equal(A, A.T)
        assert np.all(np.diag(A) == var + noise)
        off = A[~np.eye(200, dtype=bool)]
        assert np.all(off > 0) and np.all(off <= var)


def test_gp_assemble_closed_form_points():
    """Points at squared distance 2 ls^2 ln 2 and 2 ls^2 give var/2 and var/e."""
    ls = 0.7
    X = np.zeros((3, 8))
    X[1, 0] = ls * np.sqrt(2 * np.log(2.0))
    X[2, 3] = ls * np.sqrt(2.0)
    A = oracle.gp_assemble(X, ls, 2.0, 0.25)
    assert A[0, 0] == 2.25
    np.testing.assert_allclose(A[1, 0], 1.0, rtol=8 * U)
    np.testing.assert_allclose(A[2, 0], 2.0 / np.e, rtol=8 * U)
    assert oracle.gp_entry(X, 2, 0, ls, 2.0, 0.25) == A[2, 0]
    assert oracle.gp_entry(X, 1, 1, ls, 2.0, 0.25) == 2.25


def test_gp_lambda_min_bound():
    """lambda_min(A) >= noise: the certificate's premise."""
    X, _ = gp_inputs.gp_problem(400, seed=6)
    A = oracle.gp_assemble(X, 2.0, 1.0, 0.01)
    assert np.linalg.eigvalsh(A).min() >= 0.01 * (1 - 1e-8)


# ------------------------------------------------------ residual / refine ---

def test_residual_exact_on_integers():
    L0, A = gp_inputs.known_l0(90, "sparse-dd", seed=2)
    rng = np.random.default_rng(1)
    x = rng.integers(-5, 6, size=(90, 2)).astype(np.float64)
    b = A @ x
    r = oracle.residual(A, x, b)
    assert np.all(r == 0)
    x2 = x.copy()
    x2[3, 1] += 1.0
    r = oracle.residual(A, x2, b)
    np.testing.assert_array_equal(r[:, 1], -A[:, 3])


def test_gp_residual_matches_assembled():
    X, B = gp_inputs.gp_problem(120, seed=8, k=2)
    A = oracle.gp_assemble(X, 0.9, 1.0, 0.2)
    xs = np.random.default_rng(3).standard_normal((120, 2))
    r1 = oracle.residual(A, xs, B)
    r2 = oracle.gp_residual(X, 0.9, 1.0, 0.2, xs, B)
    np.testing.assert_allclose(r1, r2, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r1, B - A @ xs, rtol=0, atol=1e-12)


@pytest.mark.parametrize("method", ["ir", "pcg"])
def test_refinement_with_fp32_factor(method):
    n = 400
    X, B = gp_inputs.gp_problem(n, seed=12, k=3)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L, _ = oracle.cholesky(A)
    F = L.astype(np.float32).astype(np.float64)  # emulated low-precision factor
    xnp = np.linalg.solve(A, B)
    if method == "ir":
        Xs, it, cert, failed = oracle.refine(F, A, B, lam=0.1, tol=1e-10)
    else:
        Xs, it, cert, failed = oracle.pcg(F, A, B, lam=0.1, tol=1e-10)
    assert failed == 0
    assert np.all(cert <= 0.5e-10)
    assert np.all(it >= 1)  # the FP32 factor alone is not accurate enough
    for c in range(3):
        err = np.linalg.norm(Xs[:, c] - xnp[:, c]) / np.linalg.norm(xnp[:, c])
        assert err <= 1e-10
        # the certificate is a rigorous bound on the error
        assert err <= cert[c] * np.linalg.norm(Xs[:, c]) / np.linalg.norm(xnp[:, c]) * (1 + 1e-6) + 1e-15


def test_refinement_without_noise_bound():
    n = 200
    X, B = gp_inputs.gp_problem(n, seed=13, k=1)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L, _ = oracle.cholesky(A)
    F = L.astype(np.float32).astype(np.float64)
    Xs, it, cert, failed = oracle.refine(F, A, B, lam=0.0, tol=1e-12)
    assert failed == 0
    xnp = np.linalg.solve(A, B)
    assert np.linalg.norm(Xs - xnp) / np.linalg.norm(xnp) <= 1e-11


def test_certificate_matches_definition_cases():
    r = np.array([3.0, 4.0])
    x = np.array([0.0, 10.0])
    assert oracle.certificate(r, x, 0.5) == 1.0


def test_backward_error_exact_factor_is_zero():
    L0, A = gp_inputs.known_l0(60, "dense-int", seed=3)
    assert oracle.backward_error(A, L0) == 0.0
    L1 = L0.copy()
    L1[10, 3] += 1.0
    E = A - L1 @ L1.T
    np.testing.assert_allclose(oracle.backward_error(A, L1), np.linalg.norm(E) / np.linalg.norm(A), rtol=1e-12)


def test_inputs_are_seeded():
    X1, B1 = gp_inputs.gp_problem(50, seed=4, k=2)
    X2, B2 = gp_inputs.gp_problem(50, seed=4, k=2)
    assert np.array_equal(X1, X2) and np.array_equal(B1, B2)
    assert X1.flags.c_contiguous and B1.flags.f_contiguous
    assert X1.min() >= -1 and X1.max() < 1
    s = gp_inputs.serving_stream(duration_s=2.0, seed=0)
    assert len(s) > 100 and all(256 <= r.n <= 8192 and 1 <= r.k <= 64 for r in s)
    assert all(a.arrival < b.arrival for a, b in zip(s, s[1:]))


# ------------------------------------------------- conjugate gradients ---

def test_cg_shewchuk_two_by_two_hand_worked():
    # A = [[3, 2], [2, 6]], b = [2, -8], x0 = 0 (Shewchuk's example system).
    # By hand: r0 = b, u0 = 68, t = A r0 = [-10, -44], s.t = 332,
    # alpha = 68/332 = 17/83, so x1 = (17/83) b = [34/83, -136/83]; CG ends
    # at the exact solution [2, -2] after n = 2 steps.
    A = np.array([[3.0, 2.0], [2.0, 6.0]])
    b = np.array([2.0, -8.0])
    x1, it1, _, stopped = oracle.cg(A, b, eps=1e-14, max_iter=1, recompute=0)
    assert it1[0] == 1 and stopped == 1
    np.testing.assert_allclose(x1[:, 0], [34.0 / 83.0, -136.0 / 83.0], rtol=4 * U, atol=0)
    x2, it2, rr, stopped = oracle.cg(A, b, eps=1e-14, max_iter=10, recompute=0)
    assert it2[0] == 2 and stopped == 0 and rr[0] <= 1e-14
    np.testing.assert_allclose(x2[:, 0], [2.0, -2.0], rtol=8 * U, atol=8 * U)


def test_cg_scaled_identity_one_step():
    b = np.random.default_rng(0).standard_normal(50)
    x, it, rr, stopped = oracle.cg(3.0 * np.eye(50), b, eps=1e-12)
    assert it[0] == 1 and stopped == 0
    np.testing.assert_allclose(x[:, 0], b / 3.0, rtol=4 * U, atol=0)


def test_cg_finite_termination_with_three_eigenvalues():
    # A with 3 distinct eigenvalues: the Krylov space is exhausted after 3 steps.
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.array([1.0, 2.5, 7.0])[rng.integers(0, 3, 60)]
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(60)
    x, it, rr, stopped = oracle.cg(A, b, eps=1e-10, recompute=0)
    assert stopped == 0 and it[0] == 3
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x[:, 0] - xs) <= 1e-12 * np.linalg.norm(xs)


def test_cg_error_a_norm_decreases():
    # CG minimises the A-norm of the error over a growing Krylov space.
    n = 120
    X, B = gp_inputs.gp_problem(n, seed=21, k=1)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    xs = np.linalg.solve(A, B[:, 0])
    prev = np.inf
    for m in range(1, 12):
        x, it, _, _ = oracle.cg(A, B, eps=1e-15, max_iter=m, recompute=0)
        assert it[0] == m
        e = x[:, 0] - xs
        en = float(e @ A @ e)
        assert en < prev
        prev = en


def test_cg_against_lapack_on_gp_matrix():
    n = 300
    X, B = gp_inputs.gp_problem(n, seed=22, k=3)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    x, it, rr, stopped = oracle.cg(A, B, eps=1e-12, recompute=50)
    assert stopped == 0 and np.all(rr <= 1e-12)
    xs = sla.solve(A, B, assume_a="pos")
    # ||x - x*|| <= ||r|| / lambda_min, lambda_min >= noise = 0.1
    for c in range(3):
        bound = 1e-12 * np.linalg.norm(B[:, c]) / 0.1 * 1.01 + 1e-13 * np.linalg.norm(xs[:, c])
        assert np.linalg.norm(x[:, c] - xs[:, c]) <= bound


def test_cg_recompute_every_step_is_true_residual():
    n = 150
    X, B = gp_inputs.gp_problem(n, seed=23, k=1)
    A = oracle.gp_assemble(X, 0.7, 1.0, 0.05)
    for m in (1, 4, 9):
        x, it, rr, _ = oracle.cg(A, B, eps=1e-15, max_iter=m, recompute=1)
        true = np.linalg.norm(B[:, 0] - A @ x[:, 0]) / np.linalg.norm(B[:, 0])
        assert abs(rr[0] - true) <= 1e-12 * max(true, 1e-3)


def test_cg_stopping_rule_first_crossing():
    n = 200
    X, B = gp_inputs.gp_problem(n, seed=24, k=1)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    eps = 1e-3
    x, it, rr, stopped = oracle.cg(A, B, eps=eps, recompute=0)
    assert stopped == 0 and rr[0] <= eps
    _, it1, rr1, stopped1 = oracle.cg(A, B, eps=eps, max_iter=int(it[0]) - 1, recompute=0)
    assert stopped1 == 1 and rr1[0] > eps  # one iteration fewer is not enough


def test_cg_starting_guess():
    A = np.array([[3.0, 2.0], [2.0, 6.0]])
    b = np.array([[2.0], [-8.0]])
    x, it, rr, stopped = oracle.cg(A, b, X0=np.array([[2.0], [-2.0]]), eps=1e-6)
    assert it[0] == 0 and rr[0] == 0.0 and stopped == 0
    assert np.array_equal(x[:, 0], [2.0, -2.0])


# ------------------------------------------- randomized backward error ---

def test_backward_error_estimate_probe_values_brute_force():
    # each probe's ||E z||^2 against E = A - L L^T formed explicitly (numpy)
    n = 90
    X, _ = gp_inputs.gp_problem(n, seed=31, k=1)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L, _ = oracle.cholesky(A)
    L1 = L.copy()
    L1[40, 7] += 1e-6  # a planted error
    Z = np.random.default_rng(3).standard_normal((n, 3))
    E = A - L1 @ L1.T
    est, num, den = oracle.backward_error_estimate(L1, Z, A=A)
    np.testing.assert_allclose(num, np.sum((E @ Z) ** 2), rtol=1e-9)
    np.testing.assert_allclose(den, np.sum((A @ Z) ** 2), rtol=1e-12)
    # the matrix-free GP path sees the same matrix
    est2, num2, den2 = oracle.backward_error_estimate(L1, Z, Xfeat=X, lengthscale=1.0, variance=1.0, noise=0.1)
    np.testing.assert_allclose([num2, den2], [num, den], rtol=1e-12)


def test_backward_error_estimate_is_unbiased():
    # with many Gaussian probes the estimate approaches the exact checker
    n = 120
    X, _ = gp_inputs.gp_problem(n, seed=32, k=1)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    L, _ = oracle.cholesky(A)
    L[70:, 3] += 1e-7
    exact = oracle.backward_error(A, L)
    Z = np.random.default_rng(4).standard_normal((n, 400))
    est, _, _ = oracle.backward_error_estimate(L, Z, A=A)
    ratio = est / exact
    # ||A Z||^2 / k estimates ||A||_F^2 as well; both are chi-square-like
    assert 0.8 <= ratio <= 1.25, ratio


# ------------------------------------- preconditioned CG (M = F F^T) ---

def test_pcg_hand_worked_first_step():
    # A = [[3, 2], [2, 6]], b = [2, -8], F = I (so M = I and x0 = M^-1 b = b).
    # By hand: r0 = b - A x0 = [12, 36] = z0 = p0, rho = 1440, q = A p0 =
    # [108, 240], p.q = 9936, alpha = 1440/9936 = 10/69, so
    # x1 = x0 + alpha p0 = [86/23, -64/23] and r1 = [-84/23, 28/23] (r1.r0 = 0);
    # the certificate with lam = 1 is |r1| / |x1| = sqrt(7840 / 11492).
    # Two steps reach the exact solution [2, -2].  With recompute = 1 the
    # periodic branch replaces r by b - A x after every step, which must not
    # change these values beyond rounding.
    A = np.array([[3.0, 2.0], [2.0, 6.0]])
    b = np.array([2.0, -8.0])
    for rc in (0, 1):
        x1, it1, ce1, failed = oracle.pcg(np.eye(2), A, b, lam=1.0, tol=1e-300, max_iter=1, recompute=rc)
        assert it1[0] == 1 and failed == 1
        np.testing.assert_allclose(x1[:, 0], [86.0 / 23.0, -64.0 / 23.0], rtol=8 * U, atol=0)
        assert abs(ce1[0] - np.sqrt(7840.0 / 11492.0)) <= 16 * U
        x2, it2, ce2, failed = oracle.pcg(np.eye(2), A, b, lam=1.0, tol=1e-14, max_iter=5, recompute=rc)
        assert failed == 0 and it2[0] == 2
        np.testing.assert_allclose(x2[:, 0], [2.0, -2.0], rtol=16 * U, atol=16 * U)


def _true_cert(A, b, x, lam):
    r = b.astype(np.longdouble) - A.astype(np.longdouble) @ x.astype(np.longdouble)
    xn = np.sqrt(np.sum(x.astype(np.longdouble) ** 2))
    return float(np.sqrt(np.sum(r * r)) / (lam * xn))


def test_pcg_recompute_branch_takes_true_residual():
    """The periodic recomputation (every `recompute` iterations) replaces the
    recurrence residual by b - A x: the certificate reported after a step
    that recomputes equals the one of the true residual (numpy, long double).
    Run far past the residual floor (80 steps, Jacobi preconditioner), the
    recurrence residual without recomputation drifts many orders below the
    true one; with the recomputation it stays on it."""
    n, lam = 150, 0.05
    X, B = gp_inputs.gp_problem(n, seed=23, k=1)
    A = oracle.gp_assemble(X, 0.7, 1.0, lam)
    F = np.diag(np.sqrt(np.diag(A)))  # M = diag(A): many iterations
    b = B[:, 0]
    for m in (3, 6, 9, 30):
        x, it, ce, _ = oracle.pcg(F, A, B, lam=lam, tol=1e-300, max_iter=m, recompute=3)
        assert it[0] == m
        t = _true_cert(A, b, x[:, 0], lam)
        assert abs(ce[0] - t) <= 1e-10 * t, (m, ce[0], t)
    # early iterates do not depend on the recomputation beyond rounding
    x3, _, _, _ = oracle.pcg(F, A, B, lam=lam, tol=1e-300, max_iter=9, recompute=3)
    x0, _, _, _ = oracle.pcg(F, A, B, lam=lam, tol=1e-300, max_iter=9, recompute=0)
    assert np.linalg.norm(x3 - x0) <= 1e-12 * np.linalg.norm(x0)
    # far past the floor: recomputed residual on the true one, recurrence off it
    m = 80
    xr, _, cr, _ = oracle.pcg(F, A, B, lam=lam, tol=1e-300, max_iter=m, recompute=m)
    tr = _true_cert(A, b, xr[:, 0], lam)
    assert abs(cr[0] - tr) <= 1e-2 * tr, (cr[0], tr)
    xn, _, cn, _ = oracle.pcg(F, A, B, lam=lam, tol=1e-300, max_iter=m, recompute=0)
    tn = _true_cert(A, b, xn[:, 0], lam)
    assert cn[0] <= 1e-3 * tn, (cn[0], tn)


def test_pcg_small_recompute_interval_against_lapack():
    """PCG with the true residual recomputed every second step converges to
    LAPACK's solution; the certificate bounds the true error."""
    n, lam = 300, 0.05
    X, B = gp_inputs.gp_problem(n, seed=24, k=2)
    A = oracle.gp_assemble(X, 0.7, 1.0, lam)
    F = np.diag(np.sqrt(np.diag(A)))
    xs, it, ce, failed = oracle.pcg(F, A, B, lam=lam, tol=1e-10, max_iter=2000, recompute=2)
    assert failed == 0 and np.all(it > 4)
    xnp = np.linalg.solve(A, B)
    for c in range(2):
        err = np.linalg.norm(xs[:, c] - xnp[:, c]) / np.linalg.norm(xnp[:, c])
        assert err <= 1e-10, (c, err)
        assert err <= ce[c] * np.linalg.norm(xs[:, c]) / np.linalg.norm(xnp[:, c]) * (1 + 1e-6) + 1e-15
