"""GPU tests of the refinement drivers and their failure paths, through the C ABI.

* PCG (CG preconditioned with M = F F^T) step for step against the oracle's
  PCG: F is the exact factor L0 of a known-L0 matrix (the FP64 factorisation
  reproduces L0 bit for bit, pinned by the known-L0 tests), the system matrix
  a different SPD matrix (1000 x an SE kernel matrix), so the iteration is
  non-trivial.  Both sides compute in FP64 with different summation orders;
  over the first eight steps the iterates agree to ~1e-14 (measured between
  the oracle and a numpy PCG), so the bar is 1e-11.
* the periodic recomputation (option pcg_recompute) replaces the recurrence
  residual by the true one: far past the residual floor the reported
  certificate follows the true residual with it and drifts far below it
  without it (the same property the oracle's pin checks).
* IR stagnation falls back to PCG (CHOL_FALLBACK_PCG).
* the FP16 form's non-positive pivot: shifted retry, then FP32 factor.
* a failed factor whose info the host has not read: the solve writes NaN.
"""
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


def true_cert(A, b, x, lam):
    """||b - A x|| / (lam ||x||) with the residual exact (rational arithmetic,
    rounded once): at the residual floor of these systems b - A x cancels
    about 14 digits of |A||x|, more than a long-double sum keeps."""
    from fractions import Fraction
    xf = [Fraction(float(v)) for v in x]
    r = np.empty(len(b))
    for i in range(len(b)):
        s = Fraction(float(b[i]))
        for j, a in enumerate(A[i]):
            if a != 0.0:
                s -= Fraction(float(a)) * xf[j]
        r[i] = float(s)
    return float(np.linalg.norm(r) / (lam * np.linalg.norm(x)))


def pcg_problem(n=300, k=1):
    L0, A0 = gp_inputs.known_l0(n, "sparse-dd", seed=3)
    X, B = gp_inputs.gp_problem(n, seed=31, k=k)
    lam = 0.05
    Asys = 1000.0 * oracle.gp_assemble(X, 0.7, 1.0, lam)
    return L0, A0, Asys, B, 1000.0 * lam


class _Option:
    def __init__(self, key, value):
        self.key, self.value = key, value

    def __enter__(self):
        self.old = P.get_option(self.key)
        P.set_option(self.key, self.value)

    def __exit__(self, *exc):
        P.set_option(self.key, self.old)


@pytest.mark.parametrize("recompute", [0, 2, 3])
def test_pcg_steps_match_oracle(recompute):
    L0, A0, Asys, B, lam = pcg_problem()
    F = P.chol_factor(dev(A0), "fp64", 128)
    assert np.array_equal(np.tril(host(P.chol_factor_to_dense(F))), L0)
    Ad = dev(Asys)
    with _Option("pcg_recompute", recompute):
        for m in (1, 2, 3, 4, 6, 8):
            xo, it, ce, failed = oracle.pcg(L0, Asys, B, lam=lam, tol=1e-300, max_iter=m, recompute=recompute)
            assert it[0] == m and failed == 1
            res = P.chol_refine_solve(F, dev(B), A=Ad, noise=lam, tol=1e-300, max_iter=m, method="pcg",
                                      raise_on_fail=False)
            assert res.iters == m and not res.converged and res.fallback_used == 0
            x = host(res.X)[:, 0]
            err = np.linalg.norm(x - xo[:, 0]) / np.linalg.norm(xo[:, 0])
            assert err <= 1e-11, (recompute, m, err)
            assert abs(res.cert - ce[0]) <= 1e-9 * ce[0], (recompute, m, res.cert, ce[0])


def test_pcg_recompute_takes_true_residual():
    L0, A0, Asys, B, lam = pcg_problem()
    F = P.chol_factor(dev(A0), "fp64", 128)
    Ad = dev(Asys)
    b = B[:, 0]
    m = 120  # far past the residual floor (the certificate bottoms out near 1e-14 by step ~100)
    # recomputation at the last step: the reported certificate is the true one
    with _Option("pcg_recompute", m):
        res = P.chol_refine_solve(F, dev(B), A=Ad, noise=lam, tol=1e-300, max_iter=m, method="pcg",
                                  raise_on_fail=False)
    t = true_cert(Asys, b, host(res.X)[:, 0], lam)
    assert res.iters == m and abs(res.cert - t) <= 1e-2 * t, (res.cert, t)
    # without it the recurrence residual drifts many orders below the true one
    with _Option("pcg_recompute", 0):
        res0 = P.chol_refine_solve(F, dev(B), A=Ad, noise=lam, tol=1e-300, max_iter=m, method="pcg",
                                   raise_on_fail=False)
    t0 = true_cert(Asys, b, host(res0.X)[:, 0], lam)
    assert res0.cert <= 1e-3 * t0, (res0.cert, t0)


def test_pcg_converges_and_confirms_on_true_residual():
    L0, A0, Asys, B, lam = pcg_problem(k=3)
    F = P.chol_factor(dev(A0), "fp64", 128)
    res = P.chol_refine_solve(F, dev(B), A=dev(Asys), noise=lam, tol=1e-10, max_iter=500, method="pcg")
    assert res.converged and res.fallback_used == 0
    x = host(res.X)
    xo, it, ce, failed = oracle.pcg(L0, Asys, B, lam=lam, tol=1e-10, max_iter=500, recompute=50)
    assert failed == 0
    for c in range(3):
        assert true_cert(Asys, B[:, c], x[:, c], lam) <= 0.5e-10 * (1 + 1e-6)
        err = np.linalg.norm(x[:, c] - xo[:, c]) / np.linalg.norm(xo[:, c])
        assert err <= 2e-10, (c, err)


def test_ir_stagnation_falls_back_to_pcg():
    # M = L0 L0^T is far from A: the IR correction does not halve, so after
    # two such steps the call continues with PCG and still certifies 1e-10.
    L0, A0, Asys, B, lam = pcg_problem(k=2)
    F = P.chol_factor(dev(A0), "fp64", 128)
    res = P.chol_refine_solve(F, dev(B), A=dev(Asys), noise=lam, tol=1e-10, max_iter=500, method="ir")
    assert res.converged and res.fallback_used == P.CHOL_FALLBACK_PCG
    x = host(res.X)
    xs = np.linalg.solve(Asys, B)
    for c in range(2):
        assert true_cert(Asys, B[:, c], x[:, c], lam) <= 0.5e-10 * (1 + 1e-6)
        assert np.linalg.norm(x[:, c] - xs[:, c]) / np.linalg.norm(xs[:, c]) <= 1e-10


def test_ir_without_stagnation_keeps_ir():
    n, k = 1024, 2
    X, B = gp_inputs.gp_problem(n, seed=0, k=k)
    Xd = torch.from_numpy(X).cuda()
    Ad = P.gp_assemble(Xd, 1.0, 1.0, 0.1)
    F = P.chol_factor(Ad, "fp32", 128)
    res = P.chol_refine_solve(F, dev(B), A=Ad, noise=0.1, tol=1e-10, method="ir")
    assert res.converged and res.fallback_used == 0 and 1 <= res.iters <= 6


def test_ir_several_rhs_below_the_plain_residual_floor():
    """With several right-hand sides IR's working residuals are plain FP64;
    here their rounding (about sqrt(n) u |A||x|) lies far above the
    certificate's threshold (noise 1e-4), so the certifying residuals must
    be double-double: the call still certifies every column, and the
    certificate holds for the exactly computed residual."""
    n, k, noise = 512, 2, 1e-4
    X, B = gp_inputs.gp_problem(n, seed=7, k=k)
    A = oracle.gp_assemble(X, 1.0, 1.0, noise)
    Ad = dev(A)
    F = P.chol_factor(Ad, "fp32", 128)
    res = P.chol_refine_solve(F, dev(B), A=Ad, noise=noise, tol=1e-10, max_iter=200, method="ir")
    assert res.converged
    x = host(res.X)
    for c in range(k):
        assert true_cert(A, B[:, c], x[:, c], noise) <= 0.5e-10 * (1 + 1e-6)


def _fp16_failing_problem(noise):
    # smooth SE kernel (lengthscale 2): the smallest eigenvalue of the scaled
    # matrix is about the noise, far below the FP16 update's rounding error
    n = 512
    X, B = gp_inputs.gp_problem(n, seed=40, k=2)
    A = oracle.gp_assemble(X, 2.0, 1.0, noise)
    return A, B


def test_fp16_fails_then_fp32_fallback():
    A, B = _fp16_failing_problem(1e-3)
    Ad = dev(A)
    with _Option("fp16_shift_c", 0):
        F = P.chol_factor(Ad, "fp16_scaled", 128, panel_width=1)
    assert F.info() == 0 and F.fallback == P.CHOL_FALLBACK_FP32 and F.precision == P.CHOL_FP32
    # the factor is the FP32 one: same result as asking for FP32 directly
    F32 = P.chol_factor(Ad, "fp32", 128, panel_width=1)
    assert np.array_equal(host(P.chol_factor_to_dense(F)), host(P.chol_factor_to_dense(F32)))
    res = P.chol_refine_solve(F, dev(B), A=Ad, noise=1e-3, tol=1e-8, max_iter=200)
    assert res.converged and res.fallback_used & P.CHOL_FALLBACK_FP32
    L, info = oracle.cholesky(A)
    xref = oracle.solve(L, B)
    x = host(res.X)
    for c in range(2):
        assert np.linalg.norm(x[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c]) <= 2e-8


def test_fp16_shifted_retry():
    A, B = _fp16_failing_problem(1e-4)
    Ad = dev(A)
    with _Option("fp16_shift_c", 32):
        F = P.chol_factor(Ad, "fp16_scaled", 128, panel_width=1)
    assert F.info() == 0 and F.fallback & P.CHOL_FALLBACK_SHIFT
    res = P.chol_refine_solve(F, dev(B), A=Ad, noise=1e-4, tol=1e-6, max_iter=400)
    assert res.converged and res.fallback_used & P.CHOL_FALLBACK_SHIFT
    L, info = oracle.cholesky(A)
    xref = oracle.solve(L, B)
    x = host(res.X)
    for c in range(2):
        assert np.linalg.norm(x[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c]) <= 2e-6


def test_async_failed_factor_solve_is_nan():
    # a workspace that held a good factor, then an asynchronous factorisation
    # of a matrix that is not positive definite into it: the host has not read
    # info when it solves, so the solve must not return the old factor's
    # numbers; every entry becomes NaN, and so does the dense factor.
    n = 700
    X, B = gp_inputs.gp_problem(n, seed=8, k=3)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    ws = torch.empty(P.chol_factor_bytes(n, "fp64", 128), dtype=torch.uint8, device="cuda")
    Fg = P.chol_factor(dev(A), "fp64", 128, workspace=ws)
    Bd = dev(B)
    P.chol_solve(Fg, Bd)
    assert np.isfinite(host(Bd)).all()
    Abad = A.copy()
    Abad[400, 400] = -1.0
    Fb = P.chol_factor(dev(Abad), "fp64", 128, workspace=ws, sync=False)
    Bd = dev(B)
    P.chol_solve(Fb, Bd)
    assert np.isnan(host(Bd)).all()
    Lb = host(P.chol_factor_to_dense(Fb))
    assert np.isnan(Lb[np.tril_indices(n)]).all()
    assert Fb.info() == 401
    with pytest.raises(P.CholError):
        P.chol_solve(Fb, dev(B))


def test_solves_on_two_streams_share_a_factor():
    # the solves synchronise through words in the factor's workspace: solves
    # with one factor issued on two streams are ordered by the library
    n, k = 3000, 4
    X, B = gp_inputs.gp_problem(n, seed=9, k=k)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    xref = oracle.solve(oracle.cholesky(A)[0], B)
    F = P.chol_factor(dev(A), "fp64", 128)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for rep in range(6):
        st = s1 if rep % 2 == 0 else s2
        Bd = dev(B)
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            P.chol_solve(F, Bd, stream=st)
        outs.append((st, Bd))
    torch.cuda.synchronize()
    for _, Bd in outs:
        x = host(Bd)
        assert np.linalg.norm(x - xref) / np.linalg.norm(xref) <= 1e-10


def test_residual_is_double_double_accurate():
    """R = B - A X near a solution (|R| about 14 digits below |A||X|): the
    stored-matrix residual kernel accumulates in double-double, so each entry
    is within a few ulp of itself against the exact (rational) residual, not
    merely within u |A||X|."""
    from fractions import Fraction
    n, hp = 200, (0.7, 1.0, 0.05)
    X, B = gp_inputs.gp_problem(n, seed=41, k=2)
    A = oracle.gp_assemble(X, *hp)
    xs = np.asfortranarray(np.linalg.solve(A, B))
    U = np.finfo(np.float64).eps / 2
    R = host(P.chol_residual(dev(A), dev(xs), dev(B)))
    for c in range(2):
        xf = [Fraction(float(v)) for v in xs[:, c]]
        for i in range(n):
            s = Fraction(float(B[i, c]))
            for j in range(n):
                s -= Fraction(float(A[i, j])) * xf[j]
            ex = float(s)
            absAx = float(np.abs(A[i]) @ np.abs(xs[:, c]))
            assert abs(R[i, c] - ex) <= 2 * U * abs(ex) + 64 * n * U * U * absAx, (i, c, R[i, c], ex)
