"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (each derived from the arithmetic of the step it checks):
* integer / exact-arithmetic cases (known L0): bit-exact;
* GP assembly: entries within 4 ulp (only exp differs; sums are unfused);
* FP64 factor: backward error ||A - L L^T||_F / ||A||_F <= 1e-12, and the
  factor within 1e-11 relative (Frobenius) of the oracle's;
* FP64 solve: relative error <= 1e-10 against the oracle solve;
* mixed precision + refinement: relative error <= 1e-10 against the oracle's
  refined FP64 solution, and certified by ||r|| / (noise ||x||).
"""
import numpy as np
import pytest
import torch

import gp_inputs
import oracle
import paper_2605_13209_amd as P

pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps / 2


def dev(a):
    return P.to_colmajor(torch.from_numpy(np.asarray(a)))


def host(t):
    return t.detach().cpu().numpy()


def gpu_factor_dense(A_np, precision="fp64", tile=0):
    A = dev(A_np)
    F = P.chol_factor(A, precision, tile)
    L = host(P.chol_factor_to_dense(F))
    return F, L


# ------------------------------------------------------------- assembly ---

@pytest.mark.parametrize("n,d,hp", [(1, 8, (1.0, 1.0, 0.1)), (300, 8, (1.0, 1.0, 0.1)),
                                    (257, 3, (0.5, 2.0, 1.0)), (130, 20, (2.0, 1.0, 0.01))])
def test_gp_assemble_matches_oracle(n, d, hp):
    X, _ = gp_inputs.gp_problem(n, d=d, seed=n)
    ref = oracle.gp_assemble(X, *hp)
    A = host(P.gp_assemble(torch.from_numpy(X).cuda(), *hp, full=True))
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == hp[1] + hp[2])
    np.testing.assert_allclose(A, ref, rtol=4 * U * 2, atol=0)


def test_gp_assemble_lower_only_leaves_upper():
    n = 200
    X, _ = gp_inputs.gp_problem(n, seed=1)
    A = P.colmajor_empty(n, n)
    A.fill_(-7.0)
    P.gp_assemble(torch.from_numpy(X).cuda(), 1.0, 1.0, 0.1, full=False, out=A)
    a = host(A)
    iu = np.triu_indices(n, 1)
    assert np.all(a[iu] == -7.0)
    ref = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    il = np.tril_indices(n)
    np.testing.assert_allclose(a[il], ref[il], rtol=8 * U, atol=0)


# ----------------------------------------------------- exact known-L0 ---

@pytest.mark.parametrize("n,tile,family", [(64 * 3 + 17, 64, "dense-int"), (128 * 5 + 3, 128, "dense-int"),
                                           (777, 128, "sparse-dd"), (256, 128, "dense-int"), (1, 64, "dense-int")])
def test_known_l0_exact_fp64(n, tile, family):
    L0, A = gp_inputs.known_l0(n, family, seed=n)
    F, L = gpu_factor_dense(A, "fp64", tile)
    assert F.info() == 0
    np.testing.assert_array_equal(L, L0)
    F.free()


@pytest.mark.parametrize("n,tile", [(300, 64), (700, 128)])
def test_known_l0_exact_fp32(n, tile):
    L0, A = gp_inputs.known_l0(n, "small-int", seed=n)
    assert np.abs(A).max() < 2**24
    _, L = gpu_factor_dense(A, "fp32", tile)
    np.testing.assert_array_equal(L, L0)


def test_known_l0_exact_solve():
    n = 500
    L0, A = gp_inputs.known_l0(n, "sparse-dd", seed=3)
    x0 = np.random.default_rng(2).integers(-3, 4, size=(n, 5)).astype(np.float64)
    b = A @ x0  # exact integers
    F = P.chol_factor(dev(A), "fp64", 128)
    B = dev(b)
    P.chol_solve(F, B)
    # forward/back substitution with an exact L0 (diagonal 32) is exact for sparse-dd
    np.testing.assert_allclose(host(B), x0, rtol=0, atol=1e-12)


# -------------------------------------------------------- GP factors ---

@pytest.mark.parametrize("n,tile", [(1024, 128), (1000, 128), (300, 64), (1000, 64), (129, 128), (2, 64)])
def test_fp64_factor_parity(n, tile):
    X, _ = gp_inputs.gp_problem(n, seed=0)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    Lref, info = oracle.cholesky(A)
    assert info == 0
    F, L = gpu_factor_dense(A, "fp64", tile)
    assert F.info() == 0
    assert np.all(np.triu(L, 1) == 0)
    be = oracle.backward_error(A, L)
    assert be <= 1e-12, be
    rel = np.linalg.norm(L - Lref) / np.linalg.norm(Lref)
    assert rel <= 1e-11, rel


@pytest.mark.parametrize("k", [1, 16])
def test_fp64_solve_parity(k):
    n = 1024
    X, B = gp_inputs.gp_problem(n, seed=0, k=k)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    Lref, _ = oracle.cholesky(A)
    xref = oracle.solve(Lref, B)
    F = P.chol_factor(dev(A), "fp64", 128)
    Bd = dev(B)
    P.chol_solve(F, Bd)
    x = host(Bd)
    for c in range(k):
        err = np.linalg.norm(x[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c])
        assert err <= 1e-10, (c, err)


@pytest.mark.parametrize("n,tile", [(1000, 128), (333, 64), (1000, 64)])
def test_fp32_factor_backward_error(n, tile):
    X, _ = gp_inputs.gp_problem(n, seed=5)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    Lref, _ = oracle.cholesky(A)
    _, L = gpu_factor_dense(A, "fp32", tile)
    be = oracle.backward_error(A, L)
    # FP32 storage and update: backward error of order n u_32 at most
    assert be <= 5e-6, be
    assert np.linalg.norm(L - Lref) / np.linalg.norm(Lref) <= 1e-3


def test_not_spd_info_matches_oracle():
    n = 300
    X, _ = gp_inputs.gp_problem(n, seed=7)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    A[200, 200] = -5.0
    _, info_ref = oracle.cholesky(A)
    assert info_ref == 201
    for prec, tile in [("fp64", 64), ("fp64", 128), ("fp32", 128)]:
        F = P.chol_factor(dev(A), prec, tile, sync=False)
        assert F.info() == info_ref, (prec, tile, F.info())
        with pytest.raises(P.CholError):
            P.chol_solve(F, dev(np.ones((n, 1))))
    A2 = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    A2[17, 3] = np.nan
    _, info2 = oracle.cholesky(A2)
    F = P.chol_factor(dev(A2), "fp64", 64, sync=False)
    assert F.info() == info2


@pytest.mark.parametrize("n,tile", [(1300, 128), (1000, 64)])
def test_schedule_invariance_bitwise(n, tile):
    """Panel width and lookahead change the schedule, not the arithmetic
    (tile 64: the one-wave-per-tile matrix-core update, ragged last tile row)."""
    X, _ = gp_inputs.gp_problem(n, seed=3)
    A = dev(oracle.gp_assemble(X, 1.0, 1.0, 0.1))
    outs = []
    try:
        # po: in-panel updates right-looking (1), left-looking (2) or recursive (3)
        for w, la, fw, po in [(1, 0, 0, 1), (2, 1, 0, 2), (4, 1, 0, 1), (4, 1, 0, 2), (3, 0, 0, 2),
                              (8, 1, 0, 1), (8, 1, 0, 2), (6, 0, 0, 1), (16, 1, 0, 2), (8, 1, 2, 2),
                              (4, 1, 1, 1), (8, 0, 3, 2), (8, 1, 0, 3), (6, 0, 0, 3), (7, 1, 0, 3),
                              (3, 1, 2, 3)]:
            P.set_option("panel_width", w)
            P.set_option("lookahead", la)
            P.set_option("first_panel_width", fw)
            P.set_option("panel_order", po)
            for prec in ("fp64", "fp32"):
                F = P.chol_factor(A, prec, tile)
                outs.append((prec, host(P.chol_factor_to_dense(F))))
    finally:
        P.set_option("panel_width", 0)
        P.set_option("lookahead", 1)
        P.set_option("first_panel_width", 0)
        P.set_option("panel_order", 0)
    for prec in ("fp64", "fp32"):
        ref = [L for p, L in outs if p == prec]
        for L in ref[1:]:
            assert np.array_equal(L, ref[0])


@pytest.mark.parametrize("n,tile", [(1300, 128), (1000, 64)])
def test_trsm_split_bitwise(n, tile):
    """Panel solves split over four workgroups per tile (a quarter of the rows
    each) give the same factor as whole-tile panel solves, and the inverted
    diagonal blocks split the same way give the same solves."""
    X, Bm = gp_inputs.gp_problem(n, seed=9, k=3)
    A = dev(oracle.gp_assemble(X, 1.0, 1.0, 0.1))
    old = P.get_option("trsm_split")
    try:
        for prec in ("fp64", "fp32"):
            Ls, Xs = [], []
            for split in (0, 1 << 20, 3):
                P.set_option("trsm_split", split)
                F = P.chol_factor(A, prec, tile)
                assert F.info() == 0
                Ls.append(host(P.chol_factor_to_dense(F)))
                Xs.append(host(P.chol_solve(F, dev(Bm))))
            assert np.array_equal(Ls[0], Ls[1]) and np.array_equal(Ls[0], Ls[2])
            assert np.array_equal(Xs[0], Xs[1]) and np.array_equal(Xs[0], Xs[2])
    finally:
        P.set_option("trsm_split", old)


@pytest.mark.parametrize("n,tile", [(1300, 128), (1000, 64)])
def test_potrf_lookahead_bitwise(n, tile):
    """Diagonal-tile factorisation with the fifth-wave lookahead gives the
    same factor as without it (FP64 and FP32), and reports the same failed
    pivot."""
    X, _ = gp_inputs.gp_problem(n, seed=11)
    A_h = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    A = dev(A_h)
    Abad_h = A_h.copy()
    Abad_h[n - 37, n - 37] = -1.0
    _, info_ref = oracle.cholesky(Abad_h)
    Abad = dev(Abad_h)
    old = P.get_option("potrf_lookahead")
    try:
        for prec in ("fp64", "fp32"):
            Ls, infos = [], []
            for la in (0, 1):
                P.set_option("potrf_lookahead", la)
                F = P.chol_factor(A, prec, tile)
                assert F.info() == 0
                Ls.append(host(P.chol_factor_to_dense(F)))
                infos.append(P.chol_factor(Abad, prec, tile, sync=False).info())
            assert np.array_equal(Ls[0], Ls[1])
            assert infos[0] == infos[1] == info_ref, (prec, infos, info_ref)
    finally:
        P.set_option("potrf_lookahead", old)


def test_repeatable_bitwise():
    n = 900
    X, _ = gp_inputs.gp_problem(n, seed=4)
    A = dev(oracle.gp_assemble(X, 1.0, 1.0, 0.1))
    L1 = host(P.chol_factor_to_dense(P.chol_factor(A, "fp64", 128)))
    L2 = host(P.chol_factor_to_dense(P.chol_factor(A, "fp64", 128)))
    assert np.array_equal(L1, L2)


# ------------------------------------------------------------ residual ---

@pytest.mark.parametrize("k", [1, 3, 9])
def test_residual_matches_oracle(k):
    n = 517
    X, B = gp_inputs.gp_problem(n, seed=9, k=k)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    xs = np.asfortranarray(np.random.default_rng(1).standard_normal((n, k)))
    ref = oracle.residual(A, xs, B)
    Ad = dev(A)
    # lower triangle only is read: poison the upper part
    a = Ad.clone()
    iu = torch.triu_indices(n, n, 1)
    a[iu[0], iu[1]] = float("nan")
    R = host(P.chol_residual(a, dev(xs), dev(B)))
    scale = np.abs(A) @ np.abs(xs) + np.abs(B)
    assert np.all(np.abs(R - ref) <= 4 * U * scale)


# ------------------------------------------------- mixed precision + IR ---

@pytest.mark.parametrize("method", ["ir", "pcg"])
@pytest.mark.parametrize("matrix_free", [False, True])
def test_fp32_refine_parity(method, matrix_free):
    n, k = 1024, 3
    X, B = gp_inputs.gp_problem(n, seed=0, k=k)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    Lref, _ = oracle.cholesky(A)
    xref, _, _, failed = oracle.refine(Lref, A, B, lam=0.1, tol=1e-13)
    assert failed == 0
    Xd = torch.from_numpy(X).cuda()
    Ad = P.gp_assemble(Xd, 1.0, 1.0, 0.1)
    F = P.chol_factor(Ad, "fp32", 128)
    kw = dict(X_feat=Xd) if matrix_free else dict(A=Ad)
    res = P.chol_refine_solve(F, dev(B), lengthscale=1.0, variance=1.0, noise=0.1, tol=1e-10,
                              method=method, **kw)
    assert res.converged and res.cert <= 0.5e-10
    assert res.iters >= 1
    x = host(res.X)
    for c in range(k):
        err = np.linalg.norm(x[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c])
        assert err <= 1e-10, (c, err)
        # the reported certificate bounds the true error
        r = oracle.residual(A, x[:, c], B[:, c])
        assert oracle.certificate(r, x[:, c], 0.1) <= 1e-10


def test_fp64_refine_converges_immediately():
    n = 600
    X, B = gp_inputs.gp_problem(n, seed=2, k=2)
    Xd = torch.from_numpy(X).cuda()
    Ad = P.gp_assemble(Xd, 1.0, 1.0, 0.1)
    F = P.chol_factor(Ad, "fp64", 128)
    res = P.chol_refine_solve(F, dev(B), A=Ad, noise=0.1, tol=1e-10)
    assert res.converged and res.iters == 0


@pytest.mark.parametrize("n,tile,k", [(1000, 128, 1), (1000, 128, 3), (1000, 128, 37),
                                      (300, 64, 5), (130, 128, 2), (2000, 128, 16)])
def test_solve_shapes_parity(n, tile, k):
    # ragged last tile, every right-hand-side chunk width (1, 4, 16 and a
    # partial chunk), both tile sizes
    X, B = gp_inputs.gp_problem(n, seed=5, k=k)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    Lref, _ = oracle.cholesky(A)
    xref = oracle.solve(Lref, B)
    F = P.chol_factor(dev(A), "fp64", tile)
    Bd = dev(B)
    P.chol_solve(F, Bd)
    x = host(Bd)
    for c in range(k):
        err = np.linalg.norm(x[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c])
        assert err <= 1e-10, (c, err)


def test_solve_bounded_wait_never_hangs():
    # With a one-poll bound the inter-workgroup waits give up almost at once:
    # the solve must still finish, and every row is either right or NaN.
    # Afterwards (default bound) the same solve is exact again.
    n = 2048
    X, B = gp_inputs.gp_problem(n, seed=6, k=2)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    xref = oracle.solve(oracle.cholesky(A)[0], B)
    F = P.chol_factor(dev(A), "fp64", 128)
    old = P.get_option("solve_spin_max")
    try:
        P.set_option("solve_spin_max", 1)
        Bd = dev(B)
        P.chol_solve(F, Bd)
        x = host(Bd)
    finally:
        P.set_option("solve_spin_max", old)
    ok = np.isnan(x) | (np.abs(x - xref) <= 1e-8 * np.abs(xref).max())
    assert ok.all()
    Bd = dev(B)
    P.chol_solve(F, Bd)
    x = host(Bd)
    assert np.isfinite(x).all()
    assert np.linalg.norm(x - xref) / np.linalg.norm(xref) <= 1e-10


def test_full_size_sampled_parity():
    """The bench configuration (n = 32768, tile 128, automatic schedule: panel
    width 8, lookahead) checked where the oracle can follow it: sampled
    entries of L L^T against the oracle's A_ij, within the classical
    componentwise bound (n+1)u/(1-(n+1)u) |L||L^T|; the backward error of the
    whole factor by the oracle's randomized estimate (<= 1e-12); and the k = 1
    solve through the oracle's matrix-free residual and rigorous certificate."""
    n = 32768
    X, B = gp_inputs.gp_problem(n, seed=0, k=1)
    hp = (1.0, 1.0, 0.1)
    Ad = P.gp_assemble(torch.from_numpy(X).cuda(), *hp, full=False)
    F = P.chol_factor(Ad, "fp64", 128)
    assert F.info() == 0
    Ld = P.chol_factor_to_dense(F)
    rng = np.random.default_rng(7)
    pairs = [(int(i), int(rng.integers(0, i + 1))) for i in rng.integers(0, n, size=48)]
    pairs += [(n - 1, n - 1), (n - 1, 0), (128, 127), (0, 0)]
    rows = sorted({r for pr in pairs for r in pr})
    Lrows = {r: host(Ld[r, :]).astype(np.float64) for r in rows}
    gam = (n + 1) * U / (1 - (n + 1) * U)
    for i, j in pairs:
        li, lj = Lrows[i][: j + 1], Lrows[j][: j + 1]
        s = float(np.sum(li.astype(np.longdouble) * lj.astype(np.longdouble)))
        a = oracle.gp_entry(X, i, j, *hp)
        # plus the assembly difference (exp within a few ulp of the oracle's)
        bound = gam * float(np.sum(np.abs(li) * np.abs(lj))) + 8 * U * abs(a)
        assert abs(s - a) <= bound, (i, j, s, a, bound)
    assert np.all(host(Ld[0, 1:64]) == 0.0)  # upper triangle written as zero
    # the whole factor: Hutchinson estimate of ||A - L L^T||_F / ||A||_F with
    # A matrix-free from the features (4 Gaussian probes, long double)
    Lh = host(Ld)
    Z = np.random.default_rng(11).standard_normal((n, 4))
    est, _, _ = oracle.backward_error_estimate(Lh, Z, Xfeat=X, lengthscale=hp[0], variance=hp[1], noise=hp[2])
    assert est <= 1e-12, est
    del Ld, Lh
    Bd = dev(B)
    P.chol_solve(F, Bd)
    x = host(Bd)[:, 0]
    r = oracle.gp_residual(X, *hp, x, B[:, 0])
    assert oracle.certificate(r, x, hp[2]) <= 1e-10


def test_full_size_fp64_n65536():
    """The headline FP64 configuration (n = 65536, tile 128, automatic
    schedule), the first FP64 order whose packed element offsets pass 2^31:
    sampled entries of L L^T against the oracle's A_ij within the
    componentwise bound, the randomized backward error of the whole factor
    (A matrix-free from the features, long double) <= 1e-12, and the k = 1
    solve certified to 1e-10 by the oracle's matrix-free residual."""
    torch.cuda.empty_cache()
    n = 65536
    X, B = gp_inputs.gp_problem(n, seed=0, k=1)
    hp = (1.0, 1.0, 0.1)
    Ad = P.gp_assemble(torch.from_numpy(X).cuda(), *hp, full=False)
    F = P.chol_factor(Ad, "fp64", 128)
    assert F.info() == 0
    del Ad
    torch.cuda.empty_cache()
    Ld = P.chol_factor_to_dense(F)
    rng = np.random.default_rng(17)
    pairs = [(int(i), int(rng.integers(0, i + 1))) for i in rng.integers(0, n, size=48)]
    # entries whose packed offsets lie past 2^31 elements, the last tile, a tile edge
    pairs += [(n - 1, n - 1), (n - 1, 0), (n - 1, n - 200), (60000, 59000), (50000, 30000), (255, 128)]
    rows = sorted({r for pr in pairs for r in pr})
    Lrows = {r: host(Ld[r, :]).astype(np.float64) for r in rows}
    gam = (n + 1) * U / (1 - (n + 1) * U)
    for i, j in pairs:
        li, lj = Lrows[i][: j + 1], Lrows[j][: j + 1]
        s = float(np.sum(li.astype(np.longdouble) * lj.astype(np.longdouble)))
        a = oracle.gp_entry(X, i, j, *hp)
        bound = gam * float(np.sum(np.abs(li) * np.abs(lj))) + 8 * U * abs(a)
        assert abs(s - a) <= bound, (i, j, s, a, bound)
    Lh = host(Ld)
    del Ld
    torch.cuda.empty_cache()
    Z = np.random.default_rng(19).standard_normal((n, 2))
    est, _, _ = oracle.backward_error_estimate(Lh, Z, Xfeat=X, lengthscale=hp[0], variance=hp[1], noise=hp[2])
    del Lh
    assert est <= 1e-12, est
    Bd = dev(B)
    P.chol_solve(F, Bd)
    x = host(Bd)[:, 0]
    r = oracle.gp_residual(X, *hp, x, B[:, 0])
    assert oracle.certificate(r, x, hp[2]) <= 1e-10
    del F
    torch.cuda.empty_cache()


def test_full_size_mixed_fp32_n65536():
    """The mixed-precision bench configuration (n = 65536, SE lengthscale 1,
    noise 0.1, one right-hand side, FP32 factor, FP64 A for the residuals):
    IR and factor-preconditioned CG both reach the 1e-10 certificate as
    recomputed by the oracle from the features (matrix-free residual, long
    double), and agree with each other within the sum of their bounds."""
    torch.cuda.empty_cache()
    n = 65536
    hp = (1.0, 1.0, 0.1)
    X, B = gp_inputs.gp_problem(n, seed=0, k=1)
    Ad = P.gp_assemble(torch.from_numpy(X).cuda(), *hp, full=False)
    F = P.chol_factor(Ad, "fp32", 128)
    assert F.info() == 0
    xs = {}
    for method in ("ir", "pcg"):
        r = P.chol_refine_solve(F, dev(B), A=Ad, noise=hp[2], tol=1e-10, method=method, max_iter=60)
        assert r.converged and r.cert <= 1e-10, (method, r.iters, r.cert)
        x = host(r.X)[:, 0]
        res = oracle.gp_residual(X, *hp, x, B[:, 0])
        assert oracle.certificate(res, x, hp[2]) <= 1e-10, method
        xs[method] = x
    gap = np.linalg.norm(xs["ir"] - xs["pcg"]) / np.linalg.norm(xs["ir"])
    assert gap <= 2e-10, gap
    del F, Ad
    torch.cuda.empty_cache()


def test_full_size_mixed_fp16_n131072():
    """The FP16 bench configuration (n = 131072, SE lengthscale 0.5, noise 1,
    eight right-hand sides; diagonally scaled FP16 update, FP32 storage, IR
    against the FP64 A): every column certified to 1e-10 by the oracle's
    matrix-free residual."""
    torch.cuda.empty_cache()
    n, k = 131072, 8
    hp = (0.5, 1.0, 1.0)
    X, B = gp_inputs.gp_problem(n, d=8, k=k, seed=0)
    Ad = P.colmajor_empty(n, n)
    P.gp_assemble(torch.from_numpy(X).cuda(), *hp, full=False, out=Ad)
    F = P.chol_factor(Ad, "fp16_scaled", 128)
    assert F.info() == 0
    r = P.chol_refine_solve(F, dev(B), A=Ad, noise=hp[2], tol=1e-10, method="ir", max_iter=60)
    assert r.converged and r.cert <= 1e-10, (r.iters, r.cert)
    x = host(r.X)
    del F, Ad, r
    torch.cuda.empty_cache()
    res = oracle.gp_residual(X, *hp, x, B)
    for c in range(k):
        assert oracle.certificate(res[:, c], x[:, c], hp[2]) <= 1e-10, c


# ----------------------------------------------------------- edge cases ---

def test_empty_and_tiny():
    F = P.chol_factor(P.colmajor_empty(0, 0), "fp64", 64)
    assert F.info() == 0 and F.n == 0
    A = dev(np.array([[4.0]]))
    F = P.chol_factor(A, "fp64", 64)
    L = host(P.chol_factor_to_dense(F))
    assert L[0, 0] == 2.0
    B = dev(np.array([[6.0, -2.0]]))
    P.chol_solve(F, B)
    np.testing.assert_array_equal(host(B), [[1.5, -0.5]])


def test_workspace_too_small_rejected():
    A = dev(np.eye(100))
    need = P.chol_factor_bytes(100, "fp64", 64)
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.CholError) as e:
        P.chol_factor(A, "fp64", 64, workspace=ws)
    assert e.value.status == -101


# ------------------------------------------------- scaled FP16 + refinement ---

def test_fp16_scaled_factor_and_refine():
    """FP16 operands / FP32 accumulation on H = A / s; refined to 1e-10 (well-conditioned GP)."""
    n, k = 1000, 2
    X, B = gp_inputs.gp_problem(n, seed=3, k=k)
    hp = (0.5, 1.0, 1.0)
    A = oracle.gp_assemble(X, *hp)
    Lref, _ = oracle.cholesky(A)
    xref, _, _, failed = oracle.refine(Lref, A, B, lam=hp[2], tol=1e-13)
    assert failed == 0
    Xd = torch.from_numpy(X).cuda()
    Ad = P.gp_assemble(Xd, *hp)
    F = P.chol_factor(Ad, "fp16_scaled", 128)
    L = host(P.chol_factor_to_dense(F))
    be = oracle.backward_error(A, L)
    assert be <= 5e-3, be  # of order u_16 = 4.9e-4 times modest growth
    for method in ("ir", "pcg"):
        res = P.chol_refine_solve(F, dev(B), A=Ad, noise=hp[2], tol=1e-10, method=method, max_iter=60)
        assert res.converged, (method, res.iters, res.cert)
        x = host(res.X)
        for c in range(k):
            err = np.linalg.norm(x[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c])
            assert err <= 1e-10, (method, c, err)


@pytest.mark.parametrize("pw,n", [(2, 1300), (3, 1300), (16, 2250), (32, 4500)])
def test_fp16_scaled_lookahead_invariance(pw, n):
    # the two FP16 panel buffers alternate between panels; with and without
    # lookahead (ragged n, a partial last panel), with right- and left-looking
    # in-panel updates, the factors are identical; width 32 (the FP16 form's
    # widest: 64 chunks of 64 columns per tile row) with a full first panel
    X, _ = gp_inputs.gp_problem(n, seed=4)
    Ad = P.gp_assemble(torch.from_numpy(X).cuda(), 0.5, 1.0, 1.0)
    Ls = []
    try:
        for la, po in ((0, 1), (1, 1), (0, 2), (1, 2), (1, 3)):
            P.set_option("panel_order", po)
            F = P.chol_factor(Ad, "fp16_scaled", 128, panel_width=pw, lookahead=la)
            assert F.info() == 0
            Ls.append(host(P.chol_factor_to_dense(F)))
    finally:
        P.set_option("panel_order", 0)
    for L in Ls[1:]:
        assert np.array_equal(Ls[0], L)
    be = oracle.backward_error(oracle.gp_assemble(X, 0.5, 1.0, 1.0), Ls[0])
    assert be <= 5e-3, be


def test_fp16_wide_update_bitwise():
    """The 2 x 2-tile FP16 trailing update (used from 16 trailing tile rows)
    gives the same factor, bit for bit, as the one-tile kernel, with and
    without lookahead (ragged n: a partial last super-tile row)."""
    n = 4100
    X, _ = gp_inputs.gp_problem(n, seed=6)
    Ad = P.gp_assemble(torch.from_numpy(X).cuda(), 0.5, 1.0, 1.0)
    Ls = []
    try:
        for wide, la in ((0, 1), (1, 1), (1, 0)):
            P.set_option("f16_wide", wide)
            F = P.chol_factor(Ad, "fp16_scaled", 128, panel_width=4, lookahead=la)
            assert F.info() == 0
            Ls.append(host(P.chol_factor_to_dense(F)))
    finally:
        P.set_option("f16_wide", 1)
    assert np.array_equal(Ls[0], Ls[1]) and np.array_equal(Ls[1], Ls[2])
    be = oracle.backward_error(oracle.gp_assemble(X, 0.5, 1.0, 1.0), Ls[1])
    assert be <= 5e-3, be


def test_fp16_scaled_solve_scaling():
    """chol_solve with the scaled factor returns A^-1 b (not H^-1 b)."""
    n = 600
    X, B = gp_inputs.gp_problem(n, seed=4, k=1)
    hp = (0.5, 2.0, 1.0)  # diagonal 3: a non-trivial scale
    A = oracle.gp_assemble(X, *hp)
    xnp = np.linalg.solve(A, B)
    F = P.chol_factor(dev(A), "fp16_scaled", 128)
    Bd = dev(B)
    P.chol_solve(F, Bd)
    err = np.linalg.norm(host(Bd) - xnp) / np.linalg.norm(xnp)
    assert err <= 5e-2, err


# ------------------------------------------------------------ HIP graphs ---

@pytest.mark.parametrize("n", [1024, 1300])
def test_graph_replay_bitwise(n):
    """Captured factorisation replayed several times, with eager work and
    synchronisations in between; every replay equals the eager factor, and a
    replay after A changed equals the eager factor of the new A."""
    X, _ = gp_inputs.gp_problem(n, seed=11)
    A = dev(oracle.gp_assemble(X, 1.0, 1.0, 0.1))
    s = torch.cuda.Stream()
    need = P.chol_factor_bytes(n, "fp64", 128)
    ws_g = torch.empty(need, dtype=torch.uint8, device="cuda")
    ws_e = torch.empty(need, dtype=torch.uint8, device="cuda")
    with torch.cuda.stream(s):
        L_eager = host(P.chol_factor_to_dense(P.chol_factor(A, "fp64", 128, workspace=ws_e, graph=0, stream=s),
                                              stream=s))
        for rep in range(4):
            F = P.chol_factor(A, "fp64", 128, workspace=ws_g, graph=1, stream=s)
            assert F.info() == 0
            L = host(P.chol_factor_to_dense(F, stream=s))
            assert np.array_equal(L, L_eager), rep
            # eager work between replays
            P.chol_factor(A, "fp64", 128, workspace=ws_e, graph=0, stream=s)
            torch.cuda.synchronize()
        A2 = dev(oracle.gp_assemble(X, 0.7, 1.0, 0.2))
        A.copy_(A2)
        torch.cuda.synchronize()
        L2_eager = host(P.chol_factor_to_dense(P.chol_factor(A, "fp64", 128, workspace=ws_e, graph=0,
                                                             stream=s), stream=s))
        F = P.chol_factor(A, "fp64", 128, workspace=ws_g, graph=1, stream=s)
        assert np.array_equal(host(P.chol_factor_to_dense(F, stream=s)), L2_eager)
