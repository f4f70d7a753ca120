"""The heterogeneous CPU + GPU factorisation (chol_factor_hetero) against the
oracle: the factor of every split of the tile rows between CPU and GPU is the
same matrix to rounding (backward error <= 1e-12, factor within 1e-11 of the
oracle's), exact-arithmetic inputs give L0 bit for bit whatever the split,
info matches the oracle's wherever the failing pivot falls, and the handle
solves like any other."""
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


# (the CPU takes part when its first rows cover at least one panel: the
# largest m with m (m + 1) / 2 <= (1 - share) N (N + 1) / 2 is >= pw)
@pytest.mark.parametrize("n,share,pw", [(2048, 0.5, 8), (2048, 0.9, 2), (3000, 0.8, 4), (1900, 0.7, 1),
                                        (4096, 0.99, 2), (2048, 1.0, 8), (1024, 0.0, 8)])
def test_hetero_factor_matches_oracle(n, share, pw):
    X, Bm = gp_inputs.gp_problem(n, seed=21, k=2)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    F, rep = P.chol_factor_hetero(dev(A), share, panel_width=pw)
    assert F.info() == 0
    L = host(P.chol_factor_to_dense(F))
    Lref, info = oracle.cholesky(A)
    assert info == 0
    assert oracle.backward_error(A, L) <= 1e-12
    assert np.linalg.norm(L - Lref) / np.linalg.norm(Lref) <= 1e-11
    Bd = dev(Bm)
    P.chol_solve(F, Bd)
    xref = oracle.solve(Lref, Bm)
    x = host(Bd)
    assert np.linalg.norm(x - xref) / np.linalg.norm(xref) <= 1e-10
    # the split that ran
    if share < 1.0:
        assert rep["cpu_tile_updates"] > 0
    else:
        assert rep["cpu_tile_updates"] == 0 and rep["handover_column"] == 0
    assert 0.0 <= rep["gpu_share_tiles"] <= 1.0


@pytest.mark.parametrize("share", [0.3, 0.6, 0.85])
def test_hetero_known_l0_exact(share):
    # integers below 2^53 and power-of-two pivots: the CPU's and the GPU's
    # substitutions both reproduce L0 exactly, wherever the border runs
    L0, A0 = gp_inputs.known_l0(2000, "dense-int", seed=2)
    F, rep = P.chol_factor_hetero(dev(A0), share, panel_width=2)
    assert F.info() == 0
    assert np.array_equal(np.tril(host(P.chol_factor_to_dense(F))), L0)
    assert rep["border_shifts"] >= 1


@pytest.mark.parametrize("col", [5, 300, 1500])
def test_hetero_info_matches_oracle(col):
    # a non-positive pivot in the CPU's first rows (5), in rows the CPU takes
    # over later (300), and in the part the GPU finishes alone (1500)
    n = 1700
    X, _ = gp_inputs.gp_problem(n, seed=22)
    A = oracle.gp_assemble(X, 1.0, 1.0, 0.1)
    A[col, col] = -1.0
    _, info_ref = oracle.cholesky(A)
    F, rep = P.chol_factor_hetero(dev(A), 0.6, panel_width=2, raise_not_spd=False)
    assert F.info() == info_ref == col + 1


def test_hetero_report_tracks_the_target():
    n = 8192
    X, _ = gp_inputs.gp_problem(n, seed=23)
    Ad = P.gp_assemble(torch.from_numpy(X).cuda(), 1.0, 1.0, 0.1, full=False)
    for share in (0.6, 0.9):
        F, rep = P.chol_factor_hetero(Ad, share)
        assert F.info() == 0
        assert abs(rep["gpu_share_tiles"] - share) <= 0.08, rep
        assert rep["bytes_h2d"] > 0 and rep["bytes_d2h"] > 0
