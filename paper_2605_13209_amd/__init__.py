"""MI355X-native dense SPD / Gaussian-process solver (blocked right-looking
Cholesky, forward/back substitution, mixed precision with iterative
refinement or factor-preconditioned CG, and a continuous-batching server).

The compute path is the HIP library ``libchol_mi355x.so`` (C ABI in
``include/chol.h``); this package is its thin binding plus host-side
orchestration.  Importing the package does not load the library; the first
call does, and raises if it is not built.
"""
from ._native import (CG_MAX_RHS, CgResult, cg_solve, cg_workspace_bytes,  # noqa: F401
                      CHOL_FP16_SCALED, CHOL_FP32, CHOL_FP64, CholError, Factor, RefineResult,
                      CHOL_FALLBACK_FP32, CHOL_FALLBACK_PCG, CHOL_FALLBACK_SHIFT,
                      chol_factor, chol_factor_bytes, chol_profile_read, chol_profile_reset, chol_factor_to_dense, chol_refine_bytes,
                      chol_refine_solve, chol_residual, chol_solve, chol_status_string, chol_tile_default,
                      colmajor_empty, get_option, gp_assemble, lib, set_option, to_colmajor,
                      chol_factor_hetero, chol_hetero_host_bytes, cg_solve_hetero, BatchEngine)
