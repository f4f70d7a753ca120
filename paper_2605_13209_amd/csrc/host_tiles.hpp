// Host (CPU) side of the heterogeneous factorisation: FP64 kernels on the
// same 128 x 128 column-major tiles as the device path, and a small thread
// pool that runs them.  These are product kernels for the CPU share of the
// work (the paper's heterogeneous Cholesky splits the blocks between the CPU
// and the GPU), not a reference: their results are checked against the
// oracle like the device path's.
#pragma once

#include <cstdint>
#include <functional>

namespace chol {
namespace host {

constexpr int HB = 128;  // tile side

// In-place Cholesky of one lower tile (strict upper part set to zero).
// Returns 0, or the 1-based local column of the first non-positive (or NaN)
// pivot.
int potrf_tile(double *L);
// X <- X L^{-T} for one tile X (substitution with the lower tile L).
void trsm_tile(const double *L, double *X);
// C -= sum_{p < np} A[p] B[p]^T (all tiles column-major 128 x 128).  With
// `lower` (a diagonal tile) the lower triangle, diagonal included, is
// updated; blocks wholly above the diagonal are skipped and the rest of the
// strict upper triangle is unspecified (never read).
void gemm_nt_tiles(double *C, const double *const *A, const double *const *B, int np, bool lower);

// Thread pool: run fn(i) for i in [0, count) on the pool's threads and the
// calling thread (dynamic assignment), returning when all are done.
void parallel_for(int64_t count, const std::function<void(int64_t)> &fn);
// Threads used (the caller included); set before the first parallel_for.
void set_threads(int n);
int threads();

}  // namespace host
}  // namespace chol

namespace chol {
namespace host {
// Both products of one lower tile T (column-major 128 x 128) in one pass:
// y_row = T x_c (overwritten) and y_col += T^T x_i.  With `diag` (a
// diagonal tile, strict upper part zero) y_row receives the full symmetric
// product T x + T^T x - diag(T) x of x = x_c and y_col is not touched.
void tile_symv_pair(const double *T, const double *x_c, const double *x_i, double *y_row,
                    double *y_col, bool diag);
}  // namespace host
}  // namespace chol
