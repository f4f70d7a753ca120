// Internal declarations shared by the HIP kernels and the host scheduler.
//
// Factor storage (the paper's layout, Implementation section: only the
// lower-triangular and diagonal square blocks are stored): an order-n matrix
// is padded to N = ceil(n / b) tiles of side b; tile (i, c), i >= c, is one
// contiguous column-major b x b block.  Tiles are ordered column of tiles by
// column of tiles, so the panel below a diagonal block (Step 2 of the blocked
// algorithm) is one contiguous range.  Padding rows/columns hold the identity,
// so the factor of the padded matrix is diag(L, I) exactly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace chol {

__host__ __device__ inline int64_t tile_col_offset(int64_t c, int64_t N) {
  return c * N - (c * (c - 1)) / 2;
}
__host__ __device__ inline int64_t tile_index(int64_t i, int64_t c, int64_t N) {
  return tile_col_offset(c, N) + (i - c);
}
__host__ __device__ inline int64_t tile_count(int64_t N) { return N * (N + 1) / 2; }

// Element storage kinds of the factor.
enum Store : int { STORE_F64 = 0, STORE_F32 = 1 };

// Descriptor of one batched column step (the serving engine): job j is at
// tile column c of its own packed FP32 matrix (tile 128); its panel solves
// are entries [trsm_begin, trsm_begin + N - c - 1) of the step's flat list,
// its trailing-triangle updates entries [upd_begin, upd_begin + R (R + 1) / 2),
// R = N - c - 1.  Jobs are ordered by both prefixes.
struct BatchJob {
  void *tiles;
  int64_t *info;
  int64_t N, c, trsm_begin, upd_begin;
  int64_t pad[2];
};
struct BatchDesc {
  int64_t njobs, trsm_total, upd_total;
  int64_t pad[5];
  BatchJob jobs[1];  // njobs entries
};
constexpr size_t batch_desc_bytes(int max_jobs) {
  return sizeof(BatchDesc) + (size_t)(max_jobs > 1 ? max_jobs - 1 : 0) * sizeof(BatchJob);
}
// One batched column step: the diagonal tiles (one workgroup per job, grid
// max_jobs), then the panel solves (grid trsm_grid, walking the flat list),
// then the trailing updates (persistent grid upd_grid, FP32 matrix cores).
void launch_batch_potrf_trsm(const BatchDesc *d, int max_jobs, int trsm_grid, hipStream_t s);
void launch_batch_update(const BatchDesc *d, int upd_grid, int super_tile, hipStream_t s);

// ---- launchers (all asynchronous on `s`) --------------------------------
// gp_assemble into a column-major matrix.
void launch_gp_assemble(const double *X, int64_t n, int64_t d, int64_t ldx, double two_l2,
                        double var, double noise, double *A, int64_t lda, int full,
                        hipStream_t s);
// Matrix-free GP residual R = B - (K + noise I) Xs.
void launch_gp_residual(const double *F, int64_t n, int64_t d, int64_t ldf, double two_l2,
                        double var, double noise, const double *Xs, int64_t ldxs,
                        const double *B, int64_t ldb, double *R, int64_t ldr, int64_t nrhs,
                        hipStream_t s);

// Clear the info word (a kernel, not a memset, so graph capture is safe).
void launch_clear_i64(int64_t *p, int count, hipStream_t s);
// *out = max_i A(i, i) (column-major, leading dimension lda).
void launch_max_diag(const double *A, int64_t lda, int64_t n, double *out, hipStream_t s);

// Column-major FP64 A (lower) -> packed tiles, scaled by `scale`, identity
// padding; only tile columns [c_begin, c_end) (c_end < 0: to the last).
// diag_shift is added to the diagonal after scaling (the FP16 form's retry).
void launch_pack(const double *A, int64_t n, int64_t lda, void *tiles, int store, int b,
                 int64_t N, double scale, hipStream_t s, int64_t c_begin = 0,
                 int64_t c_end = -1, double diag_shift = 0.0);
// Packed tiles -> dense column-major FP64 L (upper set to zero), times `scale`;
// NaN everywhere in the lower triangle when *info != 0 (a failed factor).
void launch_unpack(const void *tiles, int store, int b, int64_t N, int64_t n, double scale,
                   double *L, int64_t ldl, const int64_t *info, hipStream_t s);

// Step 1: factor diagonal tile c in place (FP64 arithmetic).  Sets *info.
// la: with the fifth-wave lookahead inside the tile (same result; faster
// alone, but its fifth wave is harder to place beside trailing updates).
void launch_potrf(void *tiles, int store, int b, int64_t N, int64_t c, int64_t *info,
                  hipStream_t s, bool la = false);
// Step 2: tiles (i, c), i in [r0, N) (r0 <= 0: c + 1): X <- X L_cc^{-T}
// (FP64 arithmetic).
// Panel solves of column steps with at most this many tiles below the
// diagonal run with four workgroups per tile (a quarter of the rows each).
void set_trsm_split_max(int64_t tiles);
void launch_trsm(void *tiles, int store, int b, int64_t N, int64_t c, const int64_t *info,
                 hipStream_t s, int64_t r0 = 0);
// Step 3: C_ik -= sum_{p in [p0, p0+pw)} L_ip L_kp^T over the region
//   mode 0 (triangle): k0 <= k <= i < N;
//   mode 1 (band)    : k in [k0, k1), k <= i < N  (k1 - k0 <= super_tile);
//   mode 2 (rectangle, FP64 tile 128): i in [r0, N), k in [k0, k1), r0 >= k1.
// fp16 = 1 takes the panel operands in FP16 from p16, the panel's FP16 copy
// written by launch_trsm_inv (FP32 storage, tile 128 only).
// max_wg > 0 caps the number of workgroups (each then walks several tiles),
// leaving workgroup slots free for kernels on other streams.
void launch_update(void *tiles, int store, int b, int64_t N, int64_t p0, int pw, int64_t k0,
                   int64_t k1, int mode, int super_tile, int fp16, const int64_t *info,
                   hipStream_t s, int64_t max_wg = 0, const void *p16 = nullptr,
                   int64_t r0 = 0);
// Kernel choice for the FP16 form's whole-triangle updates (1: 2 x 2 tiles
// per workgroup, the default; 0: one tile per workgroup).  Same result.
void set_f16_wide(int on);
// FP16 panel buffers of the FP16 form: for tile row i and chunk ch (64
// columns of the panel, two per tile column), 128 rows x 64 halves at halves
// offset (i * kP16ChunksPerTileRow + ch) * 128 * 64, up to 32 tile columns
// per panel.  Within a chunk, row r's 16-byte segment sg (columns 8 sg ..
// 8 sg + 7) sits at p16_pos(r, sg).
constexpr int kP16ChunksPerTileRow = 64;
constexpr int64_t kP16BytesPerChunk = 128 * 64 * 2;  // 128 rows x 64 columns of halves
constexpr int64_t kP16BytesPerTileRow = kP16ChunksPerTileRow * kP16BytesPerChunk;

// The update kernels' FP16 fragment reads (v_mfma_f32_16x16x32_f16: lane
// (g, q) supplies row 4q + s2 of the operand, columns 8g .. 8g + 7) have the
// 16 lanes of a lane group on rows 4q + s2, q = 0..15.  Segments are
// XOR-swizzled by q mod 8, and the stored row takes bit 5 of the logical row
// (the high bit of q) as its bit 0, so the sixteen lanes cover both 128-byte
// halves of a 256-byte line of all 64 LDS banks with distinct segments: one
// 128-bit read is conflict-free.  The low two row bits (s2) move to bits 4-5
// so that the four rows a lane reads differ by constant offsets.  The chunks
// are DMA'd verbatim, so the LDS layout equals this one.
__device__ __forceinline__ int p16_pos(int r, int sg) {
  const int pr = (r & 64) | ((r & 3) << 4) | (((r >> 2) & 7) << 1) | ((r >> 5) & 1);
  return pr * 64 + 8 * (sg ^ ((r >> 2) & 7));
}

// Step 2 of the FP16 form (FP32 tiles, tile 128): block c of dinv <- L_cc^{-T}
// (as launch_diag_inverse computes it), then the tiles (i, c), i > c, <-
// tile * dinv_c on the FP32 matrix cores, each also written in FP16 to its
// two chunks of the panel buffer p16c (the chunks of tile column c, tile row
// 0; the diagonal tile's chunks, which no update reads, are left alone).
void launch_trsm_inv(void *tiles, int64_t N, int64_t c, void *dinv, void *p16c,
                     const int64_t *info, hipStream_t s);
// After the factorisation: block c of dinv (N blocks of b x b) = L_cc^{-T}.
void launch_diag_inverse(const void *tiles, int store, int b, int64_t N, void *dinv,
                         const int64_t *info, hipStream_t s);
// Forward then back substitution, in place on B (n x nrhs, ldb), FP64
// arithmetic, one launch per direction (and per group of right-hand sides).
// sync: device scratch of sync_words ints (>= 3), cleared by the launcher;
// spin_max bounds each inter-workgroup wait (rows of an aborted solve are NaN);
// info: the factor's info word (every row is NaN when it is non-zero).
void launch_solve(const void *tiles, const void *dinv, int store, int b, int64_t N, int64_t n,
                  double *B, int64_t ldb, int64_t nrhs, int *sync, int64_t sync_words,
                  int spin_max, const int64_t *info, hipStream_t s);
// Scale B by alpha in place (used by the scaled-FP16 factor).
void launch_scale(double *B, int64_t n, int64_t ldb, int64_t nrhs, double alpha, hipStream_t s);

// R = B - A X, A symmetric from its lower triangle; exact: double-double
// accumulation (the residuals that certify), else plain FP64 (the working
// residuals of the refinement and the CG products).
void launch_symm_residual(const double *A, int64_t lda, int64_t n, const double *X,
                          int64_t ldx, const double *B, int64_t ldb, double *R, int64_t ldr,
                          int64_t nrhs, hipStream_t s, bool exact = true);
// Per-column squared 2-norms and dot products into out[nrhs] (deterministic).
void launch_col_dot(const double *x, int64_t ldx, const double *y, int64_t ldy, int64_t n,
                    int64_t nrhs, double *out, double *partial, hipStream_t s);
// y[:, c] = a[c] * x[:, c] + b[c] * y[:, c]   (coefficients from device arrays,
// with per-column active mask; NULL coefficient array means 1).
void launch_axpby(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t n,
                  int64_t nrhs, const double *a, double a_sign, const double *bcoef,
                  const int32_t *active, hipStream_t s);
// copy n x nrhs column-major blocks (masked: only columns with mask[c] != 0)
void launch_copy(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t n,
                 int64_t nrhs, hipStream_t s);
void launch_copy_masked(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t n,
                        int64_t nrhs, const int32_t *mask, hipStream_t s);
// Preconditioned CG scalars per column: alpha = rho / (-pq) on active
// columns (0 elsewhere, or for a zero / non-finite denominator); beta =
// rho_new / rho and rho <- rho_new on active columns (beta 0 elsewhere).
void launch_pcg_alpha(const double *rho, const double *pq, const int32_t *act, double *alpha,
                      int64_t nrhs, hipStream_t s);
void launch_pcg_beta(const double *rho_new, double *rho, const int32_t *act, double *beta,
                     int64_t nrhs, hipStream_t s);

// Kernel timing hooks (option "profile"): profile_begin records an event
// on s before a launch, profile_end one after it and files the pair with the
// launch's algorithmic work for chol_profile_read.
int64_t profile_option();
hipEvent_t profile_begin(hipStream_t s);
void profile_end(hipStream_t s, hipEvent_t a, double work);

// ---- conjugate gradients on the packed lower tiles (FP64) ----------------
// Partial products of every stored tile with v (K columns, ldv): part holds
// tile_count(N) * 2 * K * b doubles.  Nt >= 0: only the tiles of the leading
// Nt block rows and columns (the heterogeneous CG's GPU share).
void launch_cg_symv(const double *tiles, int b, int64_t N, const double *v, int64_t ldv, int K,
                    double *part, hipStream_t s, int64_t Nt = -1);
// Row sums of the partials; mode 0: t = A s and s.t partials, 1: r = b - A x
// for active columns and r.r partials, 2: r = s = b - A x and r.r partials.
enum { CG_RED_T = 0, CG_RED_RESID = 1, CG_RED_INIT = 2 };
// Nt >= 0: block rows [0, Nt) only, from the tiles of the leading Nt block
// rows and columns, plus `extra` (the other tiles' products for these rows).
void launch_cg_reduce(const double *part, int b, int64_t N, int K, int mode, double *t, double *sv,
                      double *r, const double *bv, int64_t ld, const int *act, double *pdot,
                      hipStream_t s, int64_t Nt = -1, const double *extra = nullptr);
// rows >= 0: block rows [0, rows) only (the scalars still sum all N partials).
void launch_cg_xr(int b, int64_t N, int K, const double *pdot, const double *u_in, const int *act,
                  double *x, double *r, const double *sv, const double *t, int64_t ld,
                  int recompute_now, double *prr, hipStream_t s, int64_t rows = -1);
void launch_cg_s(int b, int64_t N, int K, const double *prr, const double *u_in, const int *act_in,
                 double *u_out, int *act_out, const double *u0, double eps2, int *iters,
                 const double *r, double *sv, int64_t ld, hipStream_t s, int64_t rows = -1);
void launch_cg_init(int b, int64_t N, int K, const double *prr, double *u, double *u0, int *act,
                    int *iters, double eps2, hipStream_t s);
void launch_cg_copy_in(const double *src, int64_t lds, int64_t n, int64_t n_pad, int K, double *dst,
                       int64_t ld, hipStream_t s);
void launch_cg_copy_out(const double *src, int64_t ld, int64_t n, int K, double *dst, int64_t ldd,
                        hipStream_t s);

}  // namespace chol
