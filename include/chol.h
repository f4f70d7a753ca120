/*
 * chol.h - C ABI of the MI355X (gfx950) dense SPD / Gaussian-process solver.
 *
 * The library solves A x = b for a symmetric positive definite A (the
 * problem statement of the paper, Introduction and Fundamentals) through the
 * blocked right-looking Cholesky factorisation A = L L^T, L lower triangular
 * (Fundamentals, "The Cholesky decomposition", and the blocked algorithm in
 * the paper's first algorithm figure, right column: Step 1 factors the
 * diagonal block, Step 2 solves the panel below it, Step 3 updates the
 * trailing blocks), followed by forward and back substitution with L.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major: element (i, j) of a matrix with leading
 *   dimension ld sits at M[i + j*ld].  Only the lower triangle of A is read.
 * - Pointers named A, B, X, L, workspace are DEVICE pointers (HBM of the
 *   current HIP device) unless stated otherwise.  `stream` is a hipStream_t
 *   passed as void*; NULL means the default stream.  Calls are stream-ordered
 *   and return after enqueueing, unless stated otherwise.
 * - Ownership: the caller allocates and frees all device memory.  The library
 *   never allocates device memory; it owns only the small host handle
 *   returned by chol_factor (with one event for ordering solves), plus one
 *   side stream and a few events per (device, caller stream) pair used by
 *   chol_factor, created on first use and kept until the process ends.
 * - Threads: calls on different streams may run concurrently from different
 *   host threads; calls that share a stream must not overlap.
 * - Return value: CHOL_OK (0) on success; -i when argument i (1-based) is
 *   invalid; one of the negative CHOL_ERR_* codes otherwise.  Nothing is
 *   enqueued when an argument is rejected.
 * - Not positive definite: *info = j + 1 where j is the first (0-based) global
 *   column whose pivot is not positive (or is NaN), exactly as LAPACK's
 *   potrf reports it.  The factor contents are then unspecified.
 */
#ifndef CHOL_MI355X_H
#define CHOL_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define CHOL_OK 0
#define CHOL_ERR_HIP (-100)           /* a HIP runtime call failed            */
#define CHOL_ERR_WORKSPACE (-101)     /* workspace smaller than required      */
#define CHOL_ERR_NOT_CONVERGED (-102) /* refinement hit max_iter              */
#define CHOL_ERR_NOT_SPD (-103)       /* factor failed (info > 0)             */
#define CHOL_ERR_UNSUPPORTED (-104)   /* precision / tile not built           */
#define CHOL_ERR_BAD_HANDLE (-105)

/* ---- precisions of the factor ---------------------------------------- */
/* CHOL_FP64        : FP64 storage, FP64 MFMA trailing update.
 * CHOL_FP32        : FP32 storage, FP32 MFMA trailing update; the
 *                    diagonal-block factorisation and the panel solves
 *                    compute in FP64 and round their result to FP32.
 * CHOL_FP16_SCALED : FP32 storage of H = A / s (s = the largest diagonal
 *                    entry), trailing update with FP16 operands and FP32
 *                    accumulation; diagonal blocks and panel solves in FP64.
 *                    For matrices with a constant diagonal (every SE kernel
 *                    matrix) H has unit diagonal, so all |L_H| <= 1.
 * The two low-precision forms are meant to be followed by chol_refine_solve,
 * which recovers FP64 accuracy (the paper names mixed precision as future
 * work in its Conclusion).                                                  */
#define CHOL_FP64 0
#define CHOL_FP32 1
#define CHOL_FP16_SCALED 2

#define CHOL_REFINE_IR 0  /* iterative refinement                          */
#define CHOL_REFINE_PCG 1 /* CG preconditioned with M = L L^T (the paper's
                             CG algorithm, first algorithm figure, left
                             column, with the factor as preconditioner)      */

typedef struct chol_factor_s *chol_handle;

/* Fallbacks (bit flags in chol_refine_report.fallback_used and in
 * chol_factor_fallback):
 * CHOL_FALLBACK_PCG   iterative refinement stagnated (a right-hand side's
 *                     correction failed to halve in two consecutive steps)
 *                     and CG preconditioned with the factor finished the
 *                     solve from the current iterate;
 * CHOL_FALLBACK_SHIFT the FP16 form met a non-positive pivot and was
 *                     refactored with the diagonal shift c * 2^-11 added to
 *                     the scaled matrix (c = option "fp16_shift_c", 32);
 * CHOL_FALLBACK_FP32  the FP16 form failed (again) and an FP32 factor
 *                     replaced it (chol_factor_precision then reports
 *                     CHOL_FP32).                                           */
#define CHOL_FALLBACK_PCG 1
#define CHOL_FALLBACK_SHIFT 2
#define CHOL_FALLBACK_FP32 4

typedef struct {
  int32_t iters;          /* corrections (IR) plus iterations (PCG)            */
  int32_t converged;      /* 1 if every RHS met the stopping rule              */
  double cert;            /* max over RHS of the final error bound (see below) */
  double resid_norm;      /* max over RHS of ||b - A x||_2 at exit             */
  double time_ms;         /* host wall time of the call, including its sync    */
  int32_t fallback_used;  /* CHOL_FALLBACK_* flags of the factor and the call  */
  int32_t reserved;
} chol_refine_report;

/* ---- gp_assemble ------------------------------------------------------
 * Squared-exponential Gaussian-process covariance plus noise, the synthetic
 * stand-in for the paper's GP kernel matrices (Results, Experimental Setup):
 *   A_ij = variance * exp(-|x_i - x_j|^2 / (2 lengthscale^2))   (i != j)
 *   A_ii = variance + noise
 * X  : device, n x d row-major features, row stride ldx (>= d), FP64.
 * A  : device, n x n column-major FP64, leading dimension lda (>= n).
 * uplo_full = 0 writes the lower triangle only (upper untouched); 1 writes
 * the full symmetric matrix (bitwise symmetric).
 * Errors: -2 n < 0, -3 d < 1, -4 ldx < d, -5/-6/-7 non-positive lengthscale,
 * negative variance or noise, -9 lda < max(1, n).                        */
int gp_assemble(const double *X, int64_t n, int64_t d, int64_t ldx,
                double lengthscale, double variance, double noise, double *A,
                int64_t lda, int uplo_full, void *stream);

/* ---- chol_factor_bytes -------------------------------------------------
 * Device workspace, in bytes, that chol_factor needs for an order-n matrix
 * at the given precision and tile (tile 0 = the tuned default).  The factor
 * is stored as the paper stores it (Implementation section): only the
 * lower-triangular and diagonal square blocks, each block contiguous, plus
 * the N inverted diagonal blocks L_cc^{-T} that the solves apply (computed
 * once at the end of the factorisation); CHOL_FP16_SCALED adds two FP16
 * copies of a panel (N * 1 MB each, up to 32 tile columns) that its
 * trailing updates read.
 * Returns 0 for invalid arguments.  Host-only; no device work.           */
size_t chol_factor_bytes(int64_t n, int precision, int tile);

/* ---- chol_tile_default -------------------------------------------------
 * The tile chol_factor uses when called with tile = 0.                   */
int chol_tile_default(int64_t n, int precision);

/* ---- chol_factor -------------------------------------------------------
 * Factor A = L L^T (blocked right-looking, Steps 1-3 of the paper's
 * algorithm) into the workspace.
 * A         : device, n x n column-major FP64 (lower triangle read), lda.
 *             Not modified.
 * precision : CHOL_FP64 / CHOL_FP32 / CHOL_FP16_SCALED.
 * tile      : block side 64 or 128; 0 selects chol_tile_default.
 * workspace : device, >= chol_factor_bytes(n, precision, tile) bytes,
 *             256-byte aligned.  Holds the factor; must stay allocated and
 *             untouched while the handle is used.
 * F         : out, host handle of type chol_handle (free with
 *             chol_factor_free).
 * info      : out, may be NULL.  If non-NULL the call synchronises the stream
 *             and stores the LAPACK-style info (0 = success).  If NULL the
 *             call is fully asynchronous; use chol_get_info later.
 *             With CHOL_FP16_SCALED and info non-NULL, a non-positive pivot
 *             is not returned at once: the factorisation is retried with a
 *             diagonal shift, then as CHOL_FP32 (CHOL_FALLBACK_SHIFT /
 *             CHOL_FALLBACK_FP32; chol_factor_fallback reports which), and
 *             *info is the last attempt's.  The shifted factor is that of
 *             A + s c 2^-11 I (s = the largest diagonal entry of A), which the
 *             refinement then corrects.
 * Errors: -2 n < 0, -3 lda < max(1,n), -4 precision, -5 tile, -6 workspace
 * NULL or misaligned, -7 ws_bytes too small (also CHOL_ERR_WORKSPACE), -8 F
 * NULL.                                                                  */
int chol_factor(const double *A, int64_t n, int64_t lda, int precision,
                int tile, void *workspace, size_t ws_bytes, chol_handle *F,
                int64_t *info, void *stream);

/* ---- chol_factor_ex ----------------------------------------------------
 * chol_factor with per-call schedule options instead of the process-wide
 * ones (for concurrent callers such as the serving loop).  Any field <= 0
 * (or lookahead < 0) falls back to the process-wide value; opts may be NULL.
 * tile: 64 or 128 (0 = chol_tile_default); panel_width: 1..32 (above 8 only
 * for CHOL_FP16_SCALED; FP64 and FP32 use at most 8); lookahead: 0/1;
 * super_tile: 1..64.  The schedule never changes the computed factor.     */
typedef struct {
  int32_t tile;
  int32_t panel_width;
  int32_t lookahead;
  int32_t super_tile;
  int32_t graph; /* 1: capture / replay a HIP graph; 0: direct launches; <0: process-wide */
} chol_factor_opts;

int chol_factor_ex(const double *A, int64_t n, int64_t lda, int precision,
                   const chol_factor_opts *opts, void *workspace,
                   size_t ws_bytes, chol_handle *F, int64_t *info,
                   void *stream);

/* Synchronises the factor's stream and reports info (0 = success).       */
int chol_get_info(chol_handle F, int64_t *info);

/* CHOL_FALLBACK_SHIFT / CHOL_FALLBACK_FP32 flags taken by chol_factor for
 * this handle (0 = none; -1 for a NULL handle).                          */
int chol_factor_fallback(chol_handle F);

/* ---- chol_solve --------------------------------------------------------
 * B <- A^{-1} B using the factor only: forward substitution L Y = B, then
 * back substitution L^T X = Y (Fundamentals, "The Cholesky decomposition").
 * Arithmetic is FP64 whatever the factor's storage precision.  Blocked by
 * tiles: block row i is b_i minus the products with the finished blocks,
 * times the inverted diagonal block, in one kernel launch per direction.
 * B : device, n x nrhs column-major FP64, ldb >= max(1, n), overwritten.
 * The workgroups of a solve synchronise through words in the factor's
 * workspace header, so solves with one factor are serialised: a solve
 * issued on another stream than the previous solve with this factor waits
 * for it (an event; not on a capturing stream, where the earlier solves must
 * have been captured on that stream or have finished).  The first solve
 * must be stream-ordered after chol_factor by the caller, as for any
 * stream-ordered call.  Allocates nothing; may be captured into a graph.
 * Each wait between workgroups is bounded (option "solve_spin_max"); should
 * a bound ever run out, the affected rows of B are set to NaN instead of
 * hanging.
 * Errors: CHOL_ERR_BAD_HANDLE, -2 B NULL with nrhs > 0, -3 nrhs < 0,
 * -4 ldb, CHOL_ERR_NOT_SPD if the factorisation is known (on the host) to
 * have failed.  If it failed but the host has not read info yet (an
 * asynchronous chol_factor), the call returns CHOL_OK and every entry of B
 * becomes NaN: the kernels read the factor's info word.                  */
int chol_solve(chol_handle F, double *B, int64_t nrhs, int64_t ldb,
               void *stream);

/* ---- chol_refine_bytes -------------------------------------------------
 * Device workspace chol_refine_solve needs for nrhs right-hand sides (the
 * same for both methods, since refinement may fall back to PCG): five
 * n x nrhs FP64 blocks plus 138 doubles per right-hand side plus 256 bytes.
 * 0 for invalid arguments.                                                */
size_t chol_refine_bytes(int64_t n, int64_t nrhs, int method);

/* ---- chol_refine_solve -------------------------------------------------
 * Solve A X = B to FP64 accuracy with a (typically low-precision) factor F
 * of A, by iterative refinement (method CHOL_REFINE_IR) or by CG
 * preconditioned with M = F F^T (CHOL_REFINE_PCG).  Residuals r = b - A x
 * and the solution updates are computed in FP64; every residual a
 * certificate is taken from is accumulated in double-double, and with a
 * stored A, lam > 0 and several right-hand sides the working residuals of
 * IR and the products q = A p of PCG are plain FP64 (IR takes the residual
 * again in double-double before a column can stop, at the iteration limit,
 * and for good once the plain residuals stop improving).
 * A      : device, FP64 n x n column-major (lower triangle read), lda; or
 *          NULL, in which case the residual is computed matrix-free from the
 *          GP features Xf (n x d row-major, ldxf) and the hyper-parameters,
 *          with exactly the formula of gp_assemble.
 * noise  : lower bound lam on the smallest eigenvalue of A (for a GP
 *          matrix: the noise variance).  With lam > 0 the stopping rule is
 *          the certificate ||r||_2 / (lam ||x||_2) <= tol / 2, a rigorous
 *          bound on the relative error ||x - x*|| / ||x||.  With lam <= 0 it
 *          is ||d||_2 <= tol ||x||_2 for the last correction d (IR) or
 *          ||r||_2 <= tol ||b||_2 (PCG).
 * B      : device, n x nrhs column-major FP64, ldb.  Not modified.
 * X      : device, n x nrhs column-major FP64, ldxs.  Output.
 * workspace: device, 8-byte aligned, >= chol_refine_bytes(n, nrhs, method)
 *          bytes.
 * rep    : out (host), may be NULL.
 * Both methods start from x0 = M^{-1} b and stop each right-hand side on
 * its own (a finished column is left unchanged).  IR: x += M^{-1}(b - A x);
 * a column whose correction fails to halve in two consecutive steps makes
 * the call continue with PCG from the current iterate (CHOL_FALLBACK_PCG).
 * PCG: the paper's CG algorithm with the preconditioner M = F F^T: q = A p,
 * alpha = rho / p.q, x += alpha p, r -= alpha q; every `pcg_recompute`
 * iterations (option, default 50; 0 = never) r is replaced by the true
 * residual b - A x; a column that passes the stopping rule is confirmed on
 * its true residual before it stops; z = M^{-1} r, rho' = r.z,
 * p = z + (rho' / rho) p.  The scalars are computed on the device; the host
 * reads back the squared norms of r and x (and of the IR correction) once
 * per iteration to take the stopping decisions.  `iters` counts the IR
 * corrections plus the PCG iterations against max_iter.
 * Returns CHOL_ERR_NOT_CONVERGED if max_iter is reached; X then holds the
 * last iterate.                                                          */
int chol_refine_solve(chol_handle F, const double *A, int64_t lda,
                      const double *Xf, int64_t d, int64_t ldxf,
                      double lengthscale, double variance, double noise,
                      const double *B, int64_t ldb, double *X, int64_t ldxs,
                      int64_t nrhs, double tol, int max_iter, int method,
                      void *workspace, size_t ws_bytes,
                      chol_refine_report *rep, void *stream);

/* ---- chol_refine_solve_noalloc ------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * chol_refine_solve with the same arguments and results, minus the
 * workspace, which is replaced by a static device array of
 * chol_refine_noalloc_max_bytes() bytes (64 MiB) inside the library, held by
 * every GPU the library runs on until the process ends.  The call allocates
 * no device memory (no hipMalloc / hipFree, no allocating library routine).
 * It serves n x nrhs problems with chol_refine_bytes(n, nrhs, method) up to
 * that size (n * nrhs up to about 1.6 million, e.g. n = 8192 with 64
 * right-hand sides, n = 65536 with 16); larger problems return
 * CHOL_ERR_WORKSPACE before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (from several host threads or streams) race and give wrong
 * results; serialise them.  The array keeps the last call's contents; each
 * call writes every part of it before reading it.
 * Errors: those of chol_refine_solve, CHOL_ERR_WORKSPACE for a problem too
 * large for the array, CHOL_ERR_HIP if the array's device address cannot be
 * found (looked up once per device, on the first call on it).            */
size_t chol_refine_noalloc_max_bytes(void);
int chol_refine_solve_noalloc(chol_handle F, const double *A, int64_t lda,
                              const double *Xf, int64_t d, int64_t ldxf,
                              double lengthscale, double variance, double noise,
                              const double *B, int64_t ldb, double *X,
                              int64_t ldxs, int64_t nrhs, double tol,
                              int max_iter, int method,
                              chol_refine_report *rep, void *stream);

/* ---- chol_residual -----------------------------------------------------
 * R = B - A X in FP64 with A symmetric given by its lower triangle (lda),
 * all n x nrhs column-major device arrays.  Deterministic (no atomics).   */
int chol_residual(const double *A, int64_t lda, int64_t n, const double *X,
                  int64_t ldx, const double *B, int64_t ldb, double *R,
                  int64_t ldr, int64_t nrhs, void *stream);

/* ---- chol_factor_to_dense ----------------------------------------------
 * Write the factor as a dense n x n column-major FP64 matrix L (ldl): the
 * lower triangle holds L (widened from the storage precision and, for
 * CHOL_FP16_SCALED, multiplied back by sqrt(s) so that L L^T ~ A); the
 * strict upper triangle is set to zero.                                  */
int chol_factor_to_dense(chol_handle F, double *L, int64_t ldl, void *stream);

/* Host handle queries.  Values are fixed when chol_factor returns.        */
int64_t chol_factor_n(chol_handle F);
int chol_factor_tile(chol_handle F);
int chol_factor_precision(chol_handle F);

/* Frees the host handle only; the workspace stays the caller's.           */
void chol_factor_free(chol_handle F);

/* Human-readable text for a status code (static storage).                 */
const char *chol_status_string(int status);

/* ---- kernel timing ------------------------------------------------------
 * With option "profile" = 1, every launch of the Step-3 trailing-update
 * kernel is bracketed by a pair of HIP events recorded on the stream it is
 * launched on (with "profile" = 2 only the launches over a whole trailing
 * triangle, not the panel-band ones), and the launch's algorithmic flop
 * count is accumulated
 * (2 b^2 K per off-diagonal tile and b (b + 1) K per diagonal tile, K the
 * inner dimension of the launch).  chol_profile_read waits for the recorded
 * events and returns the summed kernel time (ms), the number of launches and
 * the summed flops; chol_profile_reset forgets everything recorded.  Not
 * thread-safe; meant for benchmarks.  cg_solve's tile-product launches are
 * recorded the same way (with either value of "profile"), their work being
 * bytes, not flops: 8 b^2 per stored tile (the packed triangle read once).
 * Read the records of one kind of call at a time.                          */
int chol_profile_read(double *ms, int64_t *launches, double *flops);
void chol_profile_reset(void);

/* ---- tuning knobs (process-wide; set before factorising) ---------------
 * "panel_width"  : tiles per outer step whose Step-3 update is applied in
 *                  one pass (1..32; 0 = automatic: 8 from 192 tile rows,
 *                  4 from 64, else 8, and 32 for CHOL_FP16_SCALED from 512
 *                  tile rows; default 0).  Widths above 8 apply to
 *                  CHOL_FP16_SCALED only (FP64 and FP32 use 8 then).
 * "lookahead"    : 1 overlaps the next panel's Steps 1-2 with the current
 *                  trailing update on a second stream (default 1).
 * "super_tile"   : side, in tiles, of the groups the trailing-update grid
 *                  walks through together for cache reuse (default 8).
 * "graph"        : 1 captures the factorisation's launches (on the caller's
 *                  stream and the side stream) into a HIP graph on the first
 *                  call with a given (A, lda, n, precision, tile, schedule,
 *                  workspace) and replays it on later identical calls; the
 *                  32 most recent graphs per process are kept (default 0).
 *                  Not used for CHOL_FP16_SCALED or while profiling.
 * "profile"      : 1 records kernel timing, 2 only of the triangle launches
 *                  (see chol_profile_read).
 * "solve_spin_max": polls allowed per wait inside chol_solve (default 2^20,
 *                  about a second; rows of a solve that runs out become NaN).
 * "pcg_recompute": chol_refine_solve's PCG takes the true residual every
 *                  this many iterations (default 50, the paper's periodic
 *                  recomputation; 0 = never).
 * "fp16_shift_c" : c of the FP16 form's shifted retry (default 32; 0 = go
 *                  straight to the FP32 fallback).
 * "host_threads" : threads of the heterogeneous factorisation's CPU share
 *                  (default min(16, hardware threads); only before its first
 *                  call).
 * "first_panel_width": tile columns of the first panel (1..32; 0 = the
 *                  panel width; default 0).  With lookahead the first
 *                  panel's tile columns are packed first and factored while
 *                  the rest of A is packed; a narrower first panel lets the
 *                  first trailing update start sooner.
 * "f16_wide"     : 1 (default) runs the FP16 form's whole-triangle updates
 *                  with 2 x 2 tiles per workgroup (half the operand traffic
 *                  per flop), 0 with one tile per workgroup; same result.
 * "panel_order"  : order of the updates inside a panel: 1 right-looking
 *                  (after each tile column, the panel's later columns are
 *                  updated by it), 2 left-looking (before each tile column,
 *                  it is updated by the panel's earlier columns: each panel
 *                  tile read and written once), 3 recursive (the panel's
 *                  columns halved: left half factored, right half updated by
 *                  it in one launch, then factored; down to two columns),
 *                  0 (default) automatic: 2 for CHOL_FP16_SCALED, 3 from
 *                  256 tile rows, 1 otherwise.  Same factor bit for bit.
 * "trsm_split"   : column steps with at most this many tiles below the
 *                  diagonal split each tile's panel solve (Step 2) over four
 *                  workgroups, a quarter of its rows each, which shortens
 *                  the column chain of small matrices and of the last
 *                  columns (default 64; 0 = never).  Same factor bit for bit.
 * "potrf_lookahead": 1 factors each diagonal tile (Step 1) with a fifth
 *                  wave that factors the next 16 x 16 diagonal block while
 *                  the other four apply the current block's update; 0
 *                  without; 2 (default) automatic: with it up to 64 tile
 *                  rows.  Same factor bit for bit.
 * "bulk_wg_cap"  : with lookahead, the far trailing update runs with at most
 *                  this many (persistent) workgroups, leaving slots for the
 *                  next panel's kernels (default 0 = no cap: one workgroup
 *                  per tile measured fastest on MI355X).
 * Returns CHOL_OK or -1 (unknown key) / -2 (value out of range).         */
int chol_set_option(const char *key, int64_t value);
int64_t chol_get_option(const char *key);

/* ---- continuous-batching factorisation (the serving engine) ------------
 * Many FP32 factorisations (tile 128) advance together, one tile column per
 * step: a step is one batched diagonal-tile factorisation (Step 1, a
 * workgroup per job), one batched panel solve (Step 2) and one batched
 * trailing update (Step 3, FP32 matrix cores over a flat list of every
 * job's trailing triangle), described by a device descriptor that the host
 * rewrites before each step; with use_graph the three launches are captured
 * once into a HIP graph and replayed.  Jobs join (chol_batch_add) and leave
 * (when their last column is done) between steps, so requests that arrive
 * while others are being factored share the next launches.  A job's tiles
 * receive the same operations in the same order whatever else is in the
 * batch: its factor is bitwise the same alone and in any mix.  The factor
 * is that of chol_factor(..., CHOL_FP32, 128) computed column by column
 * (panel width 1), so it is equal to it up to rounding, not bitwise.
 * desc    : device memory, 256-byte aligned, >= chol_batch_desc_bytes(max_jobs),
 *           owned by the caller and kept while the engine lives.
 * stream  : the engine's stream (all its work, packing included, runs there;
 *           required when use_graph is set).
 * chol_batch_add: A (device, column-major FP64, lower read; it must be ready,
 *   i.e. its producer synchronised, before the call) is packed into
 *   workspace (>= chol_factor_bytes(n, CHOL_FP32, 128)) on the engine's
 *   stream; *job receives the job's id.  CHOL_ERR_WORKSPACE when max_jobs
 *   jobs are active.
 * chol_batch_step: one step of every active job; *active = jobs in it,
 *   *finished = jobs whose factorisation it completed.  Thread-safe with
 *   chol_batch_add / status / take.
 * chol_batch_status: *done = 1 once the job's last step is enqueued.
 * chol_batch_take: the finished job's factor as a handle (free with
 *   chol_factor_free); the job id is then released.  chol_get_info (and so
 *   chol_refine_solve) waits for that job's kernels only, not the whole
 *   engine stream; solves on other streams are ordered by that wait.
 * Errors: CHOL_ERR_BAD_HANDLE, -i invalid argument i, CHOL_ERR_WORKSPACE,
 *   CHOL_ERR_NOT_CONVERGED (take before the job finished), CHOL_ERR_HIP.   */
typedef struct chol_batch_s *chol_batch;
size_t chol_batch_desc_bytes(int max_jobs);
int chol_batch_create(int max_jobs, void *desc, size_t desc_bytes, int use_graph,
                      void *stream, chol_batch *out);
void chol_batch_destroy(chol_batch b);
int chol_batch_add(chol_batch b, const double *A, int64_t n, int64_t lda,
                   void *workspace, size_t ws_bytes, int64_t *job);
int chol_batch_step(chol_batch b, int *active, int *finished);
int chol_batch_status(chol_batch b, int64_t job, int *done);
int chol_batch_take(chol_batch b, int64_t job, chol_handle *F);

/* ---- heterogeneous CPU + GPU factorisation ------------------------------
 * The paper's heterogeneous Cholesky (Implementation, "Cholesky
 * implementation"; Results, the heterogeneous Cholesky workload
 * distribution and its comparison with the homogeneous runs): FP64, tile
 * 128, panels of panel_width tile columns (0 = 8).  A horizontal border
 * splits the trailing matrix's tile rows: the rows above it (the diagonal
 * tile included) are factored and updated by the host CPU (the library's
 * own FP64 tile kernels on a pool of "host_threads" threads), the rows below
 * it by the GPU.  Per panel the CPU factors the diagonal tiles and solves its
 * rows, sends those tiles to the GPU (one copy per tile column), and both
 * sides apply the Step-3 update to their rows; the CPU updates the next
 * panel's columns first.  The border moves down as the trailing matrix
 * shrinks, so that about a fraction gpu_share of the Step-3 tile updates is
 * done by the GPU; each move copies whole tile rows from the GPU to the CPU.
 * When the CPU's share drops below one panel its rows return to the GPU,
 * which finishes alone.  gpu_share = 1 is the GPU alone (plain schedule,
 * no lookahead).
 * A, lda, n  : as chol_factor (device, column-major FP64, lower triangle).
 * workspace  : device, >= chol_factor_bytes(n, CHOL_FP64, 128); holds the
 *              factor afterwards (the handle works with chol_solve etc.).
 * host_ws    : HOST memory, >= chol_hetero_host_bytes(n) bytes (the packed
 *              triangle; pinned memory makes the copies asynchronous); it
 *              holds the CPU's rows while they are worked on.
 * info       : out (required): synchronous call, LAPACK-style info.
 * rep        : out, may be NULL.
 * Errors: -1 A NULL, -2 n < 0, -3 lda, -4 gpu_share outside [0, 1], -5
 * panel_width outside [0, 8], -6 workspace NULL or misaligned,
 * CHOL_ERR_WORKSPACE, -8 host_ws NULL or too small, -10 F NULL, -11 info
 * NULL, CHOL_ERR_HIP.                                                      */
typedef struct {
  double gpu_share_target;  /* as requested                                  */
  double gpu_share_tiles;   /* Step-3 tile updates (x panel columns) on the
                               GPU over all of them                          */
  double gpu_tile_updates, cpu_tile_updates;
  double bytes_h2d, bytes_d2h; /* host <-> device copies                     */
  double ms_total;          /* wall time of the call                         */
  double ms_cpu;            /* host time in the CPU's tile kernels           */
  double ms_wait_gpu;       /* host time waiting for the GPU                 */
  int32_t border_shifts;    /* border moves (including the final handover)   */
  int32_t handover_column;  /* tile column from which the GPU ran alone      */
  int32_t cpu_threads;
  int32_t reserved;
} chol_hetero_report;

size_t chol_hetero_host_bytes(int64_t n);
int chol_factor_hetero(const double *A, int64_t n, int64_t lda, double gpu_share,
                       int panel_width, void *workspace, size_t ws_bytes,
                       double *host_ws, size_t host_bytes, chol_handle *F,
                       int64_t *info, chol_hetero_report *rep, void *stream);

/* Host tile kernels of the CPU share (128 x 128 column-major FP64 tiles,
 * HOST pointers; no device work):
 * chol_host_potrf_tile: in-place Cholesky of a lower tile, strict upper part
 *   zeroed; returns 0 or the 1-based local column of the first non-positive
 *   pivot (Step 1).
 * chol_host_trsm_tile: X <- X L^{-T} by substitution (Step 2).
 * chol_host_gemm_nt_tiles: C -= sum_{p < np} A[p] B[p]^T (Step 3); with
 *   lower != 0 (a diagonal tile) the lower triangle, diagonal included, is
 *   updated and the strict upper triangle is left unspecified, as on the
 *   device.                                                                */
int chol_host_potrf_tile(double *L);
void chol_host_trsm_tile(const double *L, double *X);
void chol_host_gemm_nt_tiles(double *C, const double *const *A, const double *const *B, int np,
                             int lower);

/* ---- conjugate gradients (the paper's iterative solver) ----------------
 * The CG method of the paper (Fundamentals, "The Conjugate Gradient
 * method", and the left column of its CG / Cholesky algorithm figure), for
 * up to CG_MAX_RHS right-hand sides at once, each column with its own
 * scalars and its own stopping test:
 *   s = r = b - A x;  u = u0 = r.r
 *   while u > eps^2 u0 and fewer than max_iter iterations:
 *     t = A s;  alpha = u / s.t;  x += alpha s;
 *     r -= alpha t, except every `recompute`-th iteration, which takes the
 *       true residual r = b - A x (the paper's periodic recomputation;
 *       0 = never);
 *     v = u;  u = r.r;  beta = u / v;  s = r + beta s.
 * A is stored as in the paper's implementation: only the diagonal and lower
 * tiles (tile side `tile`, 64 or 128, 0 = 128), packed into the workspace
 * from the lower triangle of the caller's column-major A (lda >= n) at the
 * start of the call; each iteration reads that packed triangle once.
 * B (n x nrhs, ldb >= n) is read; X (n x nrhs, ldx >= n) holds the starting
 * guess on entry (zeros for the usual start) and the final iterate on exit.
 * The workspace (device, 256-byte aligned, ws_bytes >= cg_workspace_bytes)
 * holds the packed tiles, partial products, the vectors and the scalars.
 * iters (host, nrhs entries, may be NULL) receives the iterations taken per
 * column, relres (host, nrhs, may be NULL) sqrt(u / u0) at exit (0 if
 * b - A x0 = 0).
 * Synchronous: returns after the iteration has finished (the host checks the
 * columns' stopping flags one iteration behind the device, so at most one
 * extra iteration is enqueued, and it leaves finished columns unchanged).
 * Returns CHOL_OK when every column met its test, CHOL_ERR_NOT_CONVERGED
 * when some column stopped at max_iter (X still holds its iterate), -i for
 * an invalid argument i (1 <= nrhs <= CG_MAX_RHS, eps >= 0, max_iter >= 0,
 * recompute >= 0), CHOL_ERR_WORKSPACE, CHOL_ERR_UNSUPPORTED (tile) or
 * CHOL_ERR_HIP.  A that is not positive definite gives NaN or a
 * non-converged result; it is not detected otherwise.                     */
#define CG_MAX_RHS 16
size_t cg_workspace_bytes(int64_t n, int tile, int64_t nrhs);
int cg_solve(const double *A, int64_t n, int64_t lda, int tile, const double *B, int64_t ldb,
             double *X, int64_t ldx, int64_t nrhs, double eps, int64_t max_iter,
             int64_t recompute, void *workspace, size_t ws_bytes, int64_t *iters,
             double *relres, void *stream);

/* ---- heterogeneous CPU + GPU conjugate gradients -----------------------
 * The paper's heterogeneous CG (Implementation, "CG implementation";
 * Results, the heterogeneous CG workload distribution and its comparison
 * with the homogeneous runs): the CG iteration of cg_solve (one right-hand
 * side, FP64, tile 128) with the packed lower-tile matrix and every vector
 * split horizontally at a tile row S.  The GPU owns the rows above the
 * split and streams the tiles of its leading S x S triangle; the host CPU
 * owns the rows below and streams all tiles of its rows (its triangle and
 * the rectangle left of it, whose transposed products it sends to the GPU
 * as one vector per product).  Per iteration the two partial sums of s.t
 * and of r.r cross to the host (and the CPU's to the device, so that both
 * sides form the same scalars in the same order), and the two halves of s
 * change sides; an iteration that recomputes the true residual also
 * exchanges x.  S is the largest tile row with S (S + 1) / 2 <= gpu_share
 * N (N + 1) / 2 (gpu_share: the fraction of the stored tiles in the GPU's
 * triangle; 1 = the GPU alone, 0 = the CPU alone).
 * A, lda      : device, n x n column-major FP64 (lower triangle read),
 *               packed into the workspace at the start of the call.
 * B, X        : device, n FP64 each; X holds the starting guess on entry and
 *               the final iterate on exit.
 * eps, max_iter, recompute: as cg_solve.
 * workspace   : device, 256-byte aligned, >= cg_hetero_workspace_bytes(n).
 * host_ws     : HOST memory (pinned makes the copies asynchronous), >=
 *               cg_hetero_host_bytes(n, gpu_share): the CPU's tiles, their
 *               products and the host halves of the vectors.
 * iters, relres: out (host), may be NULL: iterations, sqrt(u / u0) at exit.
 * rep         : out, may be NULL.
 * Synchronous.  Returns CHOL_OK, CHOL_ERR_NOT_CONVERGED (max_iter reached),
 * -1 A, -2 n, -3 lda, -4 B or X NULL, -6 eps, -7 max_iter, -8 recompute,
 * -9 gpu_share outside [0, 1], -10 workspace, CHOL_ERR_WORKSPACE, -12
 * host_ws, CHOL_ERR_HIP.                                                   */
typedef struct {
  double gpu_share_target;  /* as requested                                  */
  double gpu_share_tiles;   /* stored tiles in the GPU's triangle / all       */
  double bytes_h2d, bytes_d2h;
  double ms_total;          /* wall time of the call                          */
  double ms_cpu;            /* host time in the CPU's tile products           */
  double ms_wait_gpu;       /* host time waiting for the GPU                  */
  int32_t iterations;
  int32_t recomputations;
  int32_t gpu_rows;         /* S, tile rows on the GPU                        */
  int32_t cpu_threads;
} cg_hetero_report;

size_t cg_hetero_workspace_bytes(int64_t n);
size_t cg_hetero_host_bytes(int64_t n, double gpu_share);
int cg_solve_hetero(const double *A, int64_t n, int64_t lda, const double *B, double *X,
                    double eps, int64_t max_iter, int64_t recompute, double gpu_share,
                    void *workspace, size_t ws_bytes, void *host_ws, size_t host_bytes,
                    int64_t *iters, double *relres, cg_hetero_report *rep, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CHOL_MI355X_H */
