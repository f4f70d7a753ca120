// Step 1 and Step 2 of the blocked right-looking Cholesky factorisation (the
// paper's algorithm figure, right column; Fundamentals, "The Cholesky
// decomposition"):
//   Step 1  A_cc <- Cholesky(A_cc)           (potrf_kernel)
//   Step 2  A_ic <- A_ic * A_cc^{-T}, i > c  (trsm_kernel)
// Both always compute in FP64, whatever the storage precision of the tiles;
// results are rounded to the storage type on the way out.  Both use
// substitution (no explicit inverse), so a factor whose entries are exact
// small integers is reproduced bit for bit.  The same substitution applied
// to the identity gives the inverted diagonal blocks L_cc^{-T} that the
// triangular solves use (diag_inverse_kernel, run once after the factorisation).
#include "internal.hpp"

namespace chol {
namespace {

// ---------------------------------------------------------------- Step 1 --
__device__ inline double readlane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// x L^T = rhs for one row x of 16 values against a 16 x 16 lower block L in
// LDS (row pitch PP) with reciprocal diagonal rdv: column by column, x_j is
// scaled and then subtracted from the later x_i (the same operations in the
// same order as the row-wise substitution), column j + 1 of L being read
// while column j is applied.
// LEAN reads each reciprocal diagonal entry one column ahead instead of all
// of them up front (fewer registers live at once).
template <int NB, int PP, bool LEAN = false>
__device__ __forceinline__ void row_solve(double (&x)[NB], const double *l, const double *rdv) {
  double rv[NB], col[2][NB];
  if (!LEAN) {
#pragma unroll
    for (int j = 0; j < NB; ++j) rv[j] = rdv[j];
  } else {
    rv[0] = rdv[0];  // then each entry one column ahead, with the column of L
  }
#pragma unroll
  for (int i = 1; i < NB; ++i) col[0][i] = l[i * PP];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j + 1 < NB) {
#pragma unroll
      for (int i = j + 2; i < NB; ++i) col[(j + 1) & 1][i] = l[i * PP + j + 1];
      if (LEAN) rv[j + 1] = rdv[j + 1];
    }
    x[j] *= rv[j];
#pragma unroll
    for (int i = j + 1; i < NB; ++i) x[i] -= x[j] * col[j & 1][i];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One workgroup of 256 threads factors a B x B diagonal tile in FP64,
// blocked by 16 columns (right-looking).  The trailing part of the tile lives
// in registers: threads form a 16 x 16 grid and thread (tr, tc) owns the
// elements (tr + 16 m, tc + 16 n) of the trailing submatrix, m, n < B/16 --
// one element of every 16 x 16 block.  For each block column:
//   (1) the diagonal block goes to LDS (one element per thread);      barrier
//   (2) one wave factors it, lane l holding row l: per column the pivot
//       comes by readlane and the scaled column goes through LDS to the
//       wave (in-order LDS within a wave, no barrier);                 barrier
//   (3) the panel below goes to LDS;                                   barrier
//       one thread per panel row solves X L_kk^T = P by substitution
//       (multiplying by the reciprocal diagonal);                      barrier
//   (4) every thread applies the rank-16 update to its trailing elements,
//       and the finished 16 columns go from LDS to HBM;                 barrier
//   (5) the registers shift by one block, so the next diagonal block is
//       again at register index 0 (all register indices stay compile-time
//       while the block loop itself is not unrolled).
// So a tile costs 5 barriers per 16 columns instead of 2 per column.  A
// failed pivot is reported by the wave of step (2) and every thread leaves
// after the barrier.  The tile is loaded through LDS a quarter at a time
// (contiguous global reads).  LDS below 36 KB.
//
// LA (lookahead inside the tile, 320 threads): a fifth wave holds no tile
// elements and does every 16 x 16 diagonal factorisation.  In block kb the
// owners first apply block kb's rank-16 update to the next diagonal block
// alone and hand it over through LDS; the fifth wave factors it while the
// owners apply the rest of the update and store block kb's columns.  The
// diagonal chain (16 dependent pivots) then runs beside the update instead
// of after it.  Every element sees the same operations in the same order
// as without lookahead, so the factor is bitwise the same.
template <int B, typename T, bool LA = false>
__device__ __forceinline__ void potrf_body(T *__restrict__ tiles, int64_t N, int64_t c,
                                           int64_t *__restrict__ info) {
  if (*info != 0) return;
  constexpr int M = B / 16;
  constexpr int NB = 16;
  constexpr int PP = NB + 2;  // pitch of the diagonal block and the panel (16-byte rows)
  constexpr int QC = 32;      // columns per staging quarter
  constexpr int LD = B + 1;
  constexpr int WORK = 2 * NB * PP + (B - NB) * PP + 4 * NB;
  constexpr int SMEM = (QC * LD > WORK) ? QC * LD : WORK;
  constexpr int DW = LA ? 256 : 0;  // first thread of the wave that factors diagonal blocks
  __shared__ __attribute__((aligned(16))) double sm[SMEM];
  __shared__ int fail;
  double *stage = sm;                        // QC x LD, while loading
  double *pn = sm + 2 * NB * PP;             // (B - NB) x PP panel below the diagonal block
  double *cb = pn + (B - NB) * PP;           // column broadcast of the factorisation
  // diagonal blocks (NB x PP) and their reciprocal diagonals, alternating by block
  auto dgs = [&](int kb) { return sm + (kb & 1) * NB * PP; };
  auto rds = [&](int kb) { return cb + NB + (kb & 1) * NB; };
  T *tile = tiles + tile_index(c, c, N) * (int64_t)(B * B);
  const int t = threadIdx.x, tc = t & 15, tr = (t >> 4) & 15;
  const bool owner = t < 256;
  if (t == 0) fail = 0;
  double a[M][M];
  {
    // all loads of a quarter are issued before any LDS store (one latency per quarter)
    constexpr int QV = QC * B / 256;
    T nxt[QV];
    if (owner) {
#pragma unroll
      for (int x = 0; x < QV; ++x) nxt[x] = tile[t + 256 * x];
    }
#pragma unroll
    for (int q4 = 0; q4 < B / QC; ++q4) {
      T cur[QV];
      if (owner) {
#pragma unroll
        for (int x = 0; x < QV; ++x) cur[x] = nxt[x];
        if (q4 + 1 < B / QC) {
#pragma unroll
          for (int x = 0; x < QV; ++x) nxt[x] = tile[(q4 + 1) * QC * B + t + 256 * x];
        }
#pragma unroll
        for (int x = 0; x < QV; ++x) {
          const int e = t + 256 * x, r = e % B, cc = e / B;
          stage[cc * LD + r] = (double)cur[x];
        }
      }
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
          for (int nn = 0; nn < 2; ++nn)
            a[m][2 * q4 + nn] = stage[(tc + 16 * nn) * LD + tr + 16 * m];
      }
      __syncthreads();
    }
  }

  // one wave (lanes l = t - DW) factors the 16 x 16 block dg in place and
  // leaves its reciprocal diagonal in rd; returns the first failed pivot
  // (1-based) of block kb through info / fail
  auto factor_diag = [&](double *dg, double *rd, int kb) {
    const int l = t - DW;
    double x[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = (l < NB) ? dg[l * PP + j] : 0.0;
    int bad = 0;  // first failed pivot (1-based); uniform across the wave
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      double d = readlane_f64(x[k], k);
      if (!(d > 0.0)) {
        if (!bad) bad = k + 1;
        d = 1.0;  // keep going without NaNs; the result is discarded
      }
      // the pivot's reciprocal square root, and the square root as d times
      // it: one rounding more than a correctly rounded sqrt, but the
      // latter's refinement chain was the longest part of this loop
      // (POTRF 58.6 -> 48.7 us); exact for the powers of four that the
      // exact-arithmetic inputs produce
      const double rl = rsqrt(d);
      const double lkk = d * rl;
      x[k] = (l == k) ? lkk : (l > k ? x[k] * rl : x[k]);
      if (l == k) rd[k] = rl;
      if (l < NB) cb[l] = x[k];
#pragma unroll
      for (int j = k + 1; j < NB; ++j) x[j] -= x[k] * cb[j];
      __builtin_amdgcn_sched_barrier(0);
    }
    if (bad) {
      if (l == 0) {
        *info = c * B + kb * NB + bad;
        fail = 1;
      }
    } else if (l < NB) {
#pragma unroll
      for (int j = 0; j < NB; ++j) dg[l * PP + j] = x[j];
    }
  };

  if (LA) {
    // the first diagonal block, factored before the loop
    if (owner) dgs(0)[tr * PP + tc] = a[0][0];
    __syncthreads();
    if (t >= DW) factor_diag(dgs(0), rds(0), 0);
    __syncthreads();
    if (fail) return;  // uniform
  }
#pragma unroll 1
  for (int kb = 0; kb < M; ++kb) {
    const int rem = M - kb;  // register blocks still trailing
    double *dg = dgs(kb), *rd = rds(kb);
    if (!LA) {
      // (1) diagonal block to LDS
      dg[tr * PP + tc] = a[0][0];
      __syncthreads();
      // (2) one wave factors it
      if (t < 64) factor_diag(dg, rd, kb);
      __syncthreads();
      if (fail) return;  // uniform
    }
    if (kb + 1 < M) {
      // (3) panel below to LDS, solved row by row
      const int PR = B - NB * (kb + 1);
      if (owner) {
#pragma unroll
        for (int m = 1; m < M; ++m)
          if (m < rem) pn[(tr + 16 * (m - 1)) * PP + tc] = a[m][0];
      }
      __syncthreads();
      if (t < PR) {
        double x[NB];
#pragma unroll
        for (int j = 0; j < NB; j += 2) *(double2 *)&x[j] = *(const double2 *)&pn[t * PP + j];
        row_solve<NB, PP>(x, dg, rd);
#pragma unroll
        for (int j = 0; j < NB; j += 2) *(double2 *)&pn[t * PP + j] = *(const double2 *)&x[j];
      }
      __syncthreads();
      if (LA) {
        // (4a) the next diagonal block's update first, handed to the fifth wave
        if (owner) {
#pragma unroll
          for (int k = 0; k < NB; k += 2) {
            const double2 pr = *(const double2 *)&pn[tr * PP + k];
            const double2 pc = *(const double2 *)&pn[tc * PP + k];
            a[1][1] -= pr.x * pc.x;
            a[1][1] -= pr.y * pc.y;
          }
          dgs(kb + 1)[tr * PP + tc] = a[1][1];
        }
        __syncthreads();
        if (t >= DW) factor_diag(dgs(kb + 1), rds(kb + 1), kb + 1);
      }
      // (4) rank-16 update of the trailing elements (blocks m >= n >= 1;
      // with LA the block (1, 1) is done)
      if (owner) {
#pragma unroll
        for (int k = 0; k < NB; k += 2) {
          double2 pr[M], pc[M];
#pragma unroll
          for (int m = 1; m < M; ++m) {
            pr[m] = *(const double2 *)&pn[(tr + 16 * (m - 1)) * PP + k];
            pc[m] = *(const double2 *)&pn[(tc + 16 * (m - 1)) * PP + k];
          }
#pragma unroll
          for (int m = 1; m < M; ++m)
            if (m < rem) {
#pragma unroll
              for (int n = 1; n <= m; ++n) {
                if (LA && m == 1 && n == 1) continue;
                a[m][n] -= pr[m].x * pc[n].x;
                a[m][n] -= pr[m].y * pc[n].y;
              }
            }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // the finished 16 columns (zero above the diagonal) from LDS to HBM
    if (owner) {
      const int j0 = NB * kb;
      for (int e = t; e < NB * B; e += 256) {
        const int r = e % B, jj = e / B, j = j0 + jj;
        double v = 0.0;
        if (r >= j) v = (r < j0 + NB) ? dg[(r - j0) * PP + jj] : pn[(r - j0 - NB) * PP + jj];
        tile[(int64_t)j * B + r] = (T)v;
      }
    }
    __syncthreads();
    if (LA && fail) return;  // the next diagonal block failed (uniform)
    // (5) shift: the next diagonal block moves to register index 0
#pragma unroll
    for (int m = 0; m + 1 < M; ++m)
#pragma unroll
      for (int n = 0; n + 1 < M; ++n) a[m][n] = a[m + 1][n + 1];
  }
}

template <int B, typename T>
__global__ __launch_bounds__(256) void potrf_kernel(T *__restrict__ tiles, int64_t N, int64_t c,
                                                    int64_t *__restrict__ info) {
  potrf_body<B, T, false>(tiles, N, c, info);
}

// with the fifth-wave lookahead: 320 threads
template <int B, typename T>
__global__ __launch_bounds__(320) void potrf_la_kernel(T *__restrict__ tiles, int64_t N,
                                                       int64_t c, int64_t *__restrict__ info) {
  potrf_body<B, T, true>(tiles, N, c, info);
}

// ---------------------------------------------------------------- Step 2 --
// X L^T = A for a tile, L = L_cc: each row of X is an independent forward
// substitution.  One workgroup of 256 threads per tile, blocked by 16
// columns.  Column block q of L (rows 16q .. B-1, 16 columns) is staged in
// LDS (pitch 18, double-buffered: block q+1 is loaded into registers while
// block q is processed), with the reciprocal diagonal of L.  The unsolved
// part of the tile lives in registers, thread (tr, tc) owning elements
// (tr + 16 m, tc + 16 n).  For each column block:
//   (1) the owners copy the block of X to LDS;                        barrier
//   (2) one thread per row solves its 16 values against the 16 x 16
//       diagonal block of L by substitution;                           barrier
//   (3) the solved block goes to HBM and every thread subtracts its
//       product with the block's part of L from its remaining columns;
//                                                                      barrier
//   (4) the registers shift by one block column (compile-time indices
//       while the block loop is not unrolled).
// IDENT: the right-hand side is the identity (X is only written), which
// gives X = L^{-T}: the inverted diagonal blocks of the solves.
// RB < B: the workgroup solves only rows [r0, r0 + RB) of the tile (the rows
// are independent), so B / RB workgroups share a tile; thread (tr, tc) then
// owns elements (r0 + tr + 16 m, tc + 16 n), m < RB / 16, and the column
// updates shrink with the rows, while the row solves (2) keep their length.
template <int B, typename T, bool IDENT, int RB = B>
__device__ __forceinline__ void trsm_tile(const T *__restrict__ L, T *__restrict__ X, int r0 = 0) {
  constexpr int M = B / 16, MR = RB / 16, NB = 16, PP = NB + 2;
  constexpr int PF = (B * NB + 255) / 256;                  // prefetched L values per thread
  __shared__ __attribute__((aligned(16))) double ls[2][B * PP];  // L column blocks
  __shared__ __attribute__((aligned(16))) double px[B * PP];     // current block of X
  __shared__ double rdl[B];                                      // 1 / L_jj
  const int t = threadIdx.x, tc = t & 15, tr = t >> 4;
  // column block q of L: element (16 q + r, 16 q + u), r < B - 16 q, u < 16
  auto lget = [&](int q, double (&v)[PF]) {
    const int rows = B - 16 * q;
#pragma unroll
    for (int x = 0; x < PF; ++x) {
      const int e = t + 256 * x, r = e % rows, u = e / rows;
      v[x] = (e < rows * NB) ? (double)L[(int64_t)(16 * q + u) * B + 16 * q + r] : 0.0;
    }
  };
  auto lput = [&](int q, const double (&v)[PF]) {
    const int rows = B - 16 * q;
#pragma unroll
    for (int x = 0; x < PF; ++x) {
      const int e = t + 256 * x, r = e % rows, u = e / rows;
      if (e < rows * NB) ls[q & 1][r * PP + u] = v[x];
    }
  };
  double a[MR][M];
  if (IDENT) {
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
      for (int n = 0; n < M; ++n) a[m][n] = (r0 + tr + 16 * m == tc + 16 * n) ? 1.0 : 0.0;
  } else {
    // the rows into registers through LDS (the L buffers, not yet in use),
    // 32 columns at a time with contiguous reads, the next group's loads in
    // flight while the current one is redistributed
    constexpr int QC = 32, LD = RB + 1, QV = QC * RB / 256;
    static_assert(QC * LD <= 2 * B * PP, "staging fits in the L buffers");
    double *stg = &ls[0][0];
    auto src = [&](int q4, int x) -> const T & {
      const int e = t + 256 * x, r = e % RB, cc = e / RB;
      return X[(int64_t)(q4 * QC + cc) * B + r0 + r];
    };
    T nxt[QV];
#pragma unroll
    for (int x = 0; x < QV; ++x) nxt[x] = src(0, x);
#pragma unroll
    for (int q4 = 0; q4 < B / QC; ++q4) {
      T cur[QV];
#pragma unroll
      for (int x = 0; x < QV; ++x) cur[x] = nxt[x];
      if (q4 + 1 < B / QC) {
#pragma unroll
        for (int x = 0; x < QV; ++x) nxt[x] = src(q4 + 1, x);
      }
      if (q4 > 0) __syncthreads();  // previous group fully read
#pragma unroll
      for (int x = 0; x < QV; ++x) {
        const int e = t + 256 * x, r = e % RB, cc = e / RB;
        stg[cc * LD + r] = (double)cur[x];
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int nn = 0; nn < 2; ++nn)
          a[m][2 * q4 + nn] = stg[(tc + 16 * nn) * LD + tr + 16 * m];
    }
    __syncthreads();  // staging done before the L buffers are filled
  }
  {
    double v[PF];
    lget(0, v);
    lput(0, v);
  }
  for (int e = t; e < B; e += 256) rdl[e] = 1.0 / (double)L[(int64_t)e * B + e];
#pragma unroll 1
  for (int q = 0; q < M; ++q) {
    const double *lq = ls[q & 1];  // rows 16q.. of L, pitch PP
    double nxt[PF];
    // (1) block q of X to LDS
#pragma unroll
    for (int m = 0; m < MR; ++m) px[(tr + 16 * m) * PP + tc] = a[m][0];
    __syncthreads();
    // (2) one thread per row: x L_qq^T = rhs
    if (t < RB) {
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; j += 2) *(double2 *)&x[j] = *(const double2 *)&px[t * PP + j];
      row_solve<NB, PP, true>(x, lq, rdl + 16 * q);
#pragma unroll
      for (int j = 0; j < NB; j += 2) *(double2 *)&px[t * PP + j] = *(const double2 *)&x[j];
    }
    __syncthreads();
    // the next column block of L is loaded while this block is applied
    if (q + 1 < M) lget(q + 1, nxt);
    // (3) the solved block to HBM; update of the remaining columns
    for (int e = t; e < RB * NB; e += 256) {
      const int r = e % RB, u = e / RB;
      X[(int64_t)(16 * q + u) * B + r0 + r] = (T)px[r * PP + u];
    }
#pragma unroll
    for (int k = 0; k < NB; k += 2) {
      double2 xr[MR], lc[M];
#pragma unroll
      for (int m = 0; m < MR; ++m) xr[m] = *(const double2 *)&px[(tr + 16 * m) * PP + k];
#pragma unroll
      for (int n = 1; n < M; ++n) lc[n] = *(const double2 *)&lq[(tc + 16 * n) * PP + k];
#pragma unroll
      for (int n = 1; n < M; ++n)
        if (n < M - q) {
#pragma unroll
          for (int m = 0; m < MR; ++m) {
            a[m][n] -= xr[m].x * lc[n].x;
            a[m][n] -= xr[m].y * lc[n].y;
          }
        }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (q + 1 < M) lput(q + 1, nxt);  // the other buffer: last read in block q-1
    __syncthreads();
    // (4) shift: the next block column moves to register index 0
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
      for (int n = 0; n + 1 < M; ++n) a[m][n] = a[m][n + 1];
  }
}

// B / RB workgroups per tile, each solving RB of its rows.
template <int B, typename T, int RB>
__global__ __launch_bounds__(256) void trsm_kernel(T *__restrict__ tiles, int64_t N, int64_t c,
                                                   int64_t r0, const int64_t *__restrict__ info) {
  if (*info != 0) return;
  constexpr int SPLIT = B / RB;
  const int64_t i = r0 + blockIdx.x / SPLIT;
  trsm_tile<B, T, false, RB>(tiles + tile_index(c, c, N) * (int64_t)(B * B),
                             tiles + tile_index(i, c, N) * (int64_t)(B * B),
                             (int)(blockIdx.x % SPLIT) * RB);
}

// Inverted diagonal blocks for the solves: block c of dinv = L_cc^{-T}
// (column-major), B / RB workgroups per diagonal tile, each solving RB rows
// of the identity (the rows are independent, as in the panel solve).
template <int B, typename T, int RB = B>
__global__ __launch_bounds__(256) void diag_inverse_kernel(const T *__restrict__ tiles, int64_t N,
                                                           T *__restrict__ dinv,
                                                           const int64_t *__restrict__ info,
                                                           int64_t c0) {
  if (*info != 0) return;
  constexpr int SPLIT = B / RB;
  const int64_t c = c0 + blockIdx.x / SPLIT;
  trsm_tile<B, T, true, RB>(tiles + tile_index(c, c, N) * (int64_t)(B * B),
                            dinv + c * (int64_t)(B * B), (int)(blockIdx.x % SPLIT) * RB);
}

// Panel solve of the FP16 form through the inverted diagonal block: for the
// tiles (i, c), i in (c, N), X = A D with D = L_cc^{-T} (block c of dinv,
// column-major, computed right after the diagonal factorisation; the solves
// use the same blocks), as one FP32 matrix-core product per tile
// (v_mfma_f32_16x16x4_f32, the lane layout of the FP32 trailing update:
// acc[s2][u][e] = X(64 wm + 16 g + 4 e + s2, 64 wn + 4 q + u)).  A is staged
// as stored, D transposed (the B operand at contraction index k, output
// column s is D(k, s)), 32 columns at a time.  The tile is overwritten only
// after all of it has been read.  X then goes once more, rounded to FP16,
// into the tile's two 64-column chunks of the panel buffer (p16c: the chunks
// of tile column c for tile row 0), through LDS, one chunk at a time.  A
// matrix-core product instead of 128 dependent substitution steps: the FP16
// form's panel solves run beside its trailing updates, and this way they hold
// a CU for a fraction of the time.
__global__ __launch_bounds__(256) void trsm_inv_kernel(float *__restrict__ tiles, int64_t N,
                                                       int64_t c, const float *__restrict__ D,
                                                       _Float16 *__restrict__ p16c,
                                                       const int64_t *__restrict__ info) {
  constexpr int B = 128, KC = 32, PAD = B + 1;
  typedef float v4f __attribute__((ext_vector_type(4)));
  typedef _Float16 v8h __attribute__((ext_vector_type(8)));
  if (*info != 0) return;
  const int64_t i = c + 1 + blockIdx.x;
  float *X = tiles + tile_index(i, c, N) * (int64_t)(B * B);
  const float *Dc = D + c * (int64_t)(B * B);
  __shared__ __attribute__((aligned(16))) float la[KC * B], lb[KC * B];  // [k][row or column]
  __shared__ float st[64 * PAD];                                         // [column][row]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15, wm = wave >> 1, wn = wave & 1;
  v4f acc[4][4];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[s2][u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int k0 = 0; k0 < B; k0 += KC) {
    // A: columns k0 .. k0+31 of the tile, contiguous
#pragma unroll
    for (int x = 0; x < KC * B / 1024; ++x) {
      const int e = 4 * (tid + 256 * x);
      *(v4f *)&la[e] = *(const v4f *)&X[(int64_t)k0 * B + e];
    }
    // D transposed: lb[kk * B + s] = D(k0 + kk, s) = Dc[s * B + k0 + kk]
#pragma unroll
    for (int x = 0; x < KC * B / 1024; ++x) {
      const int e = tid + 256 * x, sc = e / (KC / 4), kk = 4 * (e % (KC / 4));
      const v4f v = *(const v4f *)&Dc[(int64_t)sc * B + k0 + kk];
#pragma unroll
      for (int y = 0; y < 4; ++y) lb[(kk + y) * B + sc] = v[y];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const v4f fa = *(const v4f *)&la[(4 * ks + g) * B + 64 * wm + 4 * q];
      const v4f fb = *(const v4f *)&lb[(4 * ks + g) * B + 64 * wn + 4 * q];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc[s2][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s2], fb[u], acc[s2][u], 0, 0, 0);
    }
    __syncthreads();  // the chunk's LDS is refilled next
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const v4f v = {acc[0][u][e], acc[1][u][e], acc[2][u][e], acc[3][u][e]};
      *(v4f *)&X[(int64_t)(64 * wn + 4 * q + u) * B + 64 * wm + 16 * g + 4 * e] = v;
    }
  // FP16 copy: columns 64 h .. 64 h + 63 (the waves with wn == h) through LDS
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    if (wn == h) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2)
            st[(4 * q + u) * PAD + 64 * wm + 16 * g + 4 * e + s2] = acc[s2][u][e];
    }
    __syncthreads();
    _Float16 *dst = p16c + (i * kP16ChunksPerTileRow + h) * (int64_t)(B * 64);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int e = tid + 256 * x, r = e / 8, sg = e % 8;
      v8h v;
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (_Float16)st[(8 * sg + j) * PAD + r];
      *(v8h *)(dst + p16_pos(r, sg)) = v;
    }
    __syncthreads();  // st is refilled for the second chunk
  }
}

// Batched column step of several factorisations at once (the serving
// engine): job j of the descriptor is at tile column c_j of its own packed
// matrix.  One workgroup per job factors its diagonal tile (with the
// fifth-wave lookahead: the serving orders are small, their column chain is
// the whole latency); the panel solves of all jobs form one flat list of
// quarter tiles (a quarter of a tile's rows each) that a fixed grid walks.
template <int B, typename T>
__global__ __launch_bounds__(320) void batch_potrf_kernel(const BatchDesc *__restrict__ d) {
  const int64_t j = blockIdx.x;
  if (j >= d->njobs) return;
  const BatchJob &J = d->jobs[j];
  potrf_body<B, T, true>((T *)J.tiles, J.N, J.c, J.info);
}

template <int B, typename T>
__global__ __launch_bounds__(256) void batch_trsm_kernel(const BatchDesc *__restrict__ d) {
  constexpr int RB = B / 4;
  const int64_t total = 4 * d->trsm_total, nj = d->njobs;
  for (int64_t t4 = blockIdx.x; t4 < total; t4 += gridDim.x) {
    const int64_t t = t4 / 4;
    int64_t j = 0;
    while (j + 1 < nj && d->jobs[j + 1].trsm_begin <= t) ++j;
    const BatchJob &J = d->jobs[j];
    if (*J.info != 0) continue;  // uniform over the workgroup
    T *tiles = (T *)J.tiles;
    const int64_t i = J.c + 1 + (t - J.trsm_begin);
    trsm_tile<B, T, false, RB>(tiles + tile_index(J.c, J.c, J.N) * (int64_t)(B * B),
                               tiles + tile_index(i, J.c, J.N) * (int64_t)(B * B),
                               (int)(t4 % 4) * RB);
    __syncthreads();  // the tile's LDS is reused by the next one
  }
}

template <int B>
void potrf_dispatch(void *tiles, int store, int64_t N, int64_t c, int64_t *info, hipStream_t s,
                    bool la) {
  if (la) {
    if (store == STORE_F64)
      hipLaunchKernelGGL((potrf_la_kernel<B, double>), dim3(1), dim3(320), 0, s,
                         (double *)tiles, N, c, info);
    else
      hipLaunchKernelGGL((potrf_la_kernel<B, float>), dim3(1), dim3(320), 0, s, (float *)tiles,
                         N, c, info);
  } else if (store == STORE_F64) {
    hipLaunchKernelGGL((potrf_kernel<B, double>), dim3(1), dim3(256), 0, s, (double *)tiles, N,
                       c, info);
  } else {
    hipLaunchKernelGGL((potrf_kernel<B, float>), dim3(1), dim3(256), 0, s, (float *)tiles, N, c,
                       info);
  }
}

// Column steps with at most this many tiles below the diagonal split each
// tile's panel solve over four workgroups (option "trsm_split").
int64_t g_trsm_split_max = 64;

template <int B>
void trsm_dispatch(void *tiles, int store, int64_t N, int64_t c, const int64_t *info,
                   hipStream_t s, int64_t r0) {
  if (r0 <= c) r0 = c + 1;
  const int64_t nt = N - r0;
  if (nt <= 0) return;
  // few tiles (small matrices, the last columns): four workgroups per tile,
  // a quarter of the rows each, for a shorter chain; whole tiles otherwise
  if (nt <= g_trsm_split_max) {
    constexpr int RB = B / 4;
    const dim3 grid((unsigned)(4 * nt));
    if (store == STORE_F64)
      hipLaunchKernelGGL((trsm_kernel<B, double, RB>), grid, dim3(256), 0, s, (double *)tiles, N,
                         c, r0, info);
    else
      hipLaunchKernelGGL((trsm_kernel<B, float, RB>), grid, dim3(256), 0, s, (float *)tiles, N, c,
                         r0, info);
  } else if (store == STORE_F64) {
    hipLaunchKernelGGL((trsm_kernel<B, double, B>), dim3((unsigned)nt), dim3(256), 0, s,
                       (double *)tiles, N, c, r0, info);
  } else {
    hipLaunchKernelGGL((trsm_kernel<B, float, B>), dim3((unsigned)nt), dim3(256), 0, s,
                       (float *)tiles, N, c, r0, info);
  }
}

}  // namespace

void set_trsm_split_max(int64_t tiles) { g_trsm_split_max = tiles; }

void launch_potrf(void *tiles, int store, int b, int64_t N, int64_t c, int64_t *info,
                  hipStream_t s, bool la) {
  if (c < 0 || c >= N) return;  // no such diagonal tile
  if (b == 128)
    potrf_dispatch<128>(tiles, store, N, c, info, s, la);
  else
    potrf_dispatch<64>(tiles, store, N, c, info, s, la);
}

void launch_trsm_inv(void *tiles, int64_t N, int64_t c, void *dinv, void *p16c,
                     const int64_t *info, hipStream_t s) {
  if (c < 0 || c >= N) return;
  hipLaunchKernelGGL((diag_inverse_kernel<128, float, 32>), dim3(4), dim3(256), 0, s,
                     (const float *)tiles, N, (float *)dinv, info, c);
  if (N - c - 1 > 0)
    hipLaunchKernelGGL(trsm_inv_kernel, dim3((unsigned)(N - c - 1)), dim3(256), 0, s,
                       (float *)tiles, N, c, (const float *)dinv, (_Float16 *)p16c, info);
}

void launch_diag_inverse(const void *tiles, int store, int b, int64_t N, void *dinv,
                         const int64_t *info, hipStream_t s) {
  if (N <= 0) return;
  // a quarter of the rows per workgroup where the launch is latency-bound
  // (the split's four workgroups cost more CU time than one)
  const bool split = N <= g_trsm_split_max;
  const dim3 grid((unsigned)(split ? 4 * N : N));
  const int64_t z = 0;
  if (b == 128) {
    if (store == STORE_F64 && split)
      hipLaunchKernelGGL((diag_inverse_kernel<128, double, 32>), grid, dim3(256), 0, s,
                         (const double *)tiles, N, (double *)dinv, info, z);
    else if (store == STORE_F64)
      hipLaunchKernelGGL((diag_inverse_kernel<128, double>), grid, dim3(256), 0, s,
                         (const double *)tiles, N, (double *)dinv, info, z);
    else if (split)
      hipLaunchKernelGGL((diag_inverse_kernel<128, float, 32>), grid, dim3(256), 0, s,
                         (const float *)tiles, N, (float *)dinv, info, z);
    else
      hipLaunchKernelGGL((diag_inverse_kernel<128, float>), grid, dim3(256), 0, s,
                         (const float *)tiles, N, (float *)dinv, info, z);
  } else {
    if (store == STORE_F64 && split)
      hipLaunchKernelGGL((diag_inverse_kernel<64, double, 16>), grid, dim3(256), 0, s,
                         (const double *)tiles, N, (double *)dinv, info, z);
    else if (store == STORE_F64)
      hipLaunchKernelGGL((diag_inverse_kernel<64, double>), grid, dim3(256), 0, s,
                         (const double *)tiles, N, (double *)dinv, info, z);
    else if (split)
      hipLaunchKernelGGL((diag_inverse_kernel<64, float, 16>), grid, dim3(256), 0, s,
                         (const float *)tiles, N, (float *)dinv, info, z);
    else
      hipLaunchKernelGGL((diag_inverse_kernel<64, float>), grid, dim3(256), 0, s,
                         (const float *)tiles, N, (float *)dinv, info, z);
  }
}

void launch_batch_potrf_trsm(const BatchDesc *d, int max_jobs, int trsm_grid, hipStream_t s) {
  hipLaunchKernelGGL((batch_potrf_kernel<128, float>), dim3((unsigned)max_jobs), dim3(320), 0, s, d);
  hipLaunchKernelGGL((batch_trsm_kernel<128, float>), dim3((unsigned)trsm_grid), dim3(256), 0, s, d);
}

void launch_trsm(void *tiles, int store, int b, int64_t N, int64_t c, const int64_t *info,
                 hipStream_t s, int64_t r0) {
  if (b == 128)
    trsm_dispatch<128>(tiles, store, N, c, info, s, r0);
  else
    trsm_dispatch<64>(tiles, store, N, c, info, s, r0);
}

}  // namespace chol
