// Forward and back substitution with the packed factor (the paper's solve
// step after the factorisation, Fundamentals, "The Cholesky decomposition"):
//   L Y = B  (forward),   L^T X = Y  (back),   in place on B (n x nrhs).
// Arithmetic is FP64; FP32 factor tiles are widened on load.
//
// One launch per tile step s (blocked substitution, right-looking):
//   forward step s : workgroup 0 applies tile (s, s-1) to block row s and
//                    then solves the diagonal block L_ss y_s = b_s; every
//                    other workgroup w applies tile (s+w, s-1) to block row
//                    s+w.  So block row s is final exactly when step s solves
//                    it, and every launch reads one column of tiles.
//   back step s    : the mirror image with the transposed tiles of block
//                    row s+1, solving L_ss^T x_s = y_s.
// The solves are HBM-bound (each tile of L is read once per pass); the
// diagonal solves are one wave per right-hand side with register-resident
// rows and lane broadcasts, without workgroup barriers inside the
// substitution loop (see diag_solve).  Padding rows (>= n) are treated as
// zero and never written, which is exact because the padded factor is
// diag(L, I).
#include "internal.hpp"

namespace chol {
namespace {

constexpr int NC = 8;  // right-hand sides per pass of the off-diagonal update

__device__ inline double readlane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// out_i -= L_t * y_src (TRANS = false) or out_i -= L_t^T * y_src (TRANS = true)
// for one b x b tile L_t; y_src and out are block rows of B.
template <int B, typename T, bool TRANS>
__device__ void apply_tile(const T *__restrict__ Lt, const double *ysrc_base, int64_t src_row0,
                           int64_t dst_row0, double *B_, int64_t ldb, int64_t n, int64_t nrhs,
                           double *ys, double *red, double *lt) {
  constexpr int H = 256 / B;  // threads per output row
  const int tid = threadIdx.x;
  const int o = tid % B, h = tid / B;
  for (int64_t c0 = 0; c0 < nrhs; c0 += NC) {
    const int nc = (int)min<int64_t>(NC, nrhs - c0);
    __syncthreads();
    for (int e = tid; e < B * NC; e += 256) {
      const int m = e % B, cc = e / B;
      const int64_t row = src_row0 + m;
      ys[m * NC + cc] = (cc < nc && row < n) ? ysrc_base[row + (c0 + cc) * ldb] : 0.0;
    }
    double acc[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) acc[cc] = 0.0;
    if constexpr (!TRANS) {
      __syncthreads();
      // out[o] += sum_m L[o][m] y[m]; thread part h takes m = h, h+H, ...
      for (int m = h; m < B; m += H) {
        const double l = (double)Lt[m * B + o];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) acc[cc] += l * ys[m * NC + cc];
      }
    } else {
      // out[o] += sum_r L[r][o] y[r]; stage 32-row slabs of L through LDS so
      // global reads stay contiguous along columns.
      constexpr int RS = 32;
      for (int r0 = 0; r0 < B; r0 += RS) {
        __syncthreads();
        for (int e = tid; e < RS * B; e += 256) {
          const int rr = e % RS, col = e / RS;
          lt[col * (RS + 1) + rr] = (double)Lt[col * B + r0 + rr];
        }
        __syncthreads();
        for (int rr = h; rr < RS; rr += H) {
          const double l = lt[o * (RS + 1) + rr];
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) acc[cc] += l * ys[(r0 + rr) * NC + cc];
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) red[(h * B + o) * NC + cc] = acc[cc];
    __syncthreads();
    if (h == 0) {
      const int64_t row = dst_row0 + o;
      if (row < n) {
        for (int cc = 0; cc < nc; ++cc) {
          double s = red[o * NC + cc];
          for (int hh = 1; hh < H; ++hh) s += red[(hh * B + o) * NC + cc];
          B_[row + (c0 + cc) * ldb] -= s;
        }
      }
    }
  }
}

// Diagonal solve of block row s with a column-major triangular block D:
//   LOWER (forward):  D = L_ss,   solve D y = b  for rows ascending;
//   UPPER (back):     D = L_ss^T, solve D x = y  for rows descending.
// Wave w handles right-hand sides w, w+4, ...; lane l owns rows l + 64 j.
// Step r broadcasts the finished value of row r from its lane (readlane) and
// updates the other rows with column r of D, which is contiguous in memory;
// the column values of 8 steps are loaded ahead of their use.  Divisions are
// multiplications by reciprocals of the diagonal, computed once per lane.
template <int B, typename T, bool UPPER>
__device__ void diag_solve(const T *__restrict__ D, int64_t row0, double *B_, int64_t ldb,
                           int64_t n, int64_t nrhs) {
  constexpr int J = B / 64;
  constexpr int U = 8;  // steps per prefetch batch
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double rinv[J];
#pragma unroll
  for (int j = 0; j < J; ++j) rinv[j] = 1.0 / (double)D[(lane + 64 * j) * B + lane + 64 * j];
  for (int64_t c = wave; c < nrhs; c += 4) {
    double v[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t row = row0 + lane + 64 * j;
      v[j] = (row < n) ? B_[row + c * ldb] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
      const int jr = UPPER ? J - 1 - jj : jj;  // 64-row block holding the pivot rows
      for (int b0 = 0; b0 < 64; b0 += U) {
        double col[U][J];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int r = 64 * jr + (UPPER ? 63 - b0 - q : b0 + q);
#pragma unroll
          for (int j = 0; j < J; ++j) col[q][j] = (double)D[r * B + lane + 64 * j];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int rl = UPPER ? 63 - b0 - q : b0 + q;  // lane holding row r
          const int r = 64 * jr + rl;
          const double xr = readlane_f64(v[jr], rl) * readlane_f64(rinv[jr], rl);
#pragma unroll
          for (int j = 0; j < J; ++j) {
            const int m = lane + 64 * j;
            if (m == r)
              v[j] = xr;
            else if (UPPER ? (m < r) : (m > r))
              v[j] -= col[q][j] * xr;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t row = row0 + lane + 64 * j;
      if (row < n) B_[row + c * ldb] = v[j];
    }
  }
}

template <int B, typename T>
__global__ __launch_bounds__(256) void trsv_fwd_step(const T *__restrict__ tiles, int64_t N,
                                                     int64_t n, int64_t s, double *B_,
                                                     int64_t ldb, int64_t nrhs) {
  __shared__ double ys[B * NC];
  __shared__ double red[256 * NC];
  const int64_t w = blockIdx.x;
  const int64_t i = s + w;  // target block row
  if (s > 0) {
    const T *Lt = tiles + tile_index(i, s - 1, N) * (int64_t)(B * B);
    apply_tile<B, T, false>(Lt, B_, (s - 1) * B, i * B, B_, ldb, n, nrhs, ys, red, nullptr);
  }
  if (w == 0) {
    __threadfence_block();
    __syncthreads();
    diag_solve<B, T, false>(tiles + tile_index(s, s, N) * (int64_t)(B * B), s * B, B_, ldb, n,
                            nrhs);
  }
}

template <int B, typename T>
__global__ __launch_bounds__(256) void trsv_bwd_step(const T *__restrict__ tiles,
                                                     const T *__restrict__ diag_t, int64_t N,
                                                     int64_t n, int64_t s, double *B_,
                                                     int64_t ldb, int64_t nrhs) {
  __shared__ double ys[B * NC];
  __shared__ double red[256 * NC];
  __shared__ double lt[B * 33];
  const int64_t w = blockIdx.x;
  const int64_t i = s - w;  // target block row
  if (s < N - 1) {
    const T *Lt = tiles + tile_index(s + 1, i, N) * (int64_t)(B * B);
    apply_tile<B, T, true>(Lt, B_, (s + 1) * B, i * B, B_, ldb, n, nrhs, ys, red, lt);
  }
  if (w == 0) {
    __threadfence_block();
    __syncthreads();
    diag_solve<B, T, true>(diag_t + s * (int64_t)(B * B), s * B, B_, ldb, n, nrhs);
  }
}

__global__ void scale_kernel(double *B_, int64_t n, int64_t ldb, int64_t nrhs, double alpha) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t r = e % n, c = e / n;
  B_[r + c * ldb] *= alpha;
}

template <int B, typename T>
void trsv_run(const T *tiles, const T *diag_t, int64_t N, int64_t n, double *B_, int64_t ldb,
              int64_t nrhs, bool fwd, hipStream_t st) {
  if (fwd) {
    for (int64_t s = 0; s < N; ++s) {
      const unsigned grid = (s == 0) ? 1u : (unsigned)(N - s);
      hipLaunchKernelGGL((trsv_fwd_step<B, T>), dim3(grid), dim3(256), 0, st, tiles, N, n, s, B_,
                         ldb, nrhs);
    }
  } else {
    for (int64_t s = N - 1; s >= 0; --s) {
      const unsigned grid = (s == N - 1) ? 1u : (unsigned)(s + 1);
      hipLaunchKernelGGL((trsv_bwd_step<B, T>), dim3(grid), dim3(256), 0, st, tiles, diag_t, N, n,
                         s, B_, ldb, nrhs);
    }
  }
}

void trsv_dispatch(const void *tiles, const void *dt, int store, int b, int64_t N, int64_t n,
                   double *B_, int64_t ldb, int64_t nrhs, bool fwd, hipStream_t st) {
  if (N <= 0 || nrhs <= 0) return;
  if (b == 128) {
    if (store == STORE_F64)
      trsv_run<128, double>((const double *)tiles, (const double *)dt, N, n, B_, ldb, nrhs, fwd,
                            st);
    else
      trsv_run<128, float>((const float *)tiles, (const float *)dt, N, n, B_, ldb, nrhs, fwd, st);
  } else {
    if (store == STORE_F64)
      trsv_run<64, double>((const double *)tiles, (const double *)dt, N, n, B_, ldb, nrhs, fwd,
                           st);
    else
      trsv_run<64, float>((const float *)tiles, (const float *)dt, N, n, B_, ldb, nrhs, fwd, st);
  }
}

}  // namespace

void launch_trsv_fwd(const void *tiles, int store, int b, int64_t N, int64_t n, double *B_,
                     int64_t ldb, int64_t nrhs, hipStream_t s) {
  trsv_dispatch(tiles, nullptr, store, b, N, n, B_, ldb, nrhs, true, s);
}

void launch_trsv_bwd(const void *tiles, const void *diag_t, int store, int b, int64_t N,
                     int64_t n, double *B_, int64_t ldb, int64_t nrhs, hipStream_t s) {
  trsv_dispatch(tiles, diag_t, store, b, N, n, B_, ldb, nrhs, false, s);
}

void launch_scale(double *B_, int64_t n, int64_t ldb, int64_t nrhs, double alpha, hipStream_t s) {
  const int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B_, n,
                     ldb, nrhs, alpha);
}

}  // namespace chol
