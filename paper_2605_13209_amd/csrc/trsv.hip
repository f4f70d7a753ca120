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
//                    row s+1, solving L_ss^T x_s = y_s with the transposed
//                    copy of the diagonal block kept by the factorisation.
// Each workgroup first copies its whole tile into LDS with contiguous column
// reads (one memory latency per tile), then works from LDS.  The diagonal
// solve is one wave per right-hand side: the finished value of row r is
// broadcast from its lane (readlane) and the other rows are updated with
// column r of the block, read from LDS ahead of use.  Padding rows (>= n)
// are treated as zero and never written, which is exact because the padded
// factor is diag(L, I).
#include "internal.hpp"

namespace chol {
namespace {

__device__ inline double readlane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int B>
struct Smem {
  static constexpr int P = B + 1;          // LDS pitch of a staged tile (odd: conflict-free rows)
  static constexpr int NC = 8;             // right-hand sides per pass of the tile product
  static constexpr size_t tile_off = 0;
  static constexpr size_t ys_off = tile_off + (size_t)B * P;
  static constexpr size_t red_off = ys_off + (size_t)B * NC;
  static constexpr size_t doubles = red_off + (size_t)256 * NC;
};

// Copy a b x b column-major tile into LDS (pitch P), widening to FP64.  Each
// thread keeps 8 independent 16-byte loads in flight before storing them.
template <int B, typename T>
__device__ inline void stage_tile(const T *__restrict__ src, double *dst) {
  constexpr int P = Smem<B>::P;
  constexpr int VE = 16 / sizeof(T);             // elements per 16-byte vector
  constexpr int NVEC = B * B / VE / 256;         // vectors per thread
  constexpr int BATCH = NVEC < 8 ? NVEC : 8;
  const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
#pragma unroll
  for (int b0 = 0; b0 < NVEC; b0 += BATCH) {
    uint4 r[BATCH];
#pragma unroll
    for (int x = 0; x < BATCH; ++x) r[x] = s4[threadIdx.x + 256 * (b0 + x)];
#pragma unroll
    for (int x = 0; x < BATCH; ++x) {
      const int e = (threadIdx.x + 256 * (b0 + x)) * VE;  // first element; same column
      T v[VE];
      __builtin_memcpy(v, &r[x], 16);
      double *d = dst + (e / B) * P + (e % B);
#pragma unroll
      for (int y = 0; y < VE; ++y) d[y] = (double)v[y];
    }
  }
}

// out_i -= L_t y_src (TRANS = false) or out_i -= L_t^T y_src (TRANS = true)
// with L_t staged in LDS; y_src and out are block rows of B.
template <int B, int NCH, bool TRANS>
__device__ void apply_tile(const double *lt, int64_t src_row0, int64_t dst_row0, double *B_,
                           int64_t ldb, int64_t n, int64_t nrhs, double *ys, double *red) {
  constexpr int H = 256 / B;  // threads per output row
  constexpr int P = Smem<B>::P;
  const int tid = threadIdx.x;
  const int o = tid % B, h = tid / B;
  for (int64_t c0 = 0; c0 < nrhs; c0 += NCH) {
    const int nc = (int)min<int64_t>(NCH, nrhs - c0);
    __syncthreads();
    for (int e = tid; e < B * NCH; e += 256) {
      const int m = e % B, cc = e / B;
      const int64_t row = src_row0 + m;
      ys[m * NCH + cc] = (cc < nc && row < n) ? B_[row + (c0 + cc) * ldb] : 0.0;
    }
    __syncthreads();
    double acc[NCH];
#pragma unroll
    for (int cc = 0; cc < NCH; ++cc) acc[cc] = 0.0;
#pragma unroll 8
    for (int m = h; m < B; m += H) {
      // forward: L[o][m];  back: L[m][o]
      const double l = TRANS ? lt[o * P + m] : lt[m * P + o];
#pragma unroll
      for (int cc = 0; cc < NCH; ++cc) acc[cc] += l * ys[m * NCH + cc];
    }
#pragma unroll
    for (int cc = 0; cc < NCH; ++cc) red[(h * B + o) * NCH + cc] = acc[cc];
    __syncthreads();
    if (h == 0) {
      const int64_t row = dst_row0 + o;
      if (row < n) {
        for (int cc = 0; cc < nc; ++cc) {
          double s = red[o * NCH + cc];
          for (int hh = 1; hh < H; ++hh) s += red[(hh * B + o) * NCH + cc];
          B_[row + (c0 + cc) * ldb] -= s;
        }
      }
    }
  }
}

// Diagonal solve with a column-major triangular block D staged in LDS:
//   !UPPER (forward):  D = L_ss,   solve D y = b, rows ascending;
//    UPPER (back):     D = L_ss^T, solve D x = y, rows descending.
// Wave w handles right-hand sides w, w+4, ...; lane l owns rows l + 64 j.
template <int B, bool UPPER>
__device__ void diag_solve(const double *d, int64_t row0, double *B_, int64_t ldb, int64_t n,
                           int64_t nrhs) {
  constexpr int J = B / 64;
  constexpr int P = Smem<B>::P;
  constexpr int U = 8;  // steps per batch of column reads
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double rinv[J];
#pragma unroll
  for (int j = 0; j < J; ++j) rinv[j] = 1.0 / d[(lane + 64 * j) * P + lane + 64 * j];
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
          for (int j = 0; j < J; ++j) col[q][j] = d[r * P + lane + 64 * j];
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

// FWD: workgroup w handles block row i = s + w using tile (i, s-1), and
// workgroup 0 then solves L_ss.  BWD: block row i = s - w using tile
// (s+1, i) transposed, and workgroup 0 then solves L_ss^T (from diag_t).
template <int B, typename T, int NCH, bool FWD>
__global__ __launch_bounds__(256) void trsv_step(const T *__restrict__ tiles,
                                                 const T *__restrict__ diag_t, int64_t N,
                                                 int64_t n, int64_t s, double *B_, int64_t ldb,
                                                 int64_t nrhs) {
  __shared__ double smem[Smem<B>::doubles];
  double *lt = smem + Smem<B>::tile_off;
  double *ys = smem + Smem<B>::ys_off;
  double *red = smem + Smem<B>::red_off;
  const int64_t w = blockIdx.x;
  const bool has_update = FWD ? (s > 0) : (s < N - 1);
  if (has_update) {
    const int64_t i = FWD ? s + w : s - w;
    const T *src = FWD ? tiles + tile_index(i, s - 1, N) * (int64_t)(B * B)
                       : tiles + tile_index(s + 1, i, N) * (int64_t)(B * B);
    stage_tile<B, T>(src, lt);
    apply_tile<B, NCH, !FWD>(lt, FWD ? (s - 1) * B : (s + 1) * B, i * B, B_, ldb, n, nrhs, ys, red);
  }
  if (w == 0) {
    __threadfence_block();
    __syncthreads();
    const T *dsrc = FWD ? tiles + tile_index(s, s, N) * (int64_t)(B * B) : diag_t + s * (int64_t)(B * B);
    stage_tile<B, T>(dsrc, lt);
    __syncthreads();
    diag_solve<B, !FWD>(lt, s * B, B_, ldb, n, nrhs);
  }
}

__global__ void scale_kernel(double *B_, int64_t n, int64_t ldb, int64_t nrhs, double alpha) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t r = e % n, c = e / n;
  B_[r + c * ldb] *= alpha;
}

template <int B, typename T, int NCH>
void trsv_run(const T *tiles, const T *diag_t, int64_t N, int64_t n, double *B_, int64_t ldb,
              int64_t nrhs, bool fwd, hipStream_t st) {
  const size_t sh = 0;  // all LDS is static (Smem<B>)
  if (fwd) {
    for (int64_t s = 0; s < N; ++s) {
      const unsigned grid = (s == 0) ? 1u : (unsigned)(N - s);
      hipLaunchKernelGGL((trsv_step<B, T, NCH, true>), dim3(grid), dim3(256), sh, st, tiles,
                         diag_t, N, n, s, B_, ldb, nrhs);
    }
  } else {
    for (int64_t s = N - 1; s >= 0; --s) {
      const unsigned grid = (s == N - 1) ? 1u : (unsigned)(s + 1);
      hipLaunchKernelGGL((trsv_step<B, T, NCH, false>), dim3(grid), dim3(256), sh, st, tiles,
                         diag_t, N, n, s, B_, ldb, nrhs);
    }
  }
}

template <int B, typename T>
void trsv_rhs(const T *tiles, const T *dt, int64_t N, int64_t n, double *B_, int64_t ldb,
              int64_t nrhs, bool fwd, hipStream_t st) {
  if (nrhs == 1)
    trsv_run<B, T, 1>(tiles, dt, N, n, B_, ldb, nrhs, fwd, st);
  else
    trsv_run<B, T, 8>(tiles, dt, N, n, B_, ldb, nrhs, fwd, st);
}

void trsv_dispatch(const void *tiles, const void *dt, int store, int b, int64_t N, int64_t n,
                   double *B_, int64_t ldb, int64_t nrhs, bool fwd, hipStream_t st) {
  if (N <= 0 || nrhs <= 0) return;
  if (b == 128) {
    if (store == STORE_F64)
      trsv_rhs<128, double>((const double *)tiles, (const double *)dt, N, n, B_, ldb, nrhs, fwd,
                            st);
    else
      trsv_rhs<128, float>((const float *)tiles, (const float *)dt, N, n, B_, ldb, nrhs, fwd, st);
  } else {
    if (store == STORE_F64)
      trsv_rhs<64, double>((const double *)tiles, (const double *)dt, N, n, B_, ldb, nrhs, fwd,
                           st);
    else
      trsv_rhs<64, float>((const float *)tiles, (const float *)dt, N, n, B_, ldb, nrhs, fwd, st);
  }
}

}  // namespace

void launch_trsv_fwd(const void *tiles, const void *diag_t, int store, int b, int64_t N,
                     int64_t n, double *B_, int64_t ldb, int64_t nrhs, hipStream_t s) {
  trsv_dispatch(tiles, diag_t, store, b, N, n, B_, ldb, nrhs, true, s);
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
