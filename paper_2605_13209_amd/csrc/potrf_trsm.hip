// Step 1 and Step 2 of the blocked right-looking Cholesky factorisation (the
// paper's algorithm figure, right column; Fundamentals, "The Cholesky
// decomposition"):
//   Step 1  A_cc <- Cholesky(A_cc)           (potrf_kernel)
//   Step 2  A_ic <- A_ic * A_cc^{-T}, i > c  (trsm_kernel)
// Both always compute in FP64, whatever the storage precision of the tiles;
// results are rounded to the storage type on the way out.  Both use
// substitution (no explicit inverse), so a factor whose entries are exact
// small integers is reproduced bit for bit.
#include "internal.hpp"

namespace chol {
namespace {

// ---------------------------------------------------------------- Step 1 --
// One workgroup of 256 threads factors a B x B diagonal tile held in LDS as
// FP64 (column-major, pitch B + 1).  Right-looking, unblocked: for each
// column k the pivot is checked, the column below it is divided by sqrt of
// the pivot, and the trailing lower triangle receives the rank-1 update.
// Thread t owns row k+1+(t mod B) of the trailing block and every
// (256/B)-th column of it, so a wave touches consecutive rows of one column
// (bank-conflict free) and reads L_jk as a broadcast.
template <int B, typename T>
__global__ __launch_bounds__(256) void potrf_kernel(T *__restrict__ tiles, int64_t N, int64_t c,
                                                    int64_t *__restrict__ info) {
  if (*info != 0) return;
  constexpr int LD = B + 1;
  constexpr int JS = 256 / B;  // column stride of a thread in the trailing update
  __shared__ double a[B * LD];
  T *tile = tiles + tile_index(c, c, N) * (int64_t)(B * B);
  const int t = threadIdx.x;
  for (int e = t; e < B * B; e += 256) {
    const int r = e % B, cc = e / B;
    a[cc * LD + r] = (r >= cc) ? (double)tile[e] : 0.0;
  }
  __syncthreads();
  const int ri = t % B, jg = t / B;
  for (int k = 0; k < B; ++k) {
    const double d = a[k * LD + k];
    if (!(d > 0.0)) {  // uniform: every thread read the same pivot
      if (t == 0) *info = c * B + k + 1;
      return;
    }
    const double lkk = sqrt(d);
    __syncthreads();  // all threads hold the pivot before it is overwritten
    if (t == 0) a[k * LD + k] = lkk;
    for (int i = k + 1 + t; i < B; i += 256) a[k * LD + i] = a[k * LD + i] / lkk;
    __syncthreads();
    const int i = k + 1 + ri;
    if (i < B) {
      const double lik = a[k * LD + i];
      for (int j = k + 1 + jg; j <= i; j += JS) a[j * LD + i] -= lik * a[k * LD + j];
    }
    __syncthreads();
  }
  for (int e = t; e < B * B; e += 256) {
    const int r = e % B, cc = e / B;
    tile[e] = (T)((r >= cc) ? a[cc * LD + r] : 0.0);
  }
}

// ---------------------------------------------------------------- Step 2 --
// X L^T = A for every tile (i, c), i in [c+1, N).  Each row of X is an
// independent forward substitution with L = L_cc, so one thread owns one
// row: workgroup = B threads = one tile.  Columns are processed in blocks of
// 16 held in registers; earlier solved values are re-read from the tile in
// global memory (written by the same thread).  L is read with uniform
// addresses, i.e. as broadcasts.
template <int B, typename T>
__global__ __launch_bounds__(B) void trsm_kernel(T *__restrict__ tiles, int64_t N, int64_t c,
                                                 const int64_t *__restrict__ info) {
  if (*info != 0) return;
  constexpr int CB = 16;
  const int64_t i = c + 1 + blockIdx.x;
  const T *__restrict__ L = tiles + tile_index(c, c, N) * (int64_t)(B * B);
  T *X = tiles + tile_index(i, c, N) * (int64_t)(B * B);
  const int r = threadIdx.x;
  for (int q = 0; q < B / CB; ++q) {
    double acc[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) acc[u] = (double)X[(q * CB + u) * B + r];
    for (int m = 0; m < q * CB; ++m) {
      const double xm = (double)X[m * B + r];
#pragma unroll
      for (int u = 0; u < CB; ++u) acc[u] -= xm * (double)L[m * B + q * CB + u];
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
#pragma unroll
      for (int v = 0; v < u; ++v) acc[u] -= acc[v] * (double)L[(q * CB + v) * B + q * CB + u];
      acc[u] = acc[u] / (double)L[(q * CB + u) * B + q * CB + u];
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) X[(q * CB + u) * B + r] = (T)acc[u];
  }
}

template <int B>
void potrf_dispatch(void *tiles, int store, int64_t N, int64_t c, int64_t *info, hipStream_t s) {
  if (store == STORE_F64)
    hipLaunchKernelGGL((potrf_kernel<B, double>), dim3(1), dim3(256), 0, s, (double *)tiles, N, c,
                       info);
  else
    hipLaunchKernelGGL((potrf_kernel<B, float>), dim3(1), dim3(256), 0, s, (float *)tiles, N, c,
                       info);
}

template <int B>
void trsm_dispatch(void *tiles, int store, int64_t N, int64_t c, const int64_t *info,
                   hipStream_t s) {
  const int64_t nt = N - c - 1;
  if (nt <= 0) return;
  if (store == STORE_F64)
    hipLaunchKernelGGL((trsm_kernel<B, double>), dim3((unsigned)nt), dim3(B), 0, s,
                       (double *)tiles, N, c, info);
  else
    hipLaunchKernelGGL((trsm_kernel<B, float>), dim3((unsigned)nt), dim3(B), 0, s, (float *)tiles,
                       N, c, info);
}

}  // namespace

void launch_potrf(void *tiles, int store, int b, int64_t N, int64_t c, int64_t *info,
                  hipStream_t s) {
  if (b == 128)
    potrf_dispatch<128>(tiles, store, N, c, info, s);
  else
    potrf_dispatch<64>(tiles, store, N, c, info, s);
}

void launch_trsm(void *tiles, int store, int b, int64_t N, int64_t c, const int64_t *info,
                 hipStream_t s) {
  if (b == 128)
    trsm_dispatch<128>(tiles, store, N, c, info, s);
  else
    trsm_dispatch<64>(tiles, store, N, c, info, s);
}

}  // namespace chol
