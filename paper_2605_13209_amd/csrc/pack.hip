// Conversion between a dense column-major FP64 matrix and the packed lower
// tile storage of the factor (only diagonal and below-diagonal blocks, each
// block contiguous and column-major; the paper's storage, Implementation
// section).  HBM-bound copies: one 256-thread workgroup per tile, every
// access a contiguous column segment of the tile.
#include "internal.hpp"

namespace chol {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void pack_kernel(const double *__restrict__ A, int64_t n,
                                                   int64_t lda, T *__restrict__ tiles, int b,
                                                   int64_t N, double scale, int64_t c_begin,
                                                   double diag_shift) {
  const int64_t i = blockIdx.x, c = c_begin + blockIdx.y;
  if (i < c) return;
  T *dst = tiles + tile_index(i, c, N) * (int64_t)b * b;
  const int bb = b * b, lgb = 31 - __clz(b);  // b is a power of two
  for (int e = threadIdx.x; e < bb; e += 256) {
    const int r = e & (b - 1), cc = e >> lgb;
    const int64_t gr = i * b + r, gc = c * b + cc;
    double v;
    if (gr >= n || gc >= n)
      v = (gr == gc) ? 1.0 : 0.0;  // identity padding
    else if (i == c && r < cc)
      v = 0.0;  // strict upper part of a diagonal block
    else
      v = A[gr + gc * lda] * scale + (gr == gc ? diag_shift : 0.0);
    dst[e] = (T)v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void unpack_kernel(const T *__restrict__ tiles, int b, int64_t N,
                                                     int64_t n, double scale,
                                                     double *__restrict__ L, int64_t ldl,
                                                     const int64_t *__restrict__ info) {
  const int64_t i = blockIdx.x, c = blockIdx.y;
  const bool failed = *info != 0;
  const int bb = b * b, lgb = 31 - __clz(b);  // b is a power of two
  const T *src = (i >= c) ? tiles + tile_index(i, c, N) * (int64_t)bb : nullptr;
  for (int e = threadIdx.x; e < bb; e += 256) {
    const int r = e & (b - 1), cc = e >> lgb;
    const int64_t gr = i * b + r, gc = c * b + cc;
    if (gr >= n || gc >= n) continue;
    double v = 0.0;
    if (i > c || (i == c && r >= cc)) v = failed ? __builtin_nan("") : (double)src[e] * scale;
    L[gr + gc * ldl] = v;
  }
}

}  // namespace

void launch_pack(const double *A, int64_t n, int64_t lda, void *tiles, int store, int b,
                 int64_t N, double scale, hipStream_t s, int64_t c_begin, int64_t c_end,
                 double diag_shift) {
  if (c_end < 0 || c_end > N) c_end = N;
  if (N <= 0 || c_begin < 0 || c_begin >= c_end) return;
  dim3 grid((unsigned)N, (unsigned)(c_end - c_begin));
  if (store == STORE_F64)
    hipLaunchKernelGGL(pack_kernel<double>, grid, dim3(256), 0, s, A, n, lda, (double *)tiles, b,
                       N, scale, c_begin, diag_shift);
  else
    hipLaunchKernelGGL(pack_kernel<float>, grid, dim3(256), 0, s, A, n, lda, (float *)tiles, b, N,
                       scale, c_begin, diag_shift);
}

void launch_unpack(const void *tiles, int store, int b, int64_t N, int64_t n, double scale,
                   double *L, int64_t ldl, const int64_t *info, hipStream_t s) {
  if (N <= 0) return;
  dim3 grid((unsigned)N, (unsigned)N);
  if (store == STORE_F64)
    hipLaunchKernelGGL(unpack_kernel<double>, grid, dim3(256), 0, s, (const double *)tiles, b, N,
                       n, scale, L, ldl, info);
  else
    hipLaunchKernelGGL(unpack_kernel<float>, grid, dim3(256), 0, s, (const float *)tiles, b, N, n,
                       scale, L, ldl, info);
}

}  // namespace chol
