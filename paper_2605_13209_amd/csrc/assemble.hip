// Squared-exponential GP covariance assembly and the matrix-free GP residual.
//
// The paper's matrices are GP kernel matrices (Results, Experimental Setup);
// the squared-exponential kernel plus noise is the synthetic stand-in:
//   A_ij = var * exp(-|x_i - x_j|^2 / two_l2)  (i != j),   A_ii = var + noise,
// with two_l2 = 2 * lengthscale^2.  Differences are taken directly and the
// squared distance is summed feature by feature without fused multiply-add,
// so A is bitwise symmetric and each entry differs from a correctly rounded
// evaluation only through exp.
//
// Both kernels are bound by HBM writes (assembly) or FP64 ALU work
// (matrix-free residual), not by matrix-core throughput.
#include "internal.hpp"

namespace chol {
namespace {

constexpr int kAsmTile = 64;   // 64 x 64 output block per workgroup
constexpr int kFeatChunk = 16; // features staged through LDS per pass

// Continue the squared distance s over d more features staged in LDS, in
// feature order, without contraction.
__device__ inline double sqdist(double s, const double *xi, const double *xj, int d) {
#pragma clang fp contract(off)
  for (int k = 0; k < d; ++k) {
    const double t = xi[k] - xj[k];
    s += t * t;
  }
  return s;
}

// grid: (ceil(n/64), ceil(n/64)); block 256.  Block (bx, by) writes rows
// 64*bx.., columns 64*by..; lower-only mode skips blocks above the diagonal.
__global__ __launch_bounds__(256) void gp_assemble_kernel(const double *__restrict__ X, int64_t n,
                                                          int d, int64_t ldx, double two_l2,
                                                          double var, double noise,
                                                          double *__restrict__ A, int64_t lda,
                                                          int full) {
  const int64_t i0 = (int64_t)blockIdx.x * kAsmTile;
  const int64_t j0 = (int64_t)blockIdx.y * kAsmTile;
  if (!full && j0 > i0 + kAsmTile - 1) return;
  __shared__ double xi[kAsmTile][kFeatChunk + 1];
  __shared__ double xj[kAsmTile][kFeatChunk + 1];
  const int t = threadIdx.x;
  const int r = t % kAsmTile;  // row within block (consecutive lanes -> consecutive rows)
  const int cg = t / kAsmTile; // column group 0..3
  double s[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) s[m] = 0.0;
  for (int f0 = 0; f0 < d; f0 += kFeatChunk) {
    const int fc = min(kFeatChunk, d - f0);
    __syncthreads();
    for (int e = t; e < kAsmTile * kFeatChunk; e += 256) {
      const int rr = e / kFeatChunk, ff = e % kFeatChunk;
      if (ff < fc) {
        xi[rr][ff] = (i0 + rr < n) ? X[(i0 + rr) * ldx + f0 + ff] : 0.0;
        xj[rr][ff] = (j0 + rr < n) ? X[(j0 + rr) * ldx + f0 + ff] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      s[m] = sqdist(s[m], &xi[r][0], &xj[cg + 4 * m][0], fc);
    }
  }
  const int64_t i = i0 + r;
  if (i >= n) return;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int64_t j = j0 + cg + 4 * m;
    if (j >= n) continue;
    if (!full && j > i) continue;
    double v;
    if (i == j)
      v = var + noise;
    else
      v = var * exp(-s[m] / two_l2);
    A[i + j * lda] = v;
  }
}

// Matrix-free residual.  grid: (ceil(n/64), ceil(nrhs/8)); block 256 = 4 waves.
// B == nullptr means B = 0, i.e. R = -(K + noise I) Xs.
// Each lane owns one row i and up to 8 right-hand sides; the four waves split
// the column range and their partial sums are combined in a fixed order, so
// the result is deterministic.  Products are accumulated in double-double
// (TwoProd via fma, TwoSum), so the residual keeps about FP64 relative
// accuracy even for n ~ 1e5 (its rounding would otherwise dominate the
// refinement's error certificate).
constexpr int kResRhs = 8;

__device__ inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ __launch_bounds__(256) void gp_residual_kernel(
    const double *__restrict__ F, int64_t n, int d, int64_t ldf, double two_l2, double var,
    double noise, const double *__restrict__ Xs, int64_t ldxs, const double *__restrict__ B,
    int64_t ldb, double *__restrict__ R, int64_t ldr, int64_t nrhs) {
  constexpr int JCH = 256;  // columns staged per pass
  __shared__ double fj[JCH][kFeatChunk + 1];
  __shared__ double xj[kResRhs][JCH];
  __shared__ double red_s[4][kResRhs][64], red_e[4][kResRhs][64];
  const int t = threadIdx.x, lane = t % 64, w = t / 64;
  const int64_t c0 = (int64_t)blockIdx.y * kResRhs;
  const int nc = (int)min<int64_t>(kResRhs, nrhs - c0);
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  double fi[kFeatChunk];
  const int dd = min(d, kFeatChunk);
#pragma unroll
  for (int k = 0; k < kFeatChunk; ++k) fi[k] = (i < n && k < dd) ? F[i * ldf + k] : 0.0;
  double hs[kResRhs], he[kResRhs];
#pragma unroll
  for (int q = 0; q < kResRhs; ++q) hs[q] = he[q] = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += JCH) {
    __syncthreads();
    for (int e = t; e < JCH * kFeatChunk; e += 256) {
      const int jj = e / kFeatChunk, ff = e % kFeatChunk;
      if (ff < dd) fj[jj][ff] = (j0 + jj < n) ? F[(j0 + jj) * ldf + ff] : 0.0;
    }
    for (int e = t; e < JCH * kResRhs; e += 256) {
      const int q = e / JCH, jj = e % JCH;
      xj[q][jj] = (j0 + jj < n && q < nc) ? Xs[j0 + jj + (c0 + q) * ldxs] : 0.0;
    }
    __syncthreads();
    const int jend = (int)min<int64_t>(JCH, n - j0);
    for (int jj = w; jj < jend; jj += 4) {
      const int64_t j = j0 + jj;
      double k;
      if (j == i) {
        k = var + noise;
      } else {
#pragma clang fp contract(off)
        double s = 0.0;
#pragma unroll
        for (int f = 0; f < kFeatChunk; ++f) {
          if (f < dd) {
            const double q = fi[f] - fj[jj][f];
            s += q * q;
          }
        }
        // features beyond the first 16 are read straight from memory
        for (int f = kFeatChunk; f < d; ++f) {
          const double q = (i < n ? F[i * ldf + f] : 0.0) - F[j * ldf + f];
          s += q * q;
        }
        k = var * exp(-s / two_l2);
      }
#pragma unroll
      for (int q = 0; q < kResRhs; ++q) {
        const double p = k * xj[q][jj];
        const double pe = fma(k, xj[q][jj], -p);
        double s1, e1;
        two_sum(hs[q], p, s1, e1);
        hs[q] = s1;
        he[q] += e1 + pe;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kResRhs; ++q) {
    red_s[w][q][lane] = hs[q];
    red_e[w][q][lane] = he[q];
  }
  __syncthreads();
  if (w == 0 && i < n) {
    for (int q = 0; q < nc; ++q) {
      double s = red_s[0][q][lane], e = red_e[0][q][lane];
      for (int v = 1; v < 4; ++v) {
        double s1, e1;
        two_sum(s, red_s[v][q][lane], s1, e1);
        s = s1;
        e += e1 + red_e[v][q][lane];
      }
      // r = b - (s + e) evaluated as (b - s) - e
      double r1, r2;
      two_sum(B ? B[i + (c0 + q) * ldb] : 0.0, -s, r1, r2);
      R[i + (c0 + q) * ldr] = r1 + (r2 - e);
    }
  }
}

__global__ void clear_i64_kernel(int64_t *p, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0;
}

// Largest diagonal entry of a column-major matrix (one workgroup; NaN-free
// input assumed, non-positive results are left to the caller).
__global__ __launch_bounds__(1024) void max_diag_kernel(const double *__restrict__ A, int64_t lda,
                                                        int64_t n, double *__restrict__ out) {
  __shared__ double sm[1024];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, A[i * (lda + 1)]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

}  // namespace

void launch_gp_assemble(const double *X, int64_t n, int64_t d, int64_t ldx, double two_l2,
                        double var, double noise, double *A, int64_t lda, int full,
                        hipStream_t s) {
  if (n <= 0) return;
  const int64_t nb = (n + kAsmTile - 1) / kAsmTile;
  dim3 grid((unsigned)nb, (unsigned)nb);
  hipLaunchKernelGGL(gp_assemble_kernel, grid, dim3(256), 0, s, X, n, (int)d, ldx, two_l2, var,
                     noise, A, lda, full);
}

void launch_gp_residual(const double *F, int64_t n, int64_t d, int64_t ldf, double two_l2,
                        double var, double noise, const double *Xs, int64_t ldxs,
                        const double *B, int64_t ldb, double *R, int64_t ldr, int64_t nrhs,
                        hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((nrhs + kResRhs - 1) / kResRhs));
  hipLaunchKernelGGL(gp_residual_kernel, grid, dim3(256), 0, s, F, n, (int)d, ldf, two_l2, var,
                     noise, Xs, ldxs, B, ldb, R, ldr, nrhs);
}

void launch_max_diag(const double *A, int64_t lda, int64_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(max_diag_kernel, dim3(1), dim3(1024), 0, s, A, lda, n, out);
}

void launch_clear_i64(int64_t *p, int count, hipStream_t s) {
  hipLaunchKernelGGL(clear_i64_kernel, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
}

}  // namespace chol
