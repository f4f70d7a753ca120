// FP64 vector kernels of the refinement loop: the residual R = B - A X for a
// symmetric A given by its lower triangle (the refinement counterpart of the
// paper's CG residual b - A x, first algorithm figure, left column), column
// dot products, and axpby updates.  All are HBM-bound and deterministic
// (fixed work assignment and reduction order, no atomics).
#include "internal.hpp"

namespace chol {
namespace {

__device__ inline void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Residual.  grid (ceil(n/64), ceil(nrhs/NR)); block 256.  Bm == nullptr
// means B = 0, i.e. R = -A X (the product used by the CG iteration).  A workgroup owns
// 64 rows and walks every 64-column block of the symmetric matrix: blocks
// left of the diagonal come from the lower triangle as stored, blocks right
// of it from the lower triangle transposed (both read along columns, so the
// HBM reads are contiguous).  Blocks are staged through two LDS buffers: the
// next block is loaded into registers while the current one is used, one
// barrier per block.  Lane o of the four waves accumulates row o over a
// quarter of the block's columns in double-double (TwoProd by fma, TwoSum),
// with two independent accumulators per right-hand side for instruction-level
// parallelism, so the residual's own rounding is far below FP64 round-off of
// |A||x| even at n ~ 1e5.  Every reduction has a fixed order.  Contraction is
// off in the kernel: a product fused into the following TwoSum (hs + av * xv
// as one fma) would make the error terms count the product's rounding twice.
// DD = false: the same walk with plain FP64 accumulation (one fma per product,
// error within the usual recursive-summation bound n u |A||x|), for the
// refinement's working residuals and CG products; HBM-bound where the
// double-double form is bound by FP64 arithmetic (several right-hand sides).
template <int NR, bool DD>
__global__ __launch_bounds__(256) void symm_residual_kernel(
    const double *__restrict__ A, int64_t lda, int64_t n, const double *__restrict__ X,
    int64_t ldx, const double *__restrict__ Bm, int64_t ldb, double *__restrict__ R, int64_t ldr,
    int64_t nrhs) {
#pragma clang fp contract(off)
  constexpr int P = 65;
  constexpr int NA = 2;  // accumulators per right-hand side
  __shared__ double at[2][64 * P];  // at[.][jj * P + ii] = A(I0 + ii, J0 + jj)
  __shared__ double xs[2][64 * NR];  // xs[.][jj * NR + cc]
  const int tid = threadIdx.x, o = tid & 63, h = tid >> 6;
  const int64_t I0 = (int64_t)blockIdx.x * 64;
  const int64_t c0 = (int64_t)blockIdx.y * NR;
  const int nc = (int)min<int64_t>(NR, nrhs - c0);
  const int64_t nb = (n + 63) / 64;
  // block Jb into registers (16 values of A, up to NR/4 + 1 values of X)
  constexpr int XV = (64 * NR + 255) / 256;
  double ra[16], rx[XV];
  auto fetch = [&](int64_t Jb) {
    const int64_t J0 = Jb * 64;
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      const int e = tid + 256 * x, a = e & 63, bc = e >> 6;
      double v = 0.0;
      if (J0 < I0) {
        const int64_t gi = I0 + a, gj = J0 + bc;
        if (gi < n && gj < n) v = A[gi + gj * lda];
      } else if (J0 > I0) {
        const int64_t gi = I0 + bc, gj = J0 + a;
        if (gi < n && gj < n) v = A[gj + gi * lda];
      } else if (a >= bc) {
        const int64_t gi = I0 + a, gj = I0 + bc;
        if (gi < n && gj < n) v = A[gi + gj * lda];
      }
      ra[x] = v;
    }
#pragma unroll
    for (int x = 0; x < XV; ++x) {
      const int e = tid + 256 * x, jj = e % 64, cc = e / 64;
      const int64_t gj = J0 + jj;
      rx[x] = (e < 64 * NR && gj < n && cc < nc) ? X[gj + (c0 + cc) * ldx] : 0.0;
    }
  };
  auto stash = [&](int64_t Jb, int buf) {
    const int64_t J0 = Jb * 64;
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      const int e = tid + 256 * x, a = e & 63, bc = e >> 6;
      if (J0 < I0) {
        at[buf][bc * P + a] = ra[x];
      } else if (J0 > I0) {
        at[buf][a * P + bc] = ra[x];
      } else if (a >= bc) {
        at[buf][bc * P + a] = ra[x];
        at[buf][a * P + bc] = ra[x];
      }
    }
#pragma unroll
    for (int x = 0; x < XV; ++x) {
      const int e = tid + 256 * x, jj = e % 64, cc = e / 64;
      if (e < 64 * NR) xs[buf][jj * NR + cc] = rx[x];
    }
  };
  double hs[NA][NR], he[NA][NR];
#pragma unroll
  for (int u = 0; u < NA; ++u)
#pragma unroll
    for (int cc = 0; cc < NR; ++cc) hs[u][cc] = he[u][cc] = 0.0;
  fetch(0);
  stash(0, 0);
  __syncthreads();
  for (int64_t Jb = 0; Jb < nb; ++Jb) {
    const int buf = (int)(Jb & 1);
    if (Jb + 1 < nb) fetch(Jb + 1);
    const double *ab = at[buf];
    const double *xb = xs[buf];
    // not unrolled: unrolling hoists every LDS read of the block into
    // registers (500 per lane, one wave per SIMD)
#pragma unroll 1
    for (int j2 = 0; j2 < 16; j2 += NA) {
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        const int jj = h * 16 + j2 + u;
        const double av = ab[jj * P + o];
#pragma unroll
        for (int cc = 0; cc < NR; ++cc) {
          const double xv = xb[jj * NR + cc];
          if (DD) {
            const double p = av * xv;
            const double pe = fma(av, xv, -p);
            double s1, e1;
            two_sum(hs[u][cc], p, s1, e1);
            hs[u][cc] = s1;
            he[u][cc] += e1 + pe;
          } else {
            hs[u][cc] = fma(av, xv, hs[u][cc]);
          }
        }
      }
    }
    // the other buffer was last read in the previous block, before the barrier
    if (Jb + 1 < nb) stash(Jb + 1, buf ^ 1);
    __syncthreads();
  }
  // fold the accumulators (fixed order), then the four quarters through LDS
  double *red_s = at[0], *red_e = at[1];  // 4 * 64 * NR <= 64 * P doubles for NR <= 16
#pragma unroll
  for (int cc = 0; cc < NR; ++cc) {
    double s = hs[0][cc], e = he[0][cc];
#pragma unroll
    for (int u = 1; u < NA; ++u) {
      double s1, e1;
      two_sum(s, hs[u][cc], s1, e1);
      s = s1;
      e += e1 + he[u][cc];
    }
    red_s[(h * 64 + o) * NR + cc] = s;
    red_e[(h * 64 + o) * NR + cc] = e;
  }
  __syncthreads();
  if (h == 0) {
    const int64_t row = I0 + o;
    if (row < n) {
      for (int cc = 0; cc < nc; ++cc) {
        double s = red_s[o * NR + cc], e = red_e[o * NR + cc];
        for (int q = 1; q < 4; ++q) {
          double s1, e1;
          two_sum(s, red_s[(q * 64 + o) * NR + cc], s1, e1);
          s = s1;
          e += e1 + red_e[(q * 64 + o) * NR + cc];
        }
        double r1, r2;
        two_sum(Bm ? Bm[row + (c0 + cc) * ldb] : 0.0, -s, r1, r2);
        R[row + (c0 + cc) * ldr] = r1 + (r2 - e);
      }
    }
  }
}

// Column dot products, two passes.  Pass 1: grid (nblk, nrhs), each block
// reduces a fixed strided set of rows.  Pass 2: one block per column sums
// the nblk partials in index order.
constexpr int kDotBlocks = 128;

__global__ __launch_bounds__(256) void col_dot_partial(const double *__restrict__ x, int64_t ldx,
                                                       const double *__restrict__ y, int64_t ldy,
                                                       int64_t n, double *__restrict__ partial) {
  __shared__ double sm[256];
  const int64_t c = blockIdx.y;
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + tid; r < n; r += (int64_t)kDotBlocks * 256)
    s += x[r + c * ldx] * y[r + c * ldy];
  sm[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sm[tid] += sm[tid + w];
    __syncthreads();
  }
  if (tid == 0) partial[c * kDotBlocks + blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(128) void col_dot_final(const double *__restrict__ partial,
                                                     double *__restrict__ out) {
  __shared__ double sm[kDotBlocks];
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  sm[tid] = partial[c * kDotBlocks + tid];
  __syncthreads();
  for (int w = kDotBlocks / 2; w > 0; w >>= 1) {
    if (tid < w) sm[tid] += sm[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[c] = sm[0];
}

// y = sgn * a[c] * x + bcoef[c] * y on active columns.
__global__ void axpby_kernel(const double *__restrict__ x, int64_t ldx, double *__restrict__ y,
                             int64_t ldy, int64_t n, int64_t nrhs, const double *__restrict__ a,
                             double sgn, const double *__restrict__ bcoef,
                             const int32_t *__restrict__ active) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t r = e % n, c = e / n;
  if (active && !active[c]) return;
  const double av = sgn * (a ? a[c] : 1.0);
  const double bv = bcoef ? bcoef[c] : 1.0;
  y[r + c * ldy] = av * x[r + c * ldx] + bv * y[r + c * ldy];
}

__global__ void copy_kernel(const double *__restrict__ x, int64_t ldx, double *__restrict__ y,
                            int64_t ldy, int64_t n, int64_t nrhs,
                            const int32_t *__restrict__ mask) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t r = e % n, c = e / n;
  if (mask && !mask[c]) return;
  y[r + c * ldy] = x[r + c * ldx];
}

// CG scalars, one thread per right-hand side (the preconditioned CG step:
// alpha = rho / p.A p, beta = rho_new / rho).  pq holds p.q with q = -A p.
// A zero or non-finite denominator gives a zero step instead of NaN.
__global__ void pcg_alpha_kernel(const double *__restrict__ rho, const double *__restrict__ pq,
                                 const int32_t *__restrict__ act, double *__restrict__ alpha,
                                 int64_t nrhs) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double den = -pq[c];
  alpha[c] = (act[c] && den != 0.0 && isfinite(den)) ? rho[c] / den : 0.0;
}

__global__ void pcg_beta_kernel(const double *__restrict__ rho_new, double *__restrict__ rho,
                                const int32_t *__restrict__ act, double *__restrict__ beta,
                                int64_t nrhs) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  if (!act[c]) {
    beta[c] = 0.0;
    return;
  }
  beta[c] = rho[c] != 0.0 ? rho_new[c] / rho[c] : 0.0;
  rho[c] = rho_new[c];
}

}  // namespace

void launch_symm_residual(const double *A, int64_t lda, int64_t n, const double *X, int64_t ldx,
                          const double *B, int64_t ldb, double *R, int64_t ldr, int64_t nrhs,
                          hipStream_t s, bool exact) {
  if (n <= 0 || nrhs <= 0) return;
  const unsigned gx = (unsigned)((n + 63) / 64);
  const dim3 g1(gx, 1), g8(gx, (unsigned)((nrhs + 7) / 8));
  if (nrhs == 1 && exact)
    hipLaunchKernelGGL((symm_residual_kernel<1, true>), g1, dim3(256), 0, s, A, lda, n, X, ldx,
                       B, ldb, R, ldr, nrhs);
  else if (nrhs == 1)
    hipLaunchKernelGGL((symm_residual_kernel<1, false>), g1, dim3(256), 0, s, A, lda, n, X, ldx,
                       B, ldb, R, ldr, nrhs);
  else if (exact)
    hipLaunchKernelGGL((symm_residual_kernel<8, true>), g8, dim3(256), 0, s, A, lda, n, X, ldx,
                       B, ldb, R, ldr, nrhs);
  else
    hipLaunchKernelGGL((symm_residual_kernel<8, false>), g8, dim3(256), 0, s, A, lda, n, X, ldx,
                       B, ldb, R, ldr, nrhs);
}

void launch_col_dot(const double *x, int64_t ldx, const double *y, int64_t ldy, int64_t n,
                    int64_t nrhs, double *out, double *partial, hipStream_t s) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(col_dot_partial, dim3(kDotBlocks, (unsigned)nrhs), dim3(256), 0, s, x, ldx,
                     y, ldy, n, partial);
  hipLaunchKernelGGL(col_dot_final, dim3((unsigned)nrhs), dim3(kDotBlocks), 0, s, partial, out);
}

void launch_axpby(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t n, int64_t nrhs,
                  const double *a, double a_sign, const double *bcoef, const int32_t *active,
                  hipStream_t s) {
  const int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, ldx,
                     y, ldy, n, nrhs, a, a_sign, bcoef, active);
}

void launch_copy(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t n, int64_t nrhs,
                 hipStream_t s) {
  launch_copy_masked(x, ldx, y, ldy, n, nrhs, nullptr, s);
}

void launch_copy_masked(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t n,
                        int64_t nrhs, const int32_t *mask, hipStream_t s) {
  const int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, ldx, y,
                     ldy, n, nrhs, mask);
}

void launch_pcg_alpha(const double *rho, const double *pq, const int32_t *act, double *alpha,
                      int64_t nrhs, hipStream_t s) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(pcg_alpha_kernel, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, s, rho, pq,
                     act, alpha, nrhs);
}

void launch_pcg_beta(const double *rho_new, double *rho, const int32_t *act, double *beta,
                     int64_t nrhs, hipStream_t s) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(pcg_beta_kernel, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, s, rho_new,
                     rho, act, beta, nrhs);
}

}  // namespace chol
