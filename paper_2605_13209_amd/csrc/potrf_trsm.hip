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
// One workgroup of 256 threads factors a B x B diagonal tile (B = 16 M) held
// in registers as FP64.  Threads form a 16 x 16 grid; thread (tr, tc) owns
// the elements (tr + 16 m, tc + 16 n), m, n < M (a cyclic distribution, so the
// shrinking trailing triangle stays spread over all threads).  Right-looking,
// one column k per step:
//   (1) the owner of (k, k) publishes the pivot;            barrier
//   (2) everyone checks it (uniform exit on failure); the owners of column k
//       scale it by 1/sqrt(pivot) and publish it;          barrier
//   (3) every thread applies the rank-1 update to its trailing elements.
// Register indices are compile-time: the column loop is split into an
// unrolled block index km and a runtime offset kr (k = 16 km + kr), and the
// blocks that are inactive at block km are skipped at compile time.  The tile
// is moved between HBM and registers through LDS, half a tile at a time (so
// the kernel's LDS fits next to a trailing-update workgroup on one CU), with
// contiguous global accesses.
template <int B, typename T>
__global__ __launch_bounds__(256) void potrf_kernel(T *__restrict__ tiles, int64_t N, int64_t c,
                                                    int64_t *__restrict__ info) {
  if (*info != 0) return;
  constexpr int M = B / 16;
  constexpr int LD = B + 1;
  constexpr int HC = B / 2;  // columns staged per half
  __shared__ double stage[HC * LD];
  __shared__ double col[B];
  __shared__ double piv;
  T *tile = tiles + tile_index(c, c, N) * (int64_t)(B * B);
  const int t = threadIdx.x, tc = t & 15, tr = t >> 4;
  double a[M][M];
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    for (int e = t; e < HC * B; e += 256) {
      const int r = e % B, cc = e / B;
      stage[cc * LD + r] = (double)tile[(hf * HC + cc) * B + r];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int n = hf * M / 2; n < (hf + 1) * M / 2; ++n)
        a[m][n] = stage[(tc + 16 * n - hf * HC) * LD + tr + 16 * m];
    __syncthreads();
  }

#pragma unroll
  for (int km = 0; km < M; ++km) {
    for (int kr = 0; kr < 16; ++kr) {
      const int k = 16 * km + kr;
      if (tr == kr && tc == kr) piv = a[km][km];
      __syncthreads();
      const double d = piv;
      if (!(d > 0.0)) {  // uniform: every thread read the same pivot
        if (t == 0) *info = c * B + k + 1;
        return;
      }
      const double lkk = sqrt(d);
      const double rl = 1.0 / lkk;  // the column is scaled by the reciprocal
      if (tc == kr) {
#pragma unroll
        for (int m = km; m < M; ++m) {
          const int i = tr + 16 * m;
          if (i > k) {
            a[m][km] = a[m][km] * rl;
            col[i] = a[m][km];
          } else if (i == k) {
            a[m][km] = lkk;
          }
        }
      }
      __syncthreads();
      double ci[M], cj[M];
#pragma unroll
      for (int m = km; m < M; ++m) {
        ci[m] = col[tr + 16 * m];
        cj[m] = col[tc + 16 * m];
      }
#pragma unroll
      for (int m = km; m < M; ++m) {
#pragma unroll
        for (int n = km; n <= m; ++n) {
          const int i = tr + 16 * m, j = tc + 16 * n;
          if (j > k && i >= j) a[m][n] -= ci[m] * cj[n];
        }
      }
    }
  }
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int n = hf * M / 2; n < (hf + 1) * M / 2; ++n) {
        const int i = tr + 16 * m, j = tc + 16 * n;
        stage[(j - hf * HC) * LD + i] = (i >= j) ? a[m][n] : 0.0;
      }
    __syncthreads();
    for (int e = t; e < HC * B; e += 256) {
      const int r = e % B, cc = e / B;
      tile[(hf * HC + cc) * B + r] = (T)stage[cc * LD + r];
    }
  }
}

// ---------------------------------------------------------------- Step 2 --
// X L^T = A for every tile (i, c), i in [c+1, N): each row of X is an
// independent forward substitution with L = L_cc.  One workgroup of 256
// threads per tile; thread (r, h) handles row r (r = t mod B) and owns the
// column blocks q (16 columns each) with q mod H = h (H = 256 / B), keeping
// its solved values in registers.  For block q:
//   the 16-row strip of L needed (rows 16q.., columns < 16q + 16) sits in
//   LDS and is read as broadcasts; the strip of block q+1 is loaded into
//   registers while block q computes (double-buffered strips);
//   every thread sums x_m L[16q+u][m] over its own earlier blocks;
//   the owner of block q adds the H partial sums (in a fixed order) to the
//   right-hand side and solves the 16 x 16 triangle by substitution,
//   multiplying by reciprocals of the diagonal.
// IDENT: the right-hand side is the identity (X is only written), which gives
// X = L^{-T}: used for the inverted diagonal blocks of the solves.
template <int B, typename T, bool IDENT>
__device__ __forceinline__ void trsm_tile(const T *__restrict__ L, T *__restrict__ X) {
  constexpr int CB = 16, NB = B / CB, H = 256 / B;
  __shared__ double ls[2][B * CB];         // ls[.][m * CB + u] = L[16q + u][m]
  __shared__ double part[H][CB][B + 1];    // partial sums per (h, u, row)
  const int t = threadIdx.x, r = t % B, h = t / B;
  // strip q: elements e < (q + 1) * CB * CB, e = m * CB + u -> L[m * B + 16q + u]
  for (int e = t; e < CB * CB; e += 256) ls[0][e] = (double)L[(e / CB) * B + (e % CB)];
  __syncthreads();
  double x[NB / H][CB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const double *lq = ls[q & 1];
    // prefetch the next strip into registers
    constexpr int MAXP = (NB + 1) * CB * CB / 256 + 1;
    double nxt[MAXP];
    if (q + 1 < NB) {
#pragma unroll
      for (int x2 = 0; x2 < MAXP; ++x2) {
        const int e = t + 256 * x2;
        if (e < (q + 2) * CB * CB) nxt[x2] = (double)L[(e / CB) * B + (q + 1) * CB + (e % CB)];
      }
    }
    double acc[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) acc[u] = 0.0;
#pragma unroll
    for (int qq = 0; qq < q; ++qq) {
      if (qq % H == h) {
#pragma unroll
        for (int mm = 0; mm < CB; ++mm) {
          const double xm = x[qq / H][mm];
#pragma unroll
          for (int u = 0; u < CB; ++u) acc[u] += xm * lq[(qq * CB + mm) * CB + u];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) part[h][u][r] = acc[u];
    __syncthreads();
    if (h == q % H) {
      double v[CB], rd[CB];
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        rd[u] = 1.0 / lq[(q * CB + u) * CB + u];
        double s = part[0][u][r];
#pragma unroll
        for (int hh = 1; hh < H; ++hh) s += part[hh][u][r];
        const double rhs = IDENT ? (q * CB + u == r ? 1.0 : 0.0) : (double)X[(q * CB + u) * B + r];
        v[u] = rhs - s;
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
#pragma unroll
        for (int w = 0; w < u; ++w) v[u] -= v[w] * lq[(q * CB + w) * CB + u];
        v[u] = v[u] * rd[u];
        x[q / H][u] = v[u];
        X[(q * CB + u) * B + r] = (T)v[u];
      }
    }
    if (q + 1 < NB) {
#pragma unroll
      for (int x2 = 0; x2 < MAXP; ++x2) {
        const int e = t + 256 * x2;
        if (e < (q + 2) * CB * CB) ls[(q + 1) & 1][e] = nxt[x2];
      }
    }
    __syncthreads();
  }
}

template <int B, typename T>
__global__ __launch_bounds__(256) void trsm_kernel(T *__restrict__ tiles, int64_t N, int64_t c,
                                                   const int64_t *__restrict__ info) {
  if (*info != 0) return;
  const int64_t i = c + 1 + blockIdx.x;
  trsm_tile<B, T, false>(tiles + tile_index(c, c, N) * (int64_t)(B * B),
                         tiles + tile_index(i, c, N) * (int64_t)(B * B));
}

// Inverted diagonal blocks for the solves: block c of dinv = L_cc^{-T}
// (column-major), one workgroup per diagonal tile.
template <int B, typename T>
__global__ __launch_bounds__(256) void diag_inverse_kernel(const T *__restrict__ tiles, int64_t N,
                                                           T *__restrict__ dinv,
                                                           const int64_t *__restrict__ info) {
  if (*info != 0) return;
  const int64_t c = blockIdx.x;
  trsm_tile<B, T, true>(tiles + tile_index(c, c, N) * (int64_t)(B * B),
                        dinv + c * (int64_t)(B * B));
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
    hipLaunchKernelGGL((trsm_kernel<B, double>), dim3((unsigned)nt), dim3(256), 0, s,
                       (double *)tiles, N, c, info);
  else
    hipLaunchKernelGGL((trsm_kernel<B, float>), dim3((unsigned)nt), dim3(256), 0, s,
                       (float *)tiles, N, c, info);
}

}  // namespace

void launch_potrf(void *tiles, int store, int b, int64_t N, int64_t c, int64_t *info,
                  hipStream_t s) {
  if (b == 128)
    potrf_dispatch<128>(tiles, store, N, c, info, s);
  else
    potrf_dispatch<64>(tiles, store, N, c, info, s);
}

void launch_diag_inverse(const void *tiles, int store, int b, int64_t N, void *dinv,
                         const int64_t *info, hipStream_t s) {
  if (N <= 0) return;
  const dim3 grid((unsigned)N);
  if (b == 128) {
    if (store == STORE_F64)
      hipLaunchKernelGGL((diag_inverse_kernel<128, double>), grid, dim3(256), 0, s,
                         (const double *)tiles, N, (double *)dinv, info);
    else
      hipLaunchKernelGGL((diag_inverse_kernel<128, float>), grid, dim3(256), 0, s,
                         (const float *)tiles, N, (float *)dinv, info);
  } else {
    if (store == STORE_F64)
      hipLaunchKernelGGL((diag_inverse_kernel<64, double>), grid, dim3(256), 0, s,
                         (const double *)tiles, N, (double *)dinv, info);
    else
      hipLaunchKernelGGL((diag_inverse_kernel<64, float>), grid, dim3(256), 0, s,
                         (const float *)tiles, N, (float *)dinv, info);
  }
}

void launch_trsm(void *tiles, int store, int b, int64_t N, int64_t c, const int64_t *info,
                 hipStream_t s) {
  if (b == 128)
    trsm_dispatch<128>(tiles, store, N, c, info, s);
  else
    trsm_dispatch<64>(tiles, store, N, c, info, s);
}

}  // namespace chol
