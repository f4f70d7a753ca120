// Conjugate gradients on the packed lower-tile matrix: the paper's CG method
// (Fundamentals section, "The Conjugate Gradient method"; its implementation
// keeps only the diagonal and lower blocks, Implementation section) on one
// GPU.  The only matrix traffic per iteration is one pass over the packed
// lower triangle: every off-diagonal tile serves both products it appears in
// (A_ic s_c for rows of block i and A_ic^T s_i for rows of block c).
//
// Kernels, per iteration (k right-hand sides, each with its own scalars):
//   symv_tiles   one workgroup per stored tile (packed order): both partial
//                products of the tile, written to a partial buffer;
//   symv_reduce  one workgroup per block row: sums the row's partials in a
//                fixed order, then t = A s with s.t partial dots, or the
//                residual r = b - A x (initial step, periodic recomputation)
//                with r.r partial dots;
//   cg_xr        alpha = u / s.t (every workgroup sums the N partial dots in
//                the same order, so all agree bitwise); x += alpha s and,
//                except on recomputation steps, r -= alpha t; r.r partials;
//   cg_s         u' = r.r, beta = u' / u, s = r + beta s; workgroup 0 writes
//                the next step's u, the active flags and iteration counts.
// No atomics: the result is bitwise reproducible.  Scalars and flags are
// double-buffered by step parity so that no kernel overwrites a value
// another workgroup of the same launch still reads.
#include "internal.hpp"

namespace chol {
namespace {

constexpr int kCgThreads = 512;    // symv_tiles: 8 waves per tile
constexpr int kCgWaves = kCgThreads / 64;
constexpr int kRedThreads = 512;   // symv_reduce

// Packed tile index -> (i, c): column c holds ids
// [c N - c(c-1)/2, (c+1) N - c(c+1)/2).
__device__ inline void tile_of(int64_t id, int64_t N, int64_t &i, int64_t &c) {
  const double tn = 2.0 * (double)N + 1.0;
  int64_t cc = (int64_t)((tn - sqrt(tn * tn - 8.0 * (double)id)) * 0.5);
  if (cc < 0) cc = 0;
  if (cc > N - 1) cc = N - 1;
  while (cc > 0 && tile_col_offset(cc, N) > id) --cc;
  while (cc + 1 < N && tile_col_offset(cc + 1, N) <= id) ++cc;
  c = cc;
  i = cc + (id - tile_col_offset(cc, N));
}

// Sum of CW per-lane values over the 64 lanes of a wave, for all CW values at
// once: each halving step (lane mask M) keeps half of the values and adds the
// partner lane's copy of them, so after log2(CW) steps lane l holds one
// value, that of column l / (64 / CW) summed over the lanes sharing its high
// bits; the remaining steps sum over the low bits.
template <int CW, int M, int CNT>
__device__ inline void colsum_step(double (&v)[CW], int lane) {
  if constexpr (M >= 1) {
    if constexpr (CNT > 1) {
      constexpr int H = CNT / 2;
      const bool hi = (lane & M) != 0;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const double send = hi ? v[j] : v[j + H];
        const double keep = hi ? v[j + H] : v[j];
        v[j] = keep + __shfl_xor(send, M, 64);
      }
      colsum_step<CW, M / 2, H>(v, lane);
    } else {
      v[0] += __shfl_xor(v[0], M, 64);
      colsum_step<CW, M / 2, 1>(v, lane);
    }
  }
}

// Partial buffer: part[(id * 2 + side) * K * B + k * B + r], side 0 the
// row-block product A_ic s_c (rows of block i), side 1 the transposed
// product A_ic^T s_i (rows of block c).  A diagonal tile writes the full
// symmetric product of its block (lower part mirrored) to side 0 only.
// The grid covers the leading Nt x Nt tiles (Nt = N: all of them; the
// heterogeneous CG gives the GPU the leading block rows): workgroup w takes
// tile w of the Nt-triangle's packed order, stored at its N-packed id.
template <int B>
__global__ __launch_bounds__(kCgThreads) void symv_tiles_kernel(
    const double *__restrict__ tiles, int64_t N, int64_t Nt, const double *__restrict__ v,
    int64_t ldv, int K, double *__restrict__ part) {
  constexpr int R = B / 64;         // rows per lane
  constexpr int CW = B / kCgWaves;  // columns per wave
  extern __shared__ double sv[];  // [2][K][B]: s_c, then s_i
  __shared__ double red[kCgWaves][B];
  __shared__ double pcol[B];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t i, c;
  tile_of(blockIdx.x, Nt, i, c);
  const int64_t id = tile_index(i, c, N);
  const double *T = tiles + id * (int64_t)B * B;

  // the wave's CW columns, R rows per lane: one contiguous column per wave
  // load; the tiles stream through once per product, so the loads are
  // marked non-temporal (measured 6.9 against 6.5 TB/s for a plain read)
  double a[CW][R];
#pragma unroll
  for (int j = 0; j < CW; ++j) {
    const double *col = T + (int64_t)(w * CW + j) * B + R * lane;
#pragma unroll
    for (int q = 0; q < R; ++q) a[j][q] = __builtin_nontemporal_load(col + q);
  }
  for (int e = threadIdx.x; e < K * B; e += kCgThreads) {
    const int k = e / B, r = e % B;
    sv[k * B + r] = v[(int64_t)k * ldv + c * B + r];
    sv[(K + k) * B + r] = v[(int64_t)k * ldv + i * B + r];
  }
  const bool diag = (i == c);
  if (diag) {
    // the stored upper part of a diagonal tile is zero; halving the diagonal
    // lets the row and column products each count it once in total
#pragma unroll
    for (int j = 0; j < CW; ++j)
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (R * lane + q == w * CW + j) a[j][q] *= 0.5;
  }
  __syncthreads();

  const int64_t stride = (int64_t)K * B;
  double *out_row = part + (id * 2 + 0) * stride;
  double *out_col = part + (id * 2 + 1) * stride;
  const int col_of_lane = lane / (64 / CW);
  const bool col_owner = (lane % (64 / CW)) == 0;
  for (int k = 0; k < K; ++k) {
    double pr[R];
#pragma unroll
    for (int q = 0; q < R; ++q) pr[q] = 0.0;
    double pc[CW];
    double si[R];
#pragma unroll
    for (int q = 0; q < R; ++q) si[q] = sv[(K + k) * B + R * lane + q];
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const double sc = sv[k * B + w * CW + j];
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        pr[q] = fma(a[j][q], sc, pr[q]);
        acc = fma(a[j][q], si[q], acc);
      }
      pc[j] = acc;
    }
    colsum_step<CW, 32, CW>(pc, lane);
    const double colsum = pc[0];
#pragma unroll
    for (int q = 0; q < R; ++q) red[w][R * lane + q] = pr[q];
    if (diag && col_owner) pcol[w * CW + col_of_lane] = colsum;
    __syncthreads();
    if (threadIdx.x < B) {
      const int r = threadIdx.x;
      double y = red[0][r];
#pragma unroll
      for (int q = 1; q < kCgWaves; ++q) y += red[q][r];
      if (diag) y += pcol[r];
      out_row[k * B + r] = y;
    }
    if (!diag && col_owner) out_col[k * B + w * CW + col_of_lane] = colsum;
    __syncthreads();
  }
}

// Deterministic tree sum of one value per thread over a block of NT threads
// (NT a power of two); every thread gets the result.
template <int NT>
__device__ inline double block_sum(double x, double *sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
#pragma unroll
  for (int m = NT / 2; m >= 1; m >>= 1) {
    if (threadIdx.x < m) sh[threadIdx.x] += sh[threadIdx.x + m];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}


// One workgroup per block row i: y = sum over the row's N partials in the
// order c = 0..i (side 0 of tile (i, c)), then q = i+1..Nt-1 (side 1 of tile
// (q, i)); G thread groups take contiguous ranges, combined in group order.
// Nt < N (heterogeneous CG): the products of tiles in rows >= Nt reach these
// rows through `extra` (n_pad x K, ld), added last.
//   CG_RED_T     t_i = y;                         pdot = s_i . t_i
//   CG_RED_RESID r_i = b_i - y (active columns);  pdot = r_i . r_i
//   CG_RED_INIT  r_i = s_i = b_i - y;             pdot = r_i . r_i
template <int B>
__global__ __launch_bounds__(kRedThreads) void symv_reduce_kernel(
    const double *__restrict__ part, int64_t N, int64_t Nt, int K, int mode, double *__restrict__ t,
    double *__restrict__ s, double *__restrict__ r, const double *__restrict__ bv, int64_t ld,
    const int *__restrict__ act, double *__restrict__ pdot, const double *__restrict__ extra) {
  constexpr int G = kRedThreads / B;
  __shared__ double gsum[G][B];
  __shared__ double sh[kRedThreads];
  const int64_t i = blockIdx.x;
  const int row = threadIdx.x % B, g = threadIdx.x / B;
  const int64_t stride = (int64_t)K * B;
  const int64_t per = (Nt + G - 1) / G;
  const int64_t e0 = g * per, e1 = (e0 + per < Nt) ? e0 + per : Nt;
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
#pragma unroll 8
    for (int64_t e = e0; e < e1; ++e) {
      const double *p = (e <= i) ? part + (tile_index(i, e, N) * 2 + 0) * stride
                                 : part + (tile_index(e, i, N) * 2 + 1) * stride;
      acc += p[k * B + row];
    }
    gsum[g][row] = acc;
    __syncthreads();
    double dot = 0.0;
    if (g == 0) {
      double y = gsum[0][row];
#pragma unroll
      for (int q = 1; q < G; ++q) y += gsum[q][row];
      const int64_t o = (int64_t)k * ld + i * B + row;
      if (extra) y += extra[o];
      if (mode == CG_RED_T) {
        t[o] = y;
        dot = s[o] * y;
      } else {
        double rv = r[o];
        if (mode == CG_RED_INIT || act[k]) rv = bv[o] - y;
        r[o] = rv;
        if (mode == CG_RED_INIT) s[o] = rv;
        dot = rv * rv;
      }
    }
    __syncthreads();
    const double tot = block_sum<kRedThreads>(dot, sh);  // other groups add zeros
    if (threadIdx.x == 0) pdot[i * K + k] = tot;
  }
}

// Fixed-order sum of p[e * K + k], e < N, by B threads (strided partial sums,
// then a tree): the same value in every workgroup.
template <int B>
__device__ inline double sum_partials(const double *__restrict__ p, int64_t N, int K, int k,
                                      double *sh) {
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < N; e += B) acc += p[e * K + k];
  return block_sum<B>(acc, sh);
}

// x += alpha s; r -= alpha t (unless this step recomputes r); r.r partials.
template <int B>
__global__ __launch_bounds__(B) void cg_xr_kernel(int64_t N, int K, const double *__restrict__ pdot,
                                                  const double *__restrict__ u_in,
                                                  const int *__restrict__ act, double *__restrict__ x,
                                                  double *__restrict__ r, const double *__restrict__ s,
                                                  const double *__restrict__ t, int64_t ld,
                                                  int recompute_now, double *__restrict__ prr) {
  __shared__ double sh[B];
  const int64_t i = blockIdx.x;
  for (int k = 0; k < K; ++k) {
    const double st = sum_partials<B>(pdot, N, K, k, sh);
    const double alpha = u_in[k] / st;
    const int64_t o = (int64_t)k * ld + i * B + threadIdx.x;
    double rv = r[o];
    if (act[k]) {
      x[o] = fma(alpha, s[o], x[o]);
      if (!recompute_now) {
        rv = fma(-alpha, t[o], rv);
        r[o] = rv;
      }
    }
    if (!recompute_now) {
      const double tot = block_sum<B>(rv * rv, sh);
      if (threadIdx.x == 0) prr[i * K + k] = tot;
    }
  }
}

// u' = r.r; beta = u' / u; s = r + beta s (active columns).  Workgroup 0
// writes the next step's scalars: u_out = u' (or u for finished columns),
// act_out = act && u' > eps^2 u0, iters += act.
template <int B>
__global__ __launch_bounds__(B) void cg_s_kernel(int64_t N, int K, const double *__restrict__ prr,
                                                 const double *__restrict__ u_in,
                                                 const int *__restrict__ act_in,
                                                 double *__restrict__ u_out, int *__restrict__ act_out,
                                                 const double *__restrict__ u0, double eps2,
                                                 int *__restrict__ iters, const double *__restrict__ r,
                                                 double *__restrict__ s, int64_t ld) {
  __shared__ double sh[B];
  const int64_t i = blockIdx.x;
  for (int k = 0; k < K; ++k) {
    const double un = sum_partials<B>(prr, N, K, k, sh);
    const int a = act_in[k];
    if (a) {
      const double beta = un / u_in[k];
      const int64_t o = (int64_t)k * ld + i * B + threadIdx.x;
      s[o] = fma(beta, s[o], r[o]);
    }
    if (i == 0 && threadIdx.x == 0) {
      u_out[k] = a ? un : u_in[k];
      act_out[k] = (a && un > eps2 * u0[k]) ? 1 : 0;
      iters[k] += a;
    }
  }
}

// Initial scalars: u = u0 = r.r, act = u > eps^2 u0, iters = 0 (one workgroup).
template <int B>
__global__ __launch_bounds__(B) void cg_init_kernel(int64_t N, int K, const double *__restrict__ prr,
                                                    double *__restrict__ u, double *__restrict__ u0,
                                                    int *__restrict__ act, int *__restrict__ iters,
                                                    double eps2) {
  __shared__ double sh[B];
  for (int k = 0; k < K; ++k) {
    const double un = sum_partials<B>(prr, N, K, k, sh);
    if (threadIdx.x == 0) {
      u[k] = un;
      u0[k] = un;
      act[k] = un > eps2 * un ? 1 : 0;
      iters[k] = 0;
    }
  }
}

// dst (n_pad x K, ld) <- src (n x K, lds), zero rows n..n_pad-1; or back.
__global__ __launch_bounds__(256) void cg_copy_in_kernel(const double *__restrict__ src,
                                                         int64_t lds, int64_t n, int64_t n_pad,
                                                         int K, double *__restrict__ dst, int64_t ld) {
  const int64_t tot = n_pad * K;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t k = e / n_pad, row = e % n_pad;
    dst[k * ld + row] = row < n ? src[k * lds + row] : 0.0;
  }
}
__global__ __launch_bounds__(256) void cg_copy_out_kernel(const double *__restrict__ src, int64_t ld,
                                                          int64_t n, int K, double *__restrict__ dst,
                                                          int64_t ldd) {
  const int64_t tot = n * K;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t k = e / n, row = e % n;
    dst[k * ldd + row] = src[k * ld + row];
  }
}

unsigned copy_grid(int64_t tot) {
  int64_t g = (tot + 255) / 256;
  if (g > 8192) g = 8192;
  return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

void launch_cg_symv(const double *tiles, int b, int64_t N, const double *v, int64_t ldv, int K,
                    double *part, hipStream_t s, int64_t Nt) {
  if (Nt < 0 || Nt > N) Nt = N;
  const unsigned grid = (unsigned)tile_count(Nt);
  if (grid == 0) return;
  if (b == 128)
    hipLaunchKernelGGL(symv_tiles_kernel<128>, dim3(grid), dim3(kCgThreads), 2 * K * 128 * 8, s, tiles, N, Nt,
                       v, ldv, K, part);
  else
    hipLaunchKernelGGL(symv_tiles_kernel<64>, dim3(grid), dim3(kCgThreads), 2 * K * 64 * 8, s, tiles, N, Nt,
                       v, ldv, K, part);
}

void launch_cg_reduce(const double *part, int b, int64_t N, int K, int mode, double *t, double *sv,
                      double *r, const double *bv, int64_t ld, const int *act, double *pdot,
                      hipStream_t s, int64_t Nt, const double *extra) {
  if (Nt < 0 || Nt > N) Nt = N;
  if (Nt == 0) return;
  if (b == 128)
    hipLaunchKernelGGL(symv_reduce_kernel<128>, dim3((unsigned)Nt), dim3(kRedThreads), 0, s, part, N,
                       Nt, K, mode, t, sv, r, bv, ld, act, pdot, extra);
  else
    hipLaunchKernelGGL(symv_reduce_kernel<64>, dim3((unsigned)Nt), dim3(kRedThreads), 0, s, part, N,
                       Nt, K, mode, t, sv, r, bv, ld, act, pdot, extra);
}

void launch_cg_xr(int b, int64_t N, int K, const double *pdot, const double *u_in, const int *act,
                  double *x, double *r, const double *sv, const double *t, int64_t ld,
                  int recompute_now, double *prr, hipStream_t s, int64_t rows) {
  if (rows < 0 || rows > N) rows = N;
  if (rows == 0) return;
  if (b == 128)
    hipLaunchKernelGGL(cg_xr_kernel<128>, dim3((unsigned)rows), dim3(128), 0, s, N, K, pdot, u_in, act,
                       x, r, sv, t, ld, recompute_now, prr);
  else
    hipLaunchKernelGGL(cg_xr_kernel<64>, dim3((unsigned)rows), dim3(64), 0, s, N, K, pdot, u_in, act, x,
                       r, sv, t, ld, recompute_now, prr);
}

void launch_cg_s(int b, int64_t N, int K, const double *prr, const double *u_in, const int *act_in,
                 double *u_out, int *act_out, const double *u0, double eps2, int *iters,
                 const double *r, double *sv, int64_t ld, hipStream_t s, int64_t rows) {
  if (rows < 0 || rows > N) rows = N;
  if (rows == 0) return;
  if (b == 128)
    hipLaunchKernelGGL(cg_s_kernel<128>, dim3((unsigned)rows), dim3(128), 0, s, N, K, prr, u_in, act_in,
                       u_out, act_out, u0, eps2, iters, r, sv, ld);
  else
    hipLaunchKernelGGL(cg_s_kernel<64>, dim3((unsigned)rows), dim3(64), 0, s, N, K, prr, u_in, act_in,
                       u_out, act_out, u0, eps2, iters, r, sv, ld);
}

void launch_cg_init(int b, int64_t N, int K, const double *prr, double *u, double *u0, int *act,
                    int *iters, double eps2, hipStream_t s) {
  if (b == 128)
    hipLaunchKernelGGL(cg_init_kernel<128>, dim3(1), dim3(128), 0, s, N, K, prr, u, u0, act, iters,
                       eps2);
  else
    hipLaunchKernelGGL(cg_init_kernel<64>, dim3(1), dim3(64), 0, s, N, K, prr, u, u0, act, iters,
                       eps2);
}

void launch_cg_copy_in(const double *src, int64_t lds, int64_t n, int64_t n_pad, int K, double *dst,
                       int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(cg_copy_in_kernel, dim3(copy_grid(n_pad * K)), dim3(256), 0, s, src, lds, n,
                     n_pad, K, dst, ld);
}

void launch_cg_copy_out(const double *src, int64_t ld, int64_t n, int K, double *dst, int64_t ldd,
                        hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cg_copy_out_kernel, dim3(copy_grid(n * K)), dim3(256), 0, s, src, ld, n, K, dst,
                     ldd);
}

}  // namespace chol
