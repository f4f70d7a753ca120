// Forward and back substitution with the packed factor (the paper's solve
// step after the factorisation, Fundamentals, "The Cholesky decomposition"):
//   L Y = B  (forward),   L^T X = Y  (back),   in place on B (n x nrhs).
// Arithmetic is FP64; FP32 factor tiles are widened on load.
//
// Blocked substitution in ONE launch per direction.  Workgroup w owns block
// row i (forward: i = w; back: i = N-1-w) of up to KR right-hand sides:
//   forward : r_i = b_i - sum_{p<i} L_ip y_p,   y_i = L_ii^{-1} r_i
//   back    : r_i = y_i - sum_{p>i} L_pi^T x_p, x_i = L_ii^{-T} r_i
// with the inverted diagonal blocks D_i = L_ii^{-T} computed once after the
// factorisation (so the only sequential work per block row is two small
// matrix-vector products).  Block rows are finished strictly in order, so
// a single counter per right-hand-side chunk says how many are published.
// Publication without cache-wide maintenance: the solution blocks are
// written and read only with device-scope (agent) atomic stores and loads,
// which on gfx950 go to the coherence point (sc1) instead of resting in one
// XCD's L2.  The producer waits until its stores are acknowledged
// (s_waitcnt vmcnt(0), every thread, then a barrier) before it stores the
// counter; a consumer reads the published blocks only after its poll has
// returned the counter.  This is the ordering a release store and an
// acquire load would give, minus the L2 write-back (buffer_wbl2) and
// invalidate (buffer_inv) those add for plain accesses, which cost a large
// part of every link of the chain (n = 32768, one right-hand side: 4.34 ->
// 3.02 ms per solve, bitwise the same result).  Workgroups only wait on
// lower-numbered ones, which the hardware dispatches first, so the chain
// always progresses; as a safety net
// the wait is bounded: after spin_max polls the waiter raises the abort word,
// every other waiter then stops waiting, and the aborted block rows are
// written as NaN (never a hang, never a silently wrong number).  The same
// NaN output is written when the factorisation's info word is non-zero (a
// failed factor whose failure the host has not read yet): the chain still
// runs, so every workgroup publishes and exits as usual.
//
// Each tile a workgroup applies is loaded straight into registers before the
// wait (its memory latency hides behind the wait), 512 threads.  With 16
// right-hand sides (tile 128) both products run on the FP64 matrix cores
// (see the use_mfma branch); otherwise on the vector ALUs:
//   "N" product  out = M v    : thread (r = t mod B, g = t / B) holds
//                               M(r, g*CPG .. g*CPG+CPG-1) (coalesced),
//                               partial sums reduced over g through LDS;
//   "T" product  out = M^T v  : thread (r = t / G, g = t mod G) holds
//                               M(g*CPG .., r) (one contiguous run),
//                               partial sums reduced over the G adjacent
//                               lanes with shuffles.
// forward: off-diagonal tiles N, diagonal D_i^T = T;  back: off-diagonal T,
// diagonal D_i = N.  Padding rows (>= n) read as zero and are never written,
// which is exact because the padded factor is diag(L, I).
#include "internal.hpp"

namespace chol {
namespace {

constexpr int NT = 512;  // threads per workgroup

typedef double v4d __attribute__((ext_vector_type(4)));

// 16 right-hand sides with tile 128 run on the FP64 matrix cores.
template <int B, int KR> constexpr bool use_mfma() { return B == 128 && KR == 16; }

template <int B, int KR> struct SolveSmem {
  static constexpr int G = use_mfma<B, KR>() ? 1 : NT / B;
  static constexpr int R = use_mfma<B, KR>() ? 1 : B * KR;
  double v[B * KR];    // v[c * KR + j]: the vector block being applied
  double own[B * KR];  // this block row's right-hand side, same layout
  double red[G][R];    // partial sums of N products (VALU path)
};

// Wait until *cnt >= need.  Thread 0 polls with relaxed agent-scope loads
// (coherent, without the L2 invalidation an acquire implies, which would
// also disturb the tile streams of every workgroup on the XCD); once the
// value is reached, the barrier orders every thread's later (device-scope
// atomic) reads of the published blocks after it.  `seen` caches the last
// value thread 0 read, so blocks already known to be published cost no
// memory access.
// Returns false when the wait was abandoned (abort raised here or elsewhere).
__device__ bool wait_count(int *cnt, int *abort_word, int need, int spin_max, int &seen,
                           int *ok_sh) {
  if (threadIdx.x == 0) {
    int good = 1;
    if (seen < need) {
      int it = 0;
      for (;;) {
        seen = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (seen >= need) break;
        if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            ++it > spin_max) {
          __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    *ok_sh = good;
  }
  __syncthreads();
  return *ok_sh != 0;
}

template <int B, int KR, bool FWD, typename T>
__global__ __launch_bounds__(NT) void solve_kernel(const T *__restrict__ tiles,
                                                   const T *__restrict__ dinv, int64_t N,
                                                   int64_t n, double *__restrict__ X, int64_t ldx,
                                                   int64_t nrhs, int *__restrict__ counters,
                                                   int *__restrict__ abort_word, int spin_max,
                                                   const int64_t *__restrict__ info) {
  constexpr int G = NT / B, CPG = B / G;
  __shared__ SolveSmem<B, KR> sm;
  __shared__ int ok_sh;
  const int t = threadIdx.x;
  const int ra = t % B, ga = t / B;  // N-product mapping
  const int rb = t / G, gb = t % G;  // T-product mapping
  const int64_t w = blockIdx.x;
  const int64_t i = FWD ? w : N - 1 - w;
  const int64_t j0 = (int64_t)blockIdx.y * KR;
  int *cnt = counters + blockIdx.y;
  const int64_t BB = (int64_t)B * B;

  auto load_n = [&](const T *M, double (&m)[CPG]) {
#pragma unroll
    for (int q = 0; q < CPG; ++q) m[q] = (double)M[(ga * CPG + q) * B + ra];
  };
  auto load_t = [&](const T *M, double (&m)[CPG]) {
    const T *src = M + rb * B + gb * CPG;
    constexpr int VE = 16 / sizeof(T);
#pragma unroll
    for (int q = 0; q < CPG; q += VE) {
      T v[VE];
      *(uint4 *)&v[0] = *(const uint4 *)(src + q);
#pragma unroll
      for (int e = 0; e < VE; ++e) m[q + e] = (double)v[e];
    }
  };
  // block p of the solution (rows p*B + c) into sm.v, zero outside the matrix
  auto load_v = [&](int64_t p) {
    for (int e = t; e < B * KR; e += NT) {
      const int c = e % B, j = e / B;
      const int64_t row = p * B + c, col = j0 + j;
      sm.v[c * KR + j] = (row < n && col < nrhs)
                             ? __hip_atomic_load(&X[col * ldx + row], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : 0.0;
    }
  };
  auto prod_n = [&](const double (&m)[CPG], double (&acc)[KR]) {
#pragma unroll
    for (int q = 0; q < CPG; ++q)
#pragma unroll
      for (int j = 0; j < KR; ++j) acc[j] += m[q] * sm.v[(ga * CPG + q) * KR + j];
  };
  auto prod_t = [&](const double (&m)[CPG], double (&acc)[KR]) {
#pragma unroll
    for (int q = 0; q < CPG; ++q)
#pragma unroll
      for (int j = 0; j < KR; ++j) acc[j] += m[q] * sm.v[(gb * CPG + q) * KR + j];
  };
  auto reduce_t = [&](double (&acc)[KR]) {  // over the G adjacent lanes of one row
#pragma unroll
    for (int j = 0; j < KR; ++j)
#pragma unroll
      for (int off = 1; off < G; off <<= 1) acc[j] += __shfl_xor(acc[j], off);
  };
  auto store = [&](int64_t r, int j, double v, bool good) {
    const int64_t row = i * B + r, col = j0 + j;
    if (row < n && col < nrhs)
      __hip_atomic_store(&X[col * ldx + row], good ? v : __builtin_nan(""), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  };

  int seen = 0;
  bool good = *info == 0;
  // this block row's own right-hand side (forward b_i, back y_i), loaded up
  // front so that its latency is off the critical path
  for (int e = t; e < B * KR; e += NT) {
    const int c = e % B, j = e / B;
    const int64_t row = i * B + c, col = j0 + j;
    sm.own[c * KR + j] = (row < n && col < nrhs) ? X[col * ldx + row] : 0.0;
  }
  __syncthreads();

  if constexpr (use_mfma<B, KR>()) {
    // v_mfma_f64_16x16x4_f64, lane l = 16 g + q: A(row q, k g), B(k g, col q),
    // result element e at (row g + 4e, col q).  Wave wv owns output rows
    // 16 wv .. 16 wv + 15 (no reduction across waves); at k-step ks the lane
    // uses tile index c = 32 g + ks for both operands, so its 32 A values of
    // a transposed tile are one contiguous run.  B values are the 16 columns
    // of the vector block, read from LDS (16 consecutive doubles per g).
    const int lane = t & 63, wv = t >> 6, q = lane & 15, g = lane >> 4;
    const int r0 = 16 * wv;
    auto mload_n = [&](const T *M, double (&m)[32]) {  // A = M
#pragma unroll
      for (int ks = 0; ks < 32; ++ks) m[ks] = (double)M[(32 * g + ks) * B + r0 + q];
    };
    auto mload_t = [&](const T *M, double (&m)[32]) {  // A = M^T
      const T *src = M + (r0 + q) * B + 32 * g;
      constexpr int VE = 16 / sizeof(T);
#pragma unroll
      for (int ks = 0; ks < 32; ks += VE) {
        T v[VE];
        *(uint4 *)&v[0] = *(const uint4 *)(src + ks);
#pragma unroll
        for (int e = 0; e < VE; ++e) m[ks + e] = (double)v[e];
      }
    };
    auto mprod = [&](const double (&m)[32], v4d &a) {
#pragma unroll
      for (int ks = 0; ks < 32; ++ks)
        a = __builtin_amdgcn_mfma_f64_16x16x4f64(m[ks], sm.v[(32 * g + ks) * KR + q], a, 0, 0, 0);
    };
    double md[32], mm[32];
    v4d a = {0.0, 0.0, 0.0, 0.0};
    if (FWD) {
      mload_t(dinv + i * BB, md);  // D_i^T
      for (int64_t p = 0; p < i; ++p) {
        mload_n(tiles + tile_index(i, p, N) * BB, mm);
        good &= wait_count(cnt, abort_word, (int)(p + 1), spin_max, seen, &ok_sh);
        load_v(p);
        __syncthreads();
        mprod(mm, a);
        __syncthreads();
      }
    } else {
      mload_n(dinv + i * BB, md);  // D_i
      for (int64_t p = N - 1; p > i; --p) {
        mload_t(tiles + tile_index(p, i, N) * BB, mm);
        good &= wait_count(cnt, abort_word, (int)(N - p), spin_max, seen, &ok_sh);
        load_v(p);
        __syncthreads();
        mprod(mm, a);
        __syncthreads();
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = r0 + g + 4 * e;
      sm.v[r * KR + q] = sm.own[r * KR + q] - a[e];
    }
    __syncthreads();
    v4d y = {0.0, 0.0, 0.0, 0.0};
    mprod(md, y);
#pragma unroll
    for (int e = 0; e < 4; ++e) store(r0 + g + 4 * e, q, y[e], good);
  } else if (FWD) {
    double dm[CPG], tm[CPG], acc[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) acc[j] = 0.0;
    load_t(dinv + i * BB, dm);  // D_i^T product
    for (int64_t p = 0; p < i; ++p) {
      load_n(tiles + tile_index(i, p, N) * BB, tm);
      good &= wait_count(cnt, abort_word, (int)(p + 1), spin_max, seen, &ok_sh);
      load_v(p);
      __syncthreads();
      prod_n(tm, acc);
      __syncthreads();
    }
    // r_i = b_i - sum over the column groups
#pragma unroll
    for (int j = 0; j < KR; ++j) sm.red[ga][ra * KR + j] = acc[j];
    __syncthreads();
    if (t < B) {
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        double s = sm.red[0][t * KR + j];
#pragma unroll
        for (int g = 1; g < G; ++g) s += sm.red[g][t * KR + j];
        sm.v[t * KR + j] = sm.own[t * KR + j] - s;
      }
    }
    __syncthreads();
    // y_i = D_i^T r_i
    double y[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) y[j] = 0.0;
    prod_t(dm, y);
    reduce_t(y);
    if (gb == 0) {
#pragma unroll
      for (int j = 0; j < KR; ++j) store(rb, j, y[j], good);
    }
  } else {
    double dm[CPG], tm[CPG], acc[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) acc[j] = 0.0;
    load_n(dinv + i * BB, dm);  // D_i product
    for (int64_t p = N - 1; p > i; --p) {
      load_t(tiles + tile_index(p, i, N) * BB, tm);
      good &= wait_count(cnt, abort_word, (int)(N - p), spin_max, seen, &ok_sh);
      load_v(p);
      __syncthreads();
      prod_t(tm, acc);
      __syncthreads();
    }
    reduce_t(acc);
    if (gb == 0) {
#pragma unroll
      for (int j = 0; j < KR; ++j) sm.v[rb * KR + j] = sm.own[rb * KR + j] - acc[j];
    }
    __syncthreads();
    // x_i = D_i r_i
    double x[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) x[j] = 0.0;
    prod_n(dm, x);
#pragma unroll
    for (int j = 0; j < KR; ++j) sm.red[ga][ra * KR + j] = x[j];
    __syncthreads();
    if (t < B) {
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        double s = sm.red[0][t * KR + j];
#pragma unroll
        for (int g = 1; g < G; ++g) s += sm.red[g][t * KR + j];
        store(t, j, s, good);
      }
    }
  }
  // publish block row i
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (t == 0)
    __hip_atomic_store(cnt, FWD ? (int)(i + 1) : (int)(N - i), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void clear_i32_kernel(int *p, int count) {
  for (int e = threadIdx.x; e < count; e += blockDim.x) p[e] = 0;
}

__global__ void scale_kernel(double *B_, int64_t n, int64_t ldb, int64_t nrhs, double alpha) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t r = e % n, c = e / n;
  B_[r + c * ldb] *= alpha;
}

template <int B, int KR, typename T>
void solve_run(const T *tiles, const T *dinv, int64_t N, int64_t n, double *X, int64_t ldx,
               int64_t nrhs, int *sync, int64_t sync_words, int spin_max, const int64_t *info,
               hipStream_t s) {
  // sync = [abort, forward counters (nch), back counters (nch)]
  const int64_t max_ch = (sync_words - 1) / 2;
  for (int64_t c0 = 0; c0 < nrhs; c0 += max_ch * KR) {
    const int64_t k = nrhs - c0 < max_ch * KR ? nrhs - c0 : max_ch * KR;
    const int64_t nch = (k + KR - 1) / KR;
    hipLaunchKernelGGL(clear_i32_kernel, dim3(1), dim3(256), 0, s, sync, (int)(1 + 2 * nch));
    const dim3 grid((unsigned)N, (unsigned)nch);
    double *Xc = X + c0 * ldx;
    hipLaunchKernelGGL((solve_kernel<B, KR, true, T>), grid, dim3(NT), 0, s, tiles, dinv, N, n,
                       Xc, ldx, k, sync + 1, sync, spin_max, info);
    hipLaunchKernelGGL((solve_kernel<B, KR, false, T>), grid, dim3(NT), 0, s, tiles, dinv, N, n,
                       Xc, ldx, k, sync + 1 + nch, sync, spin_max, info);
  }
}

template <int B, typename T>
void solve_rhs(const T *tiles, const T *dinv, int64_t N, int64_t n, double *X, int64_t ldx,
               int64_t nrhs, int *sync, int64_t sync_words, int spin_max, const int64_t *info,
               hipStream_t s) {
  if (nrhs == 1)
    solve_run<B, 1, T>(tiles, dinv, N, n, X, ldx, nrhs, sync, sync_words, spin_max, info, s);
  else if (nrhs <= 4)
    solve_run<B, 4, T>(tiles, dinv, N, n, X, ldx, nrhs, sync, sync_words, spin_max, info, s);
  else
    solve_run<B, 16, T>(tiles, dinv, N, n, X, ldx, nrhs, sync, sync_words, spin_max, info, s);
}

}  // namespace

void launch_solve(const void *tiles, const void *dinv, int store, int b, int64_t N, int64_t n,
                  double *X, int64_t ldx, int64_t nrhs, int *sync, int64_t sync_words,
                  int spin_max, const int64_t *info, hipStream_t s) {
  if (N <= 0 || nrhs <= 0 || sync_words < 3) return;
  if (b == 128) {
    if (store == STORE_F64)
      solve_rhs<128, double>((const double *)tiles, (const double *)dinv, N, n, X, ldx, nrhs,
                             sync, sync_words, spin_max, info, s);
    else
      solve_rhs<128, float>((const float *)tiles, (const float *)dinv, N, n, X, ldx, nrhs, sync,
                            sync_words, spin_max, info, s);
  } else {
    if (store == STORE_F64)
      solve_rhs<64, double>((const double *)tiles, (const double *)dinv, N, n, X, ldx, nrhs,
                            sync, sync_words, spin_max, info, s);
    else
      solve_rhs<64, float>((const float *)tiles, (const float *)dinv, N, n, X, ldx, nrhs, sync,
                           sync_words, spin_max, info, s);
  }
}

void launch_scale(double *B_, int64_t n, int64_t ldb, int64_t nrhs, double alpha, hipStream_t s) {
  const int64_t tot = n * nrhs;
  if (tot <= 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, B_, n,
                     ldb, nrhs, alpha);
}

}  // namespace chol
