// CPU tile kernels and thread pool of the heterogeneous factorisation (see
// host_tiles.hpp).  The matrix product uses an 8 x 6 register block of AVX2
// fused multiply-adds (12 accumulators of 4 doubles); the processor is
// checked at run time and a plain loop nest is used without AVX2/FMA.
#include "host_tiles.hpp"

#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

namespace chol {
namespace host {

int potrf_tile(double *L) {
  // right-looking by columns: scale column j by 1/sqrt(pivot), then
  // subtract its outer product from the columns to its right
  for (int j = 0; j < HB; ++j) {
    double *cj = L + (int64_t)j * HB;
    const double d = cj[j];
    if (!(d > 0.0)) return j + 1;
    const double s = std::sqrt(d);
    cj[j] = s;
    const double r = 1.0 / s;
    for (int i = j + 1; i < HB; ++i) cj[i] *= r;
    for (int k = j + 1; k < HB; ++k) {
      double *ck = L + (int64_t)k * HB;
      const double lkj = cj[k];
      for (int i = k; i < HB; ++i) ck[i] -= cj[i] * lkj;
    }
  }
  for (int j = 1; j < HB; ++j)
    for (int i = 0; i < j; ++i) L[(int64_t)j * HB + i] = 0.0;
  return 0;
}

void trsm_tile(const double *L, double *X) {
  // X L^T = A column by column: x_c = (a_c - sum_{t<c} x_t L(c, t)) / L(c, c),
  // applied as column operations over all 128 rows at once
  for (int c = 0; c < HB; ++c) {
    double *xc = X + (int64_t)c * HB;
    const double r = 1.0 / L[(int64_t)c * HB + c];
    for (int i = 0; i < HB; ++i) xc[i] *= r;
    for (int c2 = c + 1; c2 < HB; ++c2) {
      const double l = L[(int64_t)c * HB + c2];
      double *x2 = X + (int64_t)c2 * HB;
      for (int i = 0; i < HB; ++i) x2[i] -= xc[i] * l;
    }
  }
}

namespace {

__attribute__((target("avx2,fma"))) void gemm_avx2(double *C, const double *const *A,
                                                   const double *const *B, int np, bool lower) {
  // C(r, s) -= sum_p sum_k A_p(r, k) B_p(s, k); rows in blocks of 8, columns
  // in blocks of 6 (the last block of 2)
  for (int s0 = 0; s0 < HB; s0 += 6) {
    const int ns = std::min(6, HB - s0);
    for (int r0 = lower ? (s0 & ~7) : 0; r0 < HB; r0 += 8) {
      __m256d acc[2][6];
      for (int t = 0; t < 6; ++t) acc[0][t] = acc[1][t] = _mm256_setzero_pd();
      for (int p = 0; p < np; ++p) {
        const double *a = A[p] + r0;
        const double *b = B[p] + s0;
        if (ns == 6) {
          for (int k = 0; k < HB; ++k) {
            const __m256d a0 = _mm256_loadu_pd(a + (int64_t)k * HB);
            const __m256d a1 = _mm256_loadu_pd(a + (int64_t)k * HB + 4);
            const double *bk = b + (int64_t)k * HB;
#pragma GCC unroll 6
            for (int t = 0; t < 6; ++t) {
              const __m256d bv = _mm256_broadcast_sd(bk + t);
              acc[0][t] = _mm256_fmadd_pd(a0, bv, acc[0][t]);
              acc[1][t] = _mm256_fmadd_pd(a1, bv, acc[1][t]);
            }
          }
        } else {
          for (int k = 0; k < HB; ++k) {
            const __m256d a0 = _mm256_loadu_pd(a + (int64_t)k * HB);
            const __m256d a1 = _mm256_loadu_pd(a + (int64_t)k * HB + 4);
            const double *bk = b + (int64_t)k * HB;
            for (int t = 0; t < ns; ++t) {
              const __m256d bv = _mm256_broadcast_sd(bk + t);
              acc[0][t] = _mm256_fmadd_pd(a0, bv, acc[0][t]);
              acc[1][t] = _mm256_fmadd_pd(a1, bv, acc[1][t]);
            }
          }
        }
      }
      for (int t = 0; t < ns; ++t) {
        double *c = C + (int64_t)(s0 + t) * HB + r0;
        _mm256_storeu_pd(c, _mm256_sub_pd(_mm256_loadu_pd(c), acc[0][t]));
        _mm256_storeu_pd(c + 4, _mm256_sub_pd(_mm256_loadu_pd(c + 4), acc[1][t]));
      }
    }
  }
}

void gemm_plain(double *C, const double *const *A, const double *const *B, int np, bool lower) {
  for (int p = 0; p < np; ++p)
    for (int k = 0; k < HB; ++k)
      for (int s = 0; s < HB; ++s) {
        const double b = B[p][(int64_t)k * HB + s];
        double *c = C + (int64_t)s * HB;
        const double *a = A[p] + (int64_t)k * HB;
        for (int r = lower ? s : 0; r < HB; ++r) c[r] -= a[r] * b;
      }
}

const bool g_avx2 = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");

// ----------------------------------------------------------- thread pool --
// One job at a time: the caller publishes (fn, count) with a new epoch,
// every worker wakes, claims items from a shared counter, and acknowledges
// the epoch when the counter is exhausted; the caller returns only after all
// workers have acknowledged, so no worker is still inside the job when the
// next one is published.
struct Pool {
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::vector<std::thread> workers;
  const std::function<void(int64_t)> *fn = nullptr;
  int64_t count = 0;
  std::atomic<int64_t> next{0};
  int acks = 0;        // workers finished with the current epoch
  uint64_t epoch = 0;  // job generation
  bool stop = false;
  int nthreads = 0;

  void run_items() {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= count) break;
      (*fn)(i);
    }
  }
  void worker() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return stop || epoch != seen; });
      if (stop) return;
      seen = epoch;
      lk.unlock();
      run_items();
      lk.lock();
      if (++acks == nthreads - 1) done_cv.notify_all();
    }
  }
  void start(int n) {
    nthreads = std::max(1, n);
    for (int t = 1; t < nthreads; ++t) workers.emplace_back([this] { worker(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto &w : workers) w.join();
  }
};

std::mutex g_pool_mu;  // one parallel_for at a time
int g_want_threads = 0;
Pool *g_pool = nullptr;

Pool &pool() {
  if (!g_pool) {
    int n = g_want_threads;
    if (n <= 0) n = std::min(16, (int)std::max(1u, std::thread::hardware_concurrency()));
    g_pool = new Pool();  // kept until the process ends
    g_pool->start(n);
  }
  return *g_pool;
}

}  // namespace

// 8 independent partial sums per column dot product (vectorisable without
// reassociating a single sum); fixed order, so the result is reproducible.
static inline double dot128(const double *a, const double *b) {
  double d[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = 0; r < HB; r += 8)
    for (int j = 0; j < 8; ++j) d[j] += a[r + j] * b[r + j];
  return ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7]));
}

void tile_symv_pair(const double *T, const double *x_c, const double *x_i, double *y_row,
                    double *y_col, bool diag) {
  for (int r = 0; r < HB; ++r) y_row[r] = 0.0;
  if (diag) {
    double yc[HB];
    for (int c = 0; c < HB; ++c) {
      const double *col = T + (int64_t)c * HB;
      const double xc = x_c[c];
      for (int r = 0; r < HB; ++r) y_row[r] += col[r] * xc;
      yc[c] = dot128(col, x_c) - col[c] * xc;  // the diagonal counted once, in y_row
    }
    for (int r = 0; r < HB; ++r) y_row[r] += yc[r];
    return;
  }
  for (int c = 0; c < HB; ++c) {
    const double *col = T + (int64_t)c * HB;
    const double xc = x_c[c];
    for (int r = 0; r < HB; ++r) y_row[r] += col[r] * xc;
    y_col[c] += dot128(col, x_i);
  }
}

void gemm_nt_tiles(double *C, const double *const *A, const double *const *B, int np, bool lower) {
  if (g_avx2)
    gemm_avx2(C, A, B, np, lower);
  else
    gemm_plain(C, A, B, np, lower);
}

void set_threads(int n) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (!g_pool) g_want_threads = n;
}

int threads() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  return pool().nthreads;
}

void parallel_for(int64_t count, const std::function<void(int64_t)> &fn) {
  if (count <= 0) return;
  std::lock_guard<std::mutex> job(g_pool_mu);
  Pool &P = pool();
  if (P.nthreads == 1 || count == 1) {
    for (int64_t i = 0; i < count; ++i) fn(i);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(P.mu);
    P.fn = &fn;
    P.count = count;
    P.next = 0;
    P.acks = 0;
    ++P.epoch;
  }
  P.cv.notify_all();
  P.run_items();
  std::unique_lock<std::mutex> lk(P.mu);
  P.done_cv.wait(lk, [&] { return P.acks == P.nthreads - 1; });
}

}  // namespace host
}  // namespace chol
