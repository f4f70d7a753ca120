// Heterogeneous CPU + GPU Cholesky factorisation (the paper's heterogeneous
// Cholesky: Implementation, "Cholesky implementation"; Results, its
// workload-distribution and heterogeneous-vs-homogeneous comparisons).
//
// The blocked right-looking algorithm runs panel by panel (w tile columns).
// For the current trailing matrix a horizontal border splits the tile rows:
// rows above it (the shortest rows of the lower triangle, the diagonal tile
// included) belong to the CPU, rows below it to the GPU.  Per panel:
//   CPU: Step 1 on the diagonal tiles, Step 2 on its rows of the panel
//        (and the panel's own Step-3 updates on its rows);
//   CPU -> GPU: the panel's CPU-row tiles (the diagonal tile and the
//        sub-column below it down to the border, contiguous per column);
//   GPU: Step 2 on its rows of the panel, then Step 3 on its rows;
//   CPU: Step 3 on its rows, the next panel's columns first (so the next
//        panel can be factored and sent while the rest of the update runs).
// The GPU's rows are everything from the border down, so its Step 3 is the
// trailing triangle below the border plus the rectangle of its rows left of
// the border.  Since the trailing matrix shrinks, the border moves down to
// keep the CPU's share of each panel's Step-3 tiles near 1 - gpu_share (the
// border for panel p + 1's update is set from the trailing matrix below
// that panel, and moved once it is at least one panel width away); a move
// hands whole block rows from the GPU to the CPU (GPU -> CPU copies after
// the GPU has finished the previous panel's update).  When no CPU rows are
// left below the next panel, the CPU's rows go back to the GPU, which
// finishes with the plain schedule.
//
// Storage: the device workspace of chol_factor (packed lower tiles), and a
// host array with the same packed layout in which the CPU rows live while
// the CPU owns them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/chol.h"
#include "factor_handle.hpp"
#include "host_tiles.hpp"
#include "internal.hpp"

using namespace chol;

namespace {

constexpr int B = 128;
constexpr int64_t TE = (int64_t)B * B;  // elements per tile

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

struct Hetero {
  chol_factor_s *F;
  double *H;  // host tiles (packed layout)
  double *D;  // device tiles
  int64_t N;
  int64_t w;
  double share;  // target share of the Step-3 tiles on the GPU
  int shift_min;
  hipStream_t s;
  hipEvent_t ev_gpu = nullptr;
  int64_t border = 0;  // CPU rows: [current column, border)
  int64_t info = 0;
  int rc = CHOL_OK;
  chol_hetero_report rep{};

  double *h(int64_t i, int64_t k) { return H + tile_index(i, k, N) * TE; }
  double *d(int64_t i, int64_t k) { return D + tile_index(i, k, N) * TE; }
  bool ok(hipError_t e) {
    if (e != hipSuccess && rc == CHOL_OK) rc = CHOL_ERR_HIP;
    return rc == CHOL_OK;
  }

  // CPU rows wanted for a trailing matrix starting at column c: the largest m
  // with m (m + 1) / 2 <= (1 - share) R (R + 1) / 2, R = N - c.
  int64_t cpu_rows(int64_t c) const {
    const double R = (double)(N - c);
    if (R <= 0) return 0;
    const double want = (1.0 - share) * R * (R + 1.0) / 2.0;
    int64_t m = (int64_t)std::floor((std::sqrt(8.0 * want + 1.0) - 1.0) / 2.0);
    while (m > 0 && (double)m * (m + 1) / 2.0 > want) --m;
    return std::min<int64_t>(m, N - c);
  }

  // tiles (r, k) for rows [r0, r1) and columns [k0, min(k1, r + 1)): device
  // -> host (dir 0) or host -> device (dir 1), one copy per column run
  bool copy_rows(int64_t r0, int64_t r1, int64_t k0, int64_t k1, int dir) {
    for (int64_t k = k0; k < k1 && k < r1; ++k) {
      const int64_t a = std::max(r0, k);
      if (a >= r1) continue;
      const size_t bytes = (size_t)(r1 - a) * TE * sizeof(double);
      if (dir == 0) {
        if (!ok(hipMemcpyAsync(h(a, k), d(a, k), bytes, hipMemcpyDeviceToHost, s))) return false;
        rep.bytes_d2h += (double)bytes;
      } else {
        if (!ok(hipMemcpyAsync(d(a, k), h(a, k), bytes, hipMemcpyHostToDevice, s))) return false;
        rep.bytes_h2d += (double)bytes;
      }
    }
    return true;
  }

  // CPU: Steps 1-2 of panel [c0, c1) on rows [c0, border), with the panel's
  // own Step-3 updates.  Returns false on a non-positive pivot (info set).
  bool cpu_panel(int64_t c0, int64_t c1) {
    const auto t0 = clk::now();
    for (int64_t c = c0; c < c1; ++c) {
      const int bad = host::potrf_tile(h(c, c));
      if (bad) {
        info = c * B + bad;
        return false;
      }
      const double *L = h(c, c);
      host::parallel_for(border - c - 1, [&](int64_t t) { host::trsm_tile(L, h(c + 1 + t, c)); });
      // in-panel updates: tiles (i, k), k in (c, c1), i in [k, border)
      std::vector<std::pair<int64_t, int64_t>> work;
      for (int64_t k = c + 1; k < c1; ++k)
        for (int64_t i = k; i < border; ++i) work.emplace_back(i, k);
      host::parallel_for((int64_t)work.size(), [&](int64_t t) {
        const int64_t i = work[t].first, k = work[t].second;
        const double *a = h(i, c), *b = h(k, c);
        host::gemm_nt_tiles(h(i, k), &a, &b, 1, i == k);
      });
      rep.cpu_tile_updates += (double)work.size();
    }
    rep.ms_cpu += ms_since(t0);
    return true;
  }

  // CPU: Step 3 of panel [c0, c1) on tiles (i, k), k in [k0, k1), i in
  // [max(k, r0), r1)
  void cpu_update(int64_t c0, int64_t c1, int64_t k0, int64_t k1, int64_t r0, int64_t r1) {
    const auto t0 = clk::now();
    std::vector<std::pair<int64_t, int64_t>> work;
    for (int64_t k = k0; k < k1; ++k)
      for (int64_t i = std::max(k, r0); i < r1; ++i) work.emplace_back(i, k);
    const int np = (int)(c1 - c0);
    host::parallel_for((int64_t)work.size(), [&](int64_t t) {
      const int64_t i = work[t].first, k = work[t].second;
      const double *a[16], *b[16];
      for (int q = 0; q < np; ++q) {
        a[q] = h(i, c0 + q);
        b[q] = h(k, c0 + q);
      }
      host::gemm_nt_tiles(h(i, k), a, b, np, i == k);
    });
    rep.cpu_tile_updates += (double)work.size() * np;
    rep.ms_cpu += ms_since(t0);
  }

  // GPU: Step 2 of panel [c0, c1) on rows [border, N) (column by column,
  // with the panel's own updates), then its Step 3 on rows [border, N).
  void gpu_panel_and_update(int64_t c0, int64_t c1) {
    const int64_t r0 = border;
    if (r0 >= N) return;
    for (int64_t c = c0; c < c1; ++c) {
      launch_trsm(D, STORE_F64, B, N, c, F->d_info, s, r0);
      if (c + 1 < c1) {
        launch_update(D, STORE_F64, B, N, c, 1, c + 1, c1, /*rect*/ 2, 8, 0, F->d_info, s, 0,
                      nullptr, r0);
        rep.gpu_tile_updates += (double)(N - r0) * (c1 - c - 1);
      }
    }
    const int pw = (int)(c1 - c0);
    launch_update(D, STORE_F64, B, N, c0, pw, r0, N, /*tri*/ 0, 8, 0, F->d_info, s);
    rep.gpu_tile_updates += (double)(N - r0) * (N - r0 + 1) / 2 * pw;
    if (c1 < r0) {
      launch_update(D, STORE_F64, B, N, c0, pw, c1, r0, /*rect*/ 2, 8, 0, F->d_info, s, 0,
                    nullptr, r0);
      rep.gpu_tile_updates += (double)(N - r0) * (r0 - c1) * pw;
    }
    ok(hipGetLastError());
  }

  // the CPU hit a non-positive pivot: publish info to the device so that
  // every kernel still queued skips its work
  void publish_info() {
    const int64_t v = info;
    ok(hipMemcpyAsync(F->d_info, &v, sizeof(int64_t), hipMemcpyHostToDevice, s));
    ok(hipStreamSynchronize(s));
  }

  // Step-3 tile updates of the plain schedule from column c on (each column's
  // trailing triangle), counted for the report
  void count_tail(int64_t c) {
    for (; c < N; ++c) rep.gpu_tile_updates += (double)(N - c - 1) * (N - c) / 2.0;
  }

  void wait_gpu() {
    const auto t0 = clk::now();
    ok(hipEventRecord(ev_gpu, s));
    ok(hipEventSynchronize(ev_gpu));
    rep.ms_wait_gpu += ms_since(t0);
  }

  void run() {
    const int64_t m0 = cpu_rows(0);
    border = m0 >= std::min<int64_t>(w, N) ? m0 : 0;
    if (border > 0) {
      // the CPU rows of every column, device -> host
      if (!copy_rows(0, border, 0, border, 0)) return;
      wait_gpu();
      const int64_t c1 = std::min<int64_t>(w, N);
      if (!cpu_panel(0, c1)) return publish_info();
      if (!copy_rows(0, border, 0, c1, 1)) return;
      gpu_panel_and_update(0, c1);
    }
    int64_t c0 = 0;
    while (border > c0 && rc == CHOL_OK) {
      const int64_t c1 = std::min<int64_t>(c0 + w, N);  // panel p (factored, sent)
      if (c1 >= N) break;
      const int64_t n1 = std::min<int64_t>(c1 + w, N);  // panel p + 1
      const int64_t old = border;
      // the next panel's columns first
      cpu_update(c0, c1, c1, std::min(n1, old), c1, old);
      // the border for the next panel's trailing update (rows [n1, N))
      const int64_t m = cpu_rows(n1);
      const int64_t want = n1 + m;
      if (m == 0) {
        // no CPU share left below the next panel: finish its rows' update
        // and hand them to the GPU, which completes the factorisation alone
        cpu_update(c0, c1, n1, old, n1, old);
        if (!copy_rows(c1, old, c1, old, 1)) return;
        ++rep.border_shifts;
        rep.handover_column = c1;
        border = c1;
        count_tail(c1);
        if (enqueue_factor_tail(F, c1, w, 8, s) != CHOL_OK && rc == CHOL_OK) rc = CHOL_ERR_HIP;
        return;
      }
      if (want >= border + shift_min || border < n1) {
        // rows [border, want) move to the CPU once the GPU has applied this
        // panel's update to them
        const int64_t nb = std::min<int64_t>(want, N);
        wait_gpu();
        if (!copy_rows(border, nb, c1, nb, 0)) return;
        wait_gpu();
        border = nb;
        ++rep.border_shifts;
      }
      if (!cpu_panel(c1, n1)) return publish_info();
      if (!copy_rows(c1, border, c1, n1, 1)) return;
      gpu_panel_and_update(c1, n1);
      // the rest of this panel's update on the rows the CPU had before
      cpu_update(c0, c1, n1, old, n1, old);
      c0 = c1;
    }
    if (border <= c0 && rc == CHOL_OK && c0 == 0) {
      // no CPU share at all: the plain GPU schedule
      count_tail(0);
      if (enqueue_factor_tail(F, 0, w, 8, s) != CHOL_OK && rc == CHOL_OK) rc = CHOL_ERR_HIP;
      rep.handover_column = 0;
      return;
    }
    launch_diag_inverse(D, STORE_F64, B, N, F->dinv, F->d_info, s);
    ok(hipGetLastError());
  }
};

}  // namespace

extern "C" {

size_t chol_hetero_host_bytes(int64_t n) {
  if (n < 0) return 0;
  const int64_t N = (n + B - 1) / B;
  return (size_t)tile_count(N) * (size_t)TE * sizeof(double);
}

int chol_factor_hetero(const double *A, int64_t n, int64_t lda, double gpu_share, int panel_width,
                       void *workspace, size_t ws_bytes, double *host_ws, size_t host_bytes,
                       chol_handle *Fout, int64_t *info, chol_hetero_report *rep, void *stream) {
  const auto t0 = clk::now();
  if (n > 0 && !A) return -1;
  if (n < 0) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (!(gpu_share >= 0.0 && gpu_share <= 1.0)) return -4;
  if (panel_width < 0 || panel_width > 8) return -5;
  if (!workspace || ((uintptr_t)workspace & 255)) return -6;
  if (ws_bytes < chol_factor_bytes(n, CHOL_FP64, B)) return CHOL_ERR_WORKSPACE;
  if (!host_ws || host_bytes < chol_hetero_host_bytes(n)) return -8;
  if (!Fout) return -10;
  if (!info) return -11;
  chol_factor_s *F = new chol_factor_s();
  F->n = n;
  F->b = B;
  F->N = (n + B - 1) / B;
  F->precision = CHOL_FP64;
  (void)hipGetDevice(&F->device);
  F->d_info = (int64_t *)workspace;
  F->sync = (int *)((char *)workspace + kSolveSyncOff);
  F->tiles = (char *)workspace + kHeader;
  F->dinv = (char *)F->tiles + (size_t)tile_count(F->N) * TE * sizeof(double);
  F->stream = (hipStream_t)stream;
  if (hipEventCreateWithFlags(&F->ev_solve, hipEventDisableTiming) != hipSuccess) {
    F->ev_solve = nullptr;
    delete F;
    return CHOL_ERR_HIP;
  }
  Hetero h{};
  h.F = F;
  h.H = host_ws;
  h.D = (double *)F->tiles;
  h.N = F->N;
  h.w = panel_width > 0 ? panel_width : 8;
  h.share = gpu_share;
  h.shift_min = std::max<int>(1, (int)h.w);
  h.s = F->stream;
  h.rep.gpu_share_target = gpu_share;
  if (hipEventCreateWithFlags(&h.ev_gpu, hipEventDisableTiming) != hipSuccess) {
    delete F;
    return CHOL_ERR_HIP;
  }
  launch_clear_i64(F->d_info, 1, h.s);
  launch_pack(A, n, lda, F->tiles, STORE_F64, B, F->N, 1.0, h.s);
  if (F->N > 0) h.run();
  else launch_diag_inverse(F->tiles, STORE_F64, B, F->N, F->dinv, F->d_info, h.s);
  const auto tw = clk::now();
  if (hipStreamSynchronize(h.s) != hipSuccess && h.rc == CHOL_OK) h.rc = CHOL_ERR_HIP;
  h.rep.ms_wait_gpu += ms_since(tw);
  (void)hipEventDestroy(h.ev_gpu);
  if (h.rc != CHOL_OK) {
    delete F;
    return h.rc;
  }
  int64_t v = 0;
  if (hipMemcpy(&v, F->d_info, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess) {
    delete F;
    return CHOL_ERR_HIP;
  }
  F->info = v;
  *info = v;
  *Fout = F;
  if (rep) {
    h.rep.ms_total = ms_since(t0);
    const double tot = h.rep.gpu_tile_updates + h.rep.cpu_tile_updates;
    h.rep.gpu_share_tiles = tot > 0 ? h.rep.gpu_tile_updates / tot : 1.0;
    h.rep.cpu_threads = host::threads();
    *rep = h.rep;
  }
  return CHOL_OK;
}

// Host tile kernels, exported for tests and host-side callers.
int chol_host_potrf_tile(double *L) { return host::potrf_tile(L); }
void chol_host_trsm_tile(const double *L, double *X) { host::trsm_tile(L, X); }
void chol_host_gemm_nt_tiles(double *C, const double *const *A, const double *const *Bt, int np,
                             int lower) {
  host::gemm_nt_tiles(C, A, Bt, np, lower != 0);
}

}  // extern "C"
