// Host runtime and C ABI of the MI355X dense SPD / GP solver.
//
// The factorisation driver is the blocked right-looking algorithm of the
// paper (first algorithm figure, right column): for each column of tiles,
// Step 1 factors the diagonal tile, Step 2 solves the tiles below it, and
// Step 3 updates every trailing tile.  Two gfx950-specific changes of
// schedule, neither of which changes what is computed:
//  * panel width w: the Step-3 update of w consecutive tile columns is
//    applied to the far trailing matrix in one pass (inner dimension w*b),
//    which divides the trailing matrix's HBM traffic by w; the w columns
//    themselves are updated column by column before they are factored.
//  * lookahead: the update of the next w columns is split off and run,
//    together with their Steps 1-2, on a second stream, concurrently with
//    the bulk of the current trailing update.
// Every tile receives the same sequence of updates in the same order with or
// without these options, so results are bitwise identical across them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <vector>

#include "../../include/chol.h"
#include "factor_handle.hpp"
#include "host_tiles.hpp"
#include "internal.hpp"

using namespace chol;

namespace {


struct Options {
  std::atomic<int64_t> panel_width{0};  // 0: automatic
  std::atomic<int64_t> lookahead{1};
  std::atomic<int64_t> super_tile{8};
  std::atomic<int64_t> graph{0};
  std::atomic<int64_t> profile{0};
  std::atomic<int64_t> bulk_wg_cap{0};  // workgroups of the bulk update under lookahead (0 = all)
  std::atomic<int64_t> first_panel_width{0};  // tile columns of the first panel (0 = the panel width)
  std::atomic<int64_t> f16_wide{1};  // FP16 whole-triangle update with 2 x 2 tiles per workgroup
  std::atomic<int64_t> solve_spin_max{1 << 20};  // bound of each wait inside a solve
  std::atomic<int64_t> pcg_recompute{50};  // PCG: true residual every this many iterations
  std::atomic<int64_t> fp16_shift_c{32};   // FP16 retry: diagonal shift c * 2^-11 (0 = no retry)
  std::atomic<int64_t> panel_order{0};  // in-panel updates: 0 auto, 1 right, 2 left, 3 recursive
  std::atomic<int64_t> trsm_split{64};  // panel solves split by rows up to this many tiles
  std::atomic<int64_t> potrf_lookahead{2};  // fifth-wave POTRF: 0 never, 1 always, 2 automatic
};
Options g_opt;

// Lookahead resources: a side stream and four events per (device, caller
// stream), created on first use and kept until the process ends, so that
// factorisations issued concurrently on different caller streams (e.g. by
// the serving loop's worker threads) never share them.  No device memory.
struct SideCtx {
  int device = -1;
  hipStream_t caller = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_panel = nullptr, ev_bulk = nullptr, ev_join = nullptr;
};
std::mutex g_ctx_mu;
std::vector<SideCtx *> g_ctx;

int get_ctx(hipStream_t caller, SideCtx **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CHOL_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  for (SideCtx *c : g_ctx)
    if (c->device == dev && c->caller == caller) {
      *out = c;
      return CHOL_OK;
    }
  SideCtx *c = new SideCtx();
  c->device = dev;
  c->caller = caller;
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return CHOL_ERR_HIP;
  }
  const unsigned fl = hipEventDisableTiming;
  if (hipEventCreateWithFlags(&c->ev_fork, fl) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_panel, fl) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_bulk, fl) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, fl) != hipSuccess) {
    // a half-built context is released, so a later call can try again
    for (hipEvent_t e : {c->ev_fork, c->ev_panel, c->ev_bulk, c->ev_join})
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->side);
    delete c;
    return CHOL_ERR_HIP;
  }
  g_ctx.push_back(c);
  *out = c;
  return CHOL_OK;
}

// Captured factorisations (option "graph"): one executable graph per
// (A, lda, n, precision, tile, schedule, workspace), replayed on later calls
// with the same arguments.  Kernels take buffer addresses as arguments, so a
// graph is only valid for the buffers it was captured with.
struct GraphKey {
  const void *A;
  int64_t n, lda;
  int precision, tile;
  int64_t w;
  int la, S;
  void *ws;
  bool operator==(const GraphKey &o) const {
    return A == o.A && n == o.n && lda == o.lda && precision == o.precision && tile == o.tile &&
           w == o.w && la == o.la && S == o.S && ws == o.ws;
  }
};
struct GraphEntry {
  GraphKey key;
  int device;
  hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // most recently used last
constexpr size_t kMaxGraphs = 32;

// Event-bracketed timing of the trailing-update launches (option "profile").
struct ProfRec {
  hipEvent_t a, b;
  double flops;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;      // recorded, not yet read
std::vector<hipEvent_t> g_ev_free;
double g_prof_ms = 0.0, g_prof_flops = 0.0;
int64_t g_prof_n = 0;

hipEvent_t prof_event() {
  if (!g_ev_free.empty()) {
    hipEvent_t e = g_ev_free.back();
    g_ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Algorithmic flops of one update launch (see chol.h, kernel timing).
double update_flops(int b, int64_t N, int pw, int64_t k0, int64_t k1, int mode) {
  const double K = (double)pw * b, bb = (double)b;
  const int64_t R = N - k0;
  int64_t ndiag, noff;
  if (mode == 0) {
    ndiag = R;
    noff = R * (R - 1) / 2;
  } else {
    const int64_t Kc = k1 - k0;
    ndiag = Kc;
    noff = Kc * (Kc - 1) / 2 + (R - Kc) * Kc;
  }
  return (double)noff * 2.0 * bb * bb * K + (double)ndiag * bb * (bb + 1.0) * K;
}

// launch_update, bracketed by events when profiling.
void update(void *tiles, int st, int b, int64_t N, int64_t p0, int pw, int64_t k0, int64_t k1,
            int mode, int S, int fp16, const int64_t *info, hipStream_t s, int64_t max_wg = 0,
            const void *p16 = nullptr) {
  if (N - k0 <= 0 || (mode == 1 && k1 <= k0)) return;
  const int64_t prof = g_opt.profile;
  if (!prof || (prof == 2 && mode != 0)) {
    launch_update(tiles, st, b, N, p0, pw, k0, k1, mode, S, fp16, info, s, max_wg, p16);
    return;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t a = prof_event(), e = prof_event();
  if (a) (void)hipEventRecord(a, s);
  launch_update(tiles, st, b, N, p0, pw, k0, k1, mode, S, fp16, info, s, max_wg, p16);
  if (e) (void)hipEventRecord(e, s);
  if (a && e) g_prof.push_back({a, e, update_flops(b, N, pw, k0, k1, mode)});
}

}  // namespace

// Event brackets for kernels launched by other entry points (the CG tile
// product): recorded into the same list as the trailing-update launches,
// with `work` in that kernel's own unit.
namespace chol {
int64_t profile_option() { return g_opt.profile.load(); }
hipEvent_t profile_begin(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t a = prof_event();
  if (a) (void)hipEventRecord(a, s);
  return a;
}
void profile_end(hipStream_t s, hipEvent_t a, double work) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = prof_event();
  if (e) (void)hipEventRecord(e, s);
  if (a && e) g_prof.push_back({a, e, work});
}
}  // namespace chol

namespace {

int store_of(int precision) { return precision == CHOL_FP64 ? STORE_F64 : STORE_F32; }
size_t esize_of(int precision) { return precision == CHOL_FP64 ? 8 : 4; }
bool tile_ok(int tile) { return tile == 64 || tile == 128; }

}  // namespace

#define HIP_OK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return CHOL_ERR_HIP; \
  } while (0)

extern "C" {

const char *chol_status_string(int status) {
  switch (status) {
    case CHOL_OK: return "success";
    case CHOL_ERR_HIP: return "HIP runtime error";
    case CHOL_ERR_WORKSPACE: return "workspace too small";
    case CHOL_ERR_NOT_CONVERGED: return "refinement did not converge";
    case CHOL_ERR_NOT_SPD: return "matrix is not positive definite";
    case CHOL_ERR_UNSUPPORTED: return "unsupported precision or tile";
    case CHOL_ERR_BAD_HANDLE: return "invalid factor handle";
    default: break;
  }
  if (status < 0 && status > -64) return "invalid argument";
  return "unknown status";
}

int chol_set_option(const char *key, int64_t value) {
  if (!key) return -1;
  if (!strcmp(key, "panel_width")) {
    if (value < 0 || value > 32) return -2;
    g_opt.panel_width = value;
  } else if (!strcmp(key, "lookahead")) {
    if (value < 0 || value > 1) return -2;
    g_opt.lookahead = value;
  } else if (!strcmp(key, "super_tile")) {
    if (value < 1 || value > 64) return -2;
    g_opt.super_tile = value;
  } else if (!strcmp(key, "graph")) {
    if (value < 0 || value > 1) return -2;
    g_opt.graph = value;
  } else if (!strcmp(key, "profile")) {
    if (value < 0 || value > 2) return -2;
    g_opt.profile = value;
  } else if (!strcmp(key, "solve_spin_max")) {
    if (value < 1 || value > (int64_t)1 << 30) return -2;
    g_opt.solve_spin_max = value;
  } else if (!strcmp(key, "bulk_wg_cap")) {
    if (value < 0 || value > (int64_t)1 << 30) return -2;
    g_opt.bulk_wg_cap = value;
  } else if (!strcmp(key, "first_panel_width")) {
    if (value < 0 || value > 32) return -2;
    g_opt.first_panel_width = value;
  } else if (!strcmp(key, "f16_wide")) {
    if (value < 0 || value > 1) return -2;
    g_opt.f16_wide = value;
    set_f16_wide((int)value);
  } else if (!strcmp(key, "pcg_recompute")) {
    if (value < 0 || value > (int64_t)1 << 30) return -2;
    g_opt.pcg_recompute = value;
  } else if (!strcmp(key, "fp16_shift_c")) {
    if (value < 0 || value > 1024) return -2;
    g_opt.fp16_shift_c = value;
  } else if (!strcmp(key, "trsm_split")) {
    if (value < 0 || value > (int64_t)1 << 30) return -2;
    g_opt.trsm_split = value;
    set_trsm_split_max(value);
  } else if (!strcmp(key, "potrf_lookahead")) {
    if (value < 0 || value > 2) return -2;
    g_opt.potrf_lookahead = value;
  } else if (!strcmp(key, "panel_order")) {
    if (value < 0 || value > 3) return -2;
    g_opt.panel_order = value;
  } else if (!strcmp(key, "host_threads")) {
    if (value < 1 || value > 1024) return -2;
    host::set_threads((int)value);
  } else {
    return -1;
  }
  return CHOL_OK;
}

int64_t chol_get_option(const char *key) {
  if (!key) return -1;
  if (!strcmp(key, "panel_width")) return g_opt.panel_width;
  if (!strcmp(key, "lookahead")) return g_opt.lookahead;
  if (!strcmp(key, "super_tile")) return g_opt.super_tile;
  if (!strcmp(key, "graph")) return g_opt.graph;
  if (!strcmp(key, "profile")) return g_opt.profile;
  if (!strcmp(key, "bulk_wg_cap")) return g_opt.bulk_wg_cap;
  if (!strcmp(key, "first_panel_width")) return g_opt.first_panel_width;
  if (!strcmp(key, "f16_wide")) return g_opt.f16_wide;
  if (!strcmp(key, "solve_spin_max")) return g_opt.solve_spin_max;
  if (!strcmp(key, "pcg_recompute")) return g_opt.pcg_recompute;
  if (!strcmp(key, "fp16_shift_c")) return g_opt.fp16_shift_c;
  if (!strcmp(key, "panel_order")) return g_opt.panel_order;
  if (!strcmp(key, "trsm_split")) return g_opt.trsm_split;
  if (!strcmp(key, "potrf_lookahead")) return g_opt.potrf_lookahead;
  if (!strcmp(key, "host_threads")) return host::threads();
  return -1;
}

int chol_profile_read(double *ms, int64_t *launches, double *flops) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (const ProfRec &r : g_prof) {
    float t = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      return CHOL_ERR_HIP;
    g_prof_ms += t;
    g_prof_flops += r.flops;
    ++g_prof_n;
    g_ev_free.push_back(r.a);
    g_ev_free.push_back(r.b);
  }
  g_prof.clear();
  if (ms) *ms = g_prof_ms;
  if (launches) *launches = g_prof_n;
  if (flops) *flops = g_prof_flops;
  return CHOL_OK;
}

void chol_profile_reset(void) {
  double ms;
  int64_t l;
  double f;
  (void)chol_profile_read(&ms, &l, &f);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_ms = g_prof_flops = 0.0;
  g_prof_n = 0;
}

int chol_tile_default(int64_t n, int precision) {
  (void)precision;
  return n <= 512 ? 64 : 128;
}

size_t chol_factor_bytes(int64_t n, int precision, int tile) {
  if (n < 0 || precision < CHOL_FP64 || precision > CHOL_FP16_SCALED) return 0;
  if (tile == 0) tile = chol_tile_default(n, precision);
  if (!tile_ok(tile)) return 0;
  const int64_t N = (n + tile - 1) / tile;
  // packed lower tiles, then the N inverted diagonal blocks, then (FP16 form)
  // two FP16 panel buffers
  return kHeader +
         (size_t)(tile_count(N) + N) * (size_t)tile * (size_t)tile * esize_of(precision) +
         (precision == CHOL_FP16_SCALED ? 2 * (size_t)N * (size_t)kP16BytesPerTileRow : 0);
}

int gp_assemble(const double *X, int64_t n, int64_t d, int64_t ldx, double lengthscale,
                double variance, double noise, double *A, int64_t lda, int uplo_full,
                void *stream) {
  if (n > 0 && !X) return -1;
  if (n < 0) return -2;
  if (d < 1) return -3;
  if (ldx < d) return -4;
  if (!(lengthscale > 0.0)) return -5;
  if (!(variance >= 0.0)) return -6;
  if (!(noise >= 0.0)) return -7;
  if (n > 0 && !A) return -8;
  if (lda < (n > 1 ? n : 1)) return -9;
  const double two_l2 = 2.0 * lengthscale * lengthscale;
  launch_gp_assemble(X, n, d, ldx, two_l2, variance, noise, A, lda, uplo_full ? 1 : 0,
                     (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? CHOL_OK : CHOL_ERR_HIP;
}

// FP16 panel buffer of panel number p (consecutive panels alternate
// between the two buffers).
static void *panel_buf(const chol_factor_s *F, size_t p) {
  if (!F->p16) return nullptr;
  return (char *)F->p16 + (p & 1) * (size_t)F->N * (size_t)kP16BytesPerTileRow;
}

// Steps 1-2 and the in-panel Step 3 of panel number p, columns [c0, c1).
// The in-panel updates are right-looking (after column c, one update of the
// columns c+1 .. c1-1 of the panel by column c), left-looking (before column
// c, one update of column c by the columns c0 .. c-1) or recursive (the
// columns are halved: the left half is factored, the right half receives
// the left half's update in one launch, then the right half is factored, in
// both halves the same way down to two columns).  Each tile receives the
// same products in the same order in all three (the update kernels add the
// panel columns in increasing order and store C exactly), so the factor is
// bitwise the same; left-looking and recursive read and write the panel's
// tiles fewer times.
// In the FP16 form the panel solve also writes each finished tile column in
// FP16 into its two chunks of the panel's FP16 buffer, and the
// in-panel updates run on the FP16 matrix cores from there, like every
// other trailing update of that form; the buffer then holds the whole
// converted panel for the updates right of it.
static void factor_columns(chol_factor_s *F, size_t p, int64_t cp0, int64_t c0, int64_t c1, int st,
                           hipStream_t s) {
  const int64_t N = F->N;
  const int b = F->b;
  const int fp16 = F->p16 ? 1 : 0;
  // FP16 chunks of the panel's tile column c
  auto chunks = [&](int64_t c) -> void * {
    return fp16 ? (char *)panel_buf(F, p) + 2 * (c - cp0) * kP16BytesPerChunk : nullptr;
  };
  if (F->inpanel == 2 && c1 - c0 > 2) {
    const int64_t m = c0 + (c1 - c0) / 2;
    factor_columns(F, p, cp0, c0, m, st, s);
    update(F->tiles, st, b, N, c0, (int)(m - c0), m, c1, /*band*/ 1, 8, fp16, F->d_info, s, 0,
           chunks(c0));
    factor_columns(F, p, cp0, m, c1, st, s);
    return;
  }
  for (int64_t c = c0; c < c1; ++c) {
    if (F->inpanel == 1 && c > c0)
      update(F->tiles, st, b, N, c0, (int)(c - c0), c, c + 1, /*band*/ 1, 8, fp16, F->d_info, s, 0,
             chunks(c0));
    launch_potrf(F->tiles, st, b, N, c, F->d_info, s, F->potrf_la);
    if (fp16)
      launch_trsm_inv(F->tiles, N, c, F->dinv, chunks(c), F->d_info, s);
    else
      launch_trsm(F->tiles, st, b, N, c, F->d_info, s);
    if (F->inpanel != 1 && c + 1 < c1)
      update(F->tiles, st, b, N, c, 1, c + 1, c1, /*band*/ 1, 8, fp16, F->d_info, s, 0, chunks(c));
  }
}

static void factor_panel(chol_factor_s *F, size_t p, int64_t c0, int64_t c1, int st,
                         hipStream_t s) {
  factor_columns(F, p, c0, c0, c1, st, s);
}

// The plain schedule (no lookahead) from tile column c_start on, for a
// matrix already packed whose columns left of c_start are final and whose
// trailing part has received their updates; then the inverted diagonal
// blocks.  Used by the heterogeneous driver once the CPU's share is done.
}  // extern "C"
namespace chol {
int enqueue_factor_tail(chol_factor_s *F, int64_t c_start, int64_t w, int S, hipStream_t s) {
  const int64_t N = F->N;
  const int st = store_of(F->precision);
  for (int64_t c0 = c_start; c0 < N; c0 += w) {
    const int64_t c1 = std::min<int64_t>(c0 + w, N);
    factor_panel(F, 0, c0, c1, st, s);
    if (c1 < N)
      update(F->tiles, st, F->b, N, c0, (int)(c1 - c0), c1, N, /*tri*/ 0, S, 0, F->d_info, s);
  }
  launch_diag_inverse(F->tiles, st, F->b, N, F->dinv, F->d_info, s);
  return hipGetLastError() == hipSuccess ? CHOL_OK : CHOL_ERR_HIP;
}
}  // namespace chol
extern "C" {

// Enqueue the whole factorisation (clear info, pack, column steps) on the
// factor's stream and, with lookahead, the side stream joined back into it.
// Panels: the first w0 tile columns, then w at a time.
static int enqueue_factor(chol_factor_s *F, SideCtx *ctx, const double *A, int64_t lda, int st,
                          double pack_scale, int64_t w, int64_t w0, int S, bool la) {
  const double sh = F->shift;
  const int64_t N = F->N, n = F->n;
  const int b = F->b;
  const int fp16 = F->precision == CHOL_FP16_SCALED;
  hipStream_t s = F->stream;
  std::vector<int64_t> pb{0};  // panel p covers [pb[p], pb[p + 1])
  for (int64_t c = std::min<int64_t>(w0, N); ; c = std::min<int64_t>(c + w, N)) {
    pb.push_back(c);
    if (c >= N) break;
  }
  const size_t P = pb.size() - 1;
  launch_clear_i64(F->d_info, 1, s);
  if (!la) {
    launch_pack(A, n, lda, F->tiles, st, b, N, pack_scale, s, 0, -1, sh);
    for (size_t p = 0; p < P; ++p) {
      const int64_t c0 = pb[p], c1 = pb[p + 1];
      factor_panel(F, p, c0, c1, st, s);
      if (c1 < N)
        update(F->tiles, st, b, N, c0, (int)(c1 - c0), c1, N, /*tri*/ 0, S, fp16, F->d_info, s, 0,
               panel_buf(F, p));
    }
  } else {
    // the first panel's tile columns are packed first and factored on the
    // side stream while the main stream packs the rest (enqueued before the
    // first panel's launches, so that it need not wait for the host to issue
    // them)
    hipStream_t q = ctx->side;
    launch_pack(A, n, lda, F->tiles, st, b, N, pack_scale, s, 0, pb[1], sh);
    HIP_OK(hipEventRecord(ctx->ev_fork, s));
    HIP_OK(hipStreamWaitEvent(q, ctx->ev_fork, 0));
    launch_pack(A, n, lda, F->tiles, st, b, N, pack_scale, s, pb[1], N, sh);
    HIP_OK(hipEventRecord(ctx->ev_bulk, s));  // everything packed
    factor_panel(F, 0, 0, pb[1], st, q);
    for (size_t p = 0; p < P; ++p) {
      const int64_t c0 = pb[p], c1 = pb[p + 1];   // current panel [c0, c1)
      const int64_t n1 = p + 2 <= P ? pb[p + 2] : N;  // next panel [c1, n1)
      HIP_OK(hipEventRecord(ctx->ev_panel, q));      // panel p finished
      if (c1 < N) {
        // next panel: its update by this panel (after the previous bulk update,
        // which also wrote it, or after the packing), then its Steps 1-2, all
        // on the side stream.
        HIP_OK(hipStreamWaitEvent(q, ctx->ev_bulk, 0));
        update(F->tiles, st, b, N, c0, (int)(c1 - c0), c1, n1, /*band*/ 1, 8, fp16, F->d_info, q, 0,
               panel_buf(F, p));
        factor_panel(F, p + 1, c1, n1, st, q);
      }
      // bulk update of the columns right of the next panel, on the main stream
      HIP_OK(hipStreamWaitEvent(s, ctx->ev_panel, 0));
      if (n1 < N) {
        update(F->tiles, st, b, N, c0, (int)(c1 - c0), n1, N, /*tri*/ 0, S, fp16, F->d_info, s,
               g_opt.bulk_wg_cap.load(), panel_buf(F, p));
      }
      HIP_OK(hipEventRecord(ctx->ev_bulk, s));
    }
    HIP_OK(hipEventRecord(ctx->ev_join, q));
    HIP_OK(hipStreamWaitEvent(s, ctx->ev_join, 0));
  }
  // inverted diagonal blocks for the solves (the FP16 form has made each one
  // for its panel solve, right after the diagonal factorisation)
  if (!fp16) launch_diag_inverse(F->tiles, st, b, N, F->dinv, F->d_info, s);
  return hipGetLastError() == hipSuccess ? CHOL_OK : CHOL_ERR_HIP;
}

int chol_factor(const double *A, int64_t n, int64_t lda, int precision, int tile,
                void *workspace, size_t ws_bytes, chol_handle *Fout, int64_t *info,
                void *stream) {
  chol_factor_opts o{tile, 0, -1, 0, -1};
  return chol_factor_ex(A, n, lda, precision, &o, workspace, ws_bytes, Fout, info, stream);
}

int chol_factor_ex(const double *A, int64_t n, int64_t lda, int precision,
                   const chol_factor_opts *opts, void *workspace, size_t ws_bytes,
                   chol_handle *Fout, int64_t *info, void *stream) {
  int tile = opts ? opts->tile : 0;
  if (opts && (opts->panel_width > 32 || opts->super_tile > 64 || opts->lookahead > 1)) return -5;
  if (n > 0 && !A) return -1;
  if (n < 0) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (precision < CHOL_FP64 || precision > CHOL_FP16_SCALED) return -4;
  if (tile == 0) tile = chol_tile_default(n, precision);
  if (!tile_ok(tile)) return -5;
  if (!workspace || ((uintptr_t)workspace & 255)) return -6;
  const size_t need = chol_factor_bytes(n, precision, tile);
  if (ws_bytes < need) return CHOL_ERR_WORKSPACE;
  if (!Fout) return -8;
  if (precision == CHOL_FP16_SCALED && tile != 128) return CHOL_ERR_UNSUPPORTED;

  SideCtx *ctx = nullptr;
  int rc = get_ctx((hipStream_t)stream, &ctx);
  if (rc) return rc;

  chol_factor_s *F = new chol_factor_s();
  F->n = n;
  F->b = tile;
  F->N = (n + tile - 1) / tile;
  F->precision = precision;
  (void)hipGetDevice(&F->device);
  F->d_info = (int64_t *)workspace;
  F->sync = (int *)((char *)workspace + kSolveSyncOff);
  if (hipEventCreateWithFlags(&F->ev_solve, hipEventDisableTiming) != hipSuccess) {
    F->ev_solve = nullptr;
    delete F;
    return CHOL_ERR_HIP;
  }
  F->tiles = (char *)workspace + kHeader;
  F->dinv = (char *)F->tiles + (size_t)tile_count(F->N) * (size_t)tile * tile * esize_of(precision);
  if (precision == CHOL_FP16_SCALED)
    F->p16 = (char *)F->dinv + (size_t)F->N * (size_t)tile * tile * esize_of(precision);
  F->stream = (hipStream_t)stream;
  const int st = store_of(precision);
  const int64_t N = F->N;
  const int b = F->b;
  hipStream_t s = F->stream;

  // Scaling for the FP16 form: the factor of H = A / s is computed, with s
  // the largest diagonal entry (reduced on the device into the workspace
  // header, then one 8-byte read-back).
  double pack_scale = 1.0;
  if (precision == CHOL_FP16_SCALED && n > 0) {
    double *d_mx = (double *)((char *)workspace + 64);
    launch_max_diag(A, lda, n, d_mx, s);
    double mx = 0.0;
    HIP_OK(hipMemcpyAsync(&mx, d_mx, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (!(mx > 0.0)) mx = 1.0;
    F->scale = mx;
    pack_scale = 1.0 / mx;
  }

  // panel width: tile columns per Step-3 pass over the far trailing matrix
  const int64_t pw_opt =
      (opts && opts->panel_width > 0) ? (int64_t)opts->panel_width : g_opt.panel_width.load();
  // (widths above 8 only for the FP16 form, whose update is bound by the
  // traffic of C rather than by the matrix cores)
  // automatic width, from the autotuner's sweep on MI355X: 8 for small
  // (chain-bound) and large matrices, 4 in between
  int64_t w = pw_opt > 0 ? pw_opt : (N >= 192 ? 8 : (N >= 64 ? 4 : 8));
  // FP16 form from 512 tile rows: 32 (n = 131072: factor 901 ms against 909
  // with 24, 967 with 16, 1070 with 8)
  if (pw_opt <= 0 && precision == CHOL_FP16_SCALED && N >= 512) w = 32;
  if (precision != CHOL_FP16_SCALED && w > 8) w = 8;
  const int S =
      (int)((opts && opts->super_tile > 0) ? (int64_t)opts->super_tile : g_opt.super_tile.load());
  const int fp16 = precision == CHOL_FP16_SCALED;
  const int64_t la_opt =
      (opts && opts->lookahead >= 0) ? (int64_t)opts->lookahead : g_opt.lookahead.load();
  const bool la = la_opt != 0 && N > w;
  const int64_t fw = g_opt.first_panel_width.load();
  const int64_t w0 = fw > 0 ? std::min<int64_t>(fw, w) : w;
  // in-panel update order (same factor in all).  Automatic: left-looking for
  // the FP16 form, whose in-panel updates are cheap on the matrix cores but
  // move FP32 C tiles (n = 131072: 1036 against 1102 ms right-looking, 1011
  // against 1019 ms recursive); recursive from 256 tile rows on (FP64
  // n = 32768: 200.6 against 203.0 ms, n = 65536: 1455.8 against 1466.4 ms;
  // FP32 n = 65536: 743.1 against 747.3 ms), right-looking below, where the
  // longer column chain of the other two costs more than the traffic they
  // save (FP64 n = 1024: 0.77 against 0.86 ms recursive, 1.26 left-looking;
  // n = 8192: 10.4 against 10.6 ms).
  const int64_t po = g_opt.panel_order.load();
  F->inpanel = po == 1   ? 0
               : po == 2 ? 1
               : po == 3 ? 2
               : precision == CHOL_FP16_SCALED ? 1
               : N >= 256                      ? 2
                                               : 0;
  // diagonal factorisations with the fifth-wave lookahead (same factor):
  // automatic up to 64 tile rows, where the column chain is most of the
  // factorisation (n = 1024: 0.86 -> 0.77 ms, n = 8192: 10.36 -> 9.66 ms);
  // beyond, the diagonal factorisation runs beside trailing updates, whose
  // workgroups leave room for four waves more readily than for five
  // (n = 16384: 36.7 against 37.1 ms with it, n = 32768: 201.8 against 209.5)
  const int64_t pl = g_opt.potrf_lookahead.load();
  F->potrf_la = pl == 1 || (pl == 2 && N <= 64);


  // Stream capture is not allowed on the legacy NULL stream: direct launches there.
  const bool graph = (opts && opts->graph >= 0 ? opts->graph != 0 : g_opt.graph != 0) &&
                     precision != CHOL_FP16_SCALED && !g_opt.profile && s != nullptr;
  GraphKey gk{A, n, lda, precision, tile, w * 64 + w0,
              (la ? 1 : 0) + 2 * F->inpanel + (F->potrf_la ? 8 : 0), S, workspace};
  if (graph) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (size_t e = 0; e < g_graphs.size(); ++e) {
      if (g_graphs[e].device == dev && g_graphs[e].key == gk) {
        GraphEntry ge = g_graphs[e];
        g_graphs.erase(g_graphs.begin() + e);
        g_graphs.push_back(ge);
        if (hipGraphLaunch(ge.exec, s) != hipSuccess) {
          delete F;
          return CHOL_ERR_HIP;
        }
        *Fout = F;
        if (info) return chol_get_info(F, info);
        return CHOL_OK;
      }
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      delete F;
      return CHOL_ERR_HIP;
    }
  }
  rc = enqueue_factor(F, ctx, A, lda, st, pack_scale, w, w0, S, la);
  if (rc != CHOL_OK) {
    if (graph) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    delete F;
    return rc;
  }
  if (graph) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    if (hipStreamEndCapture(s, &g) != hipSuccess ||
        hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      delete F;
      return CHOL_ERR_HIP;
    }
    (void)hipGraphDestroy(g);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> lk(g_graph_mu);
      if (g_graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
      }
      g_graphs.push_back({gk, dev, ge});
    }
    if (hipGraphLaunch(ge, s) != hipSuccess) {
      delete F;
      return CHOL_ERR_HIP;
    }
  }
  if (hipGetLastError() != hipSuccess) {
    delete F;
    return CHOL_ERR_HIP;
  }
  *Fout = F;
  if (info) {
    rc = chol_get_info(F, info);
    if (rc) return rc;
    // FP16 form, non-positive pivot: retry once with the diagonal shift
    // c u_16 I added to the scaled matrix, then fall back to an FP32 factor
    // (the FP32 factor needs less workspace than the FP16 form).
    if (*info > 0 && precision == CHOL_FP16_SCALED) {
      const int64_t c = g_opt.fp16_shift_c.load();
      if (c > 0) {
        F->shift = (double)c * 0x1p-11;
        F->fallback |= CHOL_FALLBACK_SHIFT;
        F->info = -1;
        rc = enqueue_factor(F, ctx, A, lda, st, pack_scale, w, w0, S, la);
        if (rc) return rc;
        rc = chol_get_info(F, info);
        if (rc) return rc;
      }
      if (*info > 0) {
        F->precision = CHOL_FP32;
        F->scale = 1.0;
        F->shift = 0.0;
        F->p16 = nullptr;
        F->fallback |= CHOL_FALLBACK_FP32;
        F->info = -1;
        const int64_t w32 = std::min<int64_t>(w, 8);
        rc = enqueue_factor(F, ctx, A, lda, STORE_F32, 1.0, w32, std::min(w0, w32), S,
                            la_opt != 0 && N > w32);
        if (rc) return rc;
        rc = chol_get_info(F, info);
        if (rc) return rc;
      }
    }
  }
  return CHOL_OK;
}

int chol_get_info(chol_handle F, int64_t *info) {
  if (!F) return CHOL_ERR_BAD_HANDLE;
  if (F->info < 0) {
    int64_t v = 0;
    if (F->ev_ready)
      HIP_OK(hipEventSynchronize(F->ev_ready));
    else
      HIP_OK(hipStreamSynchronize(F->stream));
    HIP_OK(hipMemcpy(&v, F->d_info, sizeof(int64_t), hipMemcpyDeviceToHost));
    F->info = v;
  }
  if (info) *info = F->info;
  return CHOL_OK;
}

int64_t chol_factor_n(chol_handle F) { return F ? F->n : -1; }
int chol_factor_tile(chol_handle F) { return F ? F->b : -1; }
int chol_factor_precision(chol_handle F) { return F ? F->precision : -1; }
int chol_factor_fallback(chol_handle F) { return F ? F->fallback : -1; }

void chol_factor_free(chol_handle F) { delete F; }

int chol_solve(chol_handle F, double *B, int64_t nrhs, int64_t ldb, void *stream) {
  if (!F) return CHOL_ERR_BAD_HANDLE;
  if (nrhs > 0 && !B) return -2;
  if (nrhs < 0) return -3;
  if (ldb < (F->n > 1 ? F->n : 1)) return -4;
  if (F->info > 0) return CHOL_ERR_NOT_SPD;
  hipStream_t s = (hipStream_t)stream;
  const int st = store_of(F->precision);
  if (F->n == 0 || nrhs == 0) return CHOL_OK;
  // order after the previous solve with this factor if it ran on another
  // stream (both use the synchronisation words in the factor's workspace);
  // skipped on a capturing stream, whose earlier solves are on that stream
  std::lock_guard<std::mutex> lk(F->solve_mu);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_OK(hipStreamIsCapturing(s, &cap));
  if (F->solved && F->last_solve != s && cap == hipStreamCaptureStatusNone)
    HIP_OK(hipStreamWaitEvent(s, F->ev_solve, 0));
  launch_solve(F->tiles, F->dinv, st, F->b, F->N, F->n, B, ldb, nrhs, F->sync, kSolveSyncWords,
               (int)g_opt.solve_spin_max.load(), F->d_info, s);
  if (F->scale != 1.0) launch_scale(B, F->n, ldb, nrhs, 1.0 / F->scale, s);
  HIP_OK(hipEventRecord(F->ev_solve, s));
  F->last_solve = s;
  F->solved = true;
  return hipGetLastError() == hipSuccess ? CHOL_OK : CHOL_ERR_HIP;
}

int chol_factor_to_dense(chol_handle F, double *L, int64_t ldl, void *stream) {
  if (!F) return CHOL_ERR_BAD_HANDLE;
  if (F->n > 0 && !L) return -2;
  if (ldl < (F->n > 1 ? F->n : 1)) return -3;
  launch_unpack(F->tiles, store_of(F->precision), F->b, F->N, F->n, std::sqrt(F->scale), L, ldl,
                F->d_info, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? CHOL_OK : CHOL_ERR_HIP;
}

int chol_residual(const double *A, int64_t lda, int64_t n, const double *X, int64_t ldx,
                  const double *B, int64_t ldb, double *R, int64_t ldr, int64_t nrhs,
                  void *stream) {
  if (n > 0 && !A) return -1;
  if (lda < (n > 1 ? n : 1)) return -2;
  if (n < 0) return -3;
  if (nrhs < 0) return -10;
  if (n > 0 && nrhs > 0 && (!X || !B || !R)) return -4;
  if (ldx < (n > 1 ? n : 1)) return -5;
  if (ldb < (n > 1 ? n : 1)) return -7;
  if (ldr < (n > 1 ? n : 1)) return -9;
  launch_symm_residual(A, lda, n, X, ldx, B, ldb, R, ldr, nrhs, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? CHOL_OK : CHOL_ERR_HIP;
}


// ---------------------------------------------------------- refinement ----
// Workspace layout: five n x nrhs FP64 blocks (leading dimension n)
//   r (residual), z (IR correction / PCG preconditioned residual), p, q = -A p,
//   t (true residual at a check),
// then per right-hand side: rr, xx, dd (squared norms of r, x and the last
// correction, read back together), rho, rho_new, pq, alpha, beta, bb (b.b);
// two int32 masks (active columns, columns being confirmed); and the
// dot-product partials (128 per right-hand side).
size_t chol_refine_bytes(int64_t n, int64_t nrhs, int method) {
  if (n < 0 || nrhs < 0 || (method != CHOL_REFINE_IR && method != CHOL_REFINE_PCG)) return 0;
  const size_t vec = (size_t)n * (size_t)nrhs * sizeof(double);
  return 5 * vec + (size_t)(9 + 1 + 128) * (size_t)nrhs * sizeof(double) + 256;
}

namespace {

// One call of chol_refine_solve: the iterative refinement of classic
// mixed-precision solvers (x <- x + M^{-1}(b - A x), M = F F^T) and the
// paper's CG algorithm preconditioned with M, on device vectors; the host
// reads back three squared norms per right-hand side per iteration and
// decides the stopping tests, the scalars of CG stay on the device.
struct Refiner {
  chol_factor_s *F;
  const double *A;
  int64_t lda;
  const double *Xf;
  int64_t d, ldxf;
  double two_l2, var, noise;
  const double *B;
  int64_t ldb;
  double *X;
  int64_t ldx, n, k;
  double tol, lam;
  bool certify;
  hipStream_t s;
  double *r, *z, *p, *q, *t;
  double *nrm;  // rr[k], xx[k], dd[k]
  double *rho, *rho_new, *pq, *alpha, *beta, *bb;
  int32_t *act, *msk;
  double *partial;
  std::vector<double> h_nrm, h_bb, cert;
  std::vector<int32_t> h_act, h_msk;
  int iters = 0;
  int fallback = 0;
  int rc = CHOL_OK;

  void setup(void *ws) {
    const size_t vec = (size_t)n * (size_t)k;
    r = (double *)ws;
    z = r + vec;
    p = z + vec;
    q = p + vec;
    t = q + vec;
    nrm = t + vec;
    rho = nrm + 3 * k;
    rho_new = rho + k;
    pq = rho_new + k;
    alpha = pq + k;
    beta = alpha + k;
    bb = beta + k;
    act = (int32_t *)(bb + k);
    msk = act + k;
    partial = (double *)act + k;  // k doubles hold the two int32 masks
    h_nrm.assign(3 * k, 0.0);
    h_bb.assign(k, 0.0);
    cert.assign(k, INFINITY);
    h_act.assign(k, 1);
    h_msk.assign(k, 0);
  }
  bool ok(hipError_t e) {
    if (e != hipSuccess && rc == CHOL_OK) rc = CHOL_ERR_HIP;
    return rc == CHOL_OK;
  }
  // out = B - A x (or -A x when rhs is false); exact = false: plain FP64
  // accumulation instead of double-double (stored A only)
  void residual(const double *x, int64_t ldxx, double *out, bool rhs = true, bool exact = true) {
    const double *Bm = rhs ? B : nullptr;
    if (A)
      launch_symm_residual(A, lda, n, x, ldxx, Bm, ldb, out, n, k, s, exact);
    else
      launch_gp_residual(Xf, n, d, ldxf, two_l2, var, noise, x, ldxx, Bm, ldb, out, n, k, s);
  }
  void msolve(double *v) {
    const int e = chol_solve(F, v, k, n, s);
    if (e && rc == CHOL_OK) rc = e;
  }
  // rr = r.r, xx = x.x (and dd = z.z), read back; one synchronisation
  bool norms(bool with_dd) {
    launch_col_dot(r, n, r, n, n, k, nrm, partial, s);
    launch_col_dot(X, ldx, X, ldx, n, k, nrm + k, partial, s);
    if (with_dd) launch_col_dot(z, n, z, n, n, k, nrm + 2 * k, partial, s);
    if (!ok(hipMemcpyAsync(h_nrm.data(), nrm, (with_dd ? 3 : 2) * k * sizeof(double),
                           hipMemcpyDeviceToHost, s)))
      return false;
    return ok(hipStreamSynchronize(s));
  }
  double cert_of(int64_t c) const {
    const double rn = std::sqrt(h_nrm[c]), xn = std::sqrt(h_nrm[k + c]);
    const double ce = certify ? rn / (lam * xn) : rn / std::sqrt(h_bb[c]);
    return std::isnan(ce) ? INFINITY : ce;
  }
  // the stopping test on the current r and x: the certificate
  // ||r|| / (lam ||x||) <= tol / 2, or without a bound on the smallest
  // eigenvalue ||r|| <= tol ||b|| (PCG; IR tests its correction)
  bool passes(int64_t c) const { return cert[c] <= (certify ? 0.5 * tol : tol); }
  bool upload(int32_t *dst, const std::vector<int32_t> &src) {
    return ok(hipMemcpyAsync(dst, src.data(), k * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  int active_count() const {
    int a = 0;
    for (int64_t c = 0; c < k; ++c) a += h_act[c];
    return a;
  }

  // Iterative refinement.  Returns true when PCG should take over (a column
  // whose correction failed to halve twice in a row: stagnation).  With a
  // certificate and a stored A the working residuals are plain FP64; the
  // residual is taken again in double-double before any column is tested
  // (as soon as one passes on the working residual, and at the iteration
  // limit), and for good once a column stalls, so every certificate comes
  // from a double-double residual.  When the last certificate times the last
  // contraction of the corrections predicts a pass for every active column
  // (with a factor 2 to spare), the residual is taken in double-double at
  // once instead of twice; when a plain residual's certificate lies far
  // (16x) above that prediction, the plain residuals have reached their own
  // rounding level and the rest are taken in double-double.  With one
  // right-hand side both forms are bound by HBM: double-double throughout.
  bool run_ir(int max_iter) {
    std::vector<double> dprev(k, INFINITY), ratio(k, INFINITY);
    std::vector<int> stall(k, 0);
    bool fast = certify && A != nullptr && k > 1;
    if (!upload(act, h_act)) return false;
    for (;;) {
      bool exact = !fast;
      if (fast && iters >= 2) {
        exact = true;
        for (int64_t c = 0; c < k; ++c)
          if (h_act[c] && !(cert[c] * ratio[c] <= 0.25 * tol)) exact = false;
      }
      residual(X, ldx, r, true, exact);
      if (!norms(iters > 0)) return false;
      if (!exact) {
        bool confirm = iters >= max_iter;
        for (int64_t c = 0; c < k; ++c) {
          if (!h_act[c]) continue;
          const double ce = cert_of(c);
          if (ce <= 0.5 * tol) confirm = true;
          if (iters >= 2 && ce > 16.0 * cert[c] * ratio[c]) confirm = true, fast = false;
        }
        if (confirm) {
          residual(X, ldx, r, true, true);
          if (!norms(iters > 0)) return false;
        }
      }
      bool changed = false;
      for (int64_t c = 0; c < k; ++c) {
        if (!h_act[c]) continue;
        if (certify) {
          cert[c] = cert_of(c);
          if (cert[c] <= 0.5 * tol) {
            h_act[c] = 0;
            changed = true;
            continue;
          }
        }
        if (iters > 0) {
          const double dn = std::sqrt(h_nrm[2 * k + c]), xn = std::sqrt(h_nrm[k + c]);
          if (!certify) {
            cert[c] = std::isnan(dn / xn) ? INFINITY : dn / xn;
            if (dn <= tol * xn) {
              h_act[c] = 0;
              changed = true;
              continue;
            }
          }
          stall[c] = dn > 0.5 * dprev[c] ? stall[c] + 1 : 0;
          if (std::isfinite(dprev[c]) && dprev[c] > 0.0) ratio[c] = dn / dprev[c];
          dprev[c] = dn;
        }
      }
      if (active_count() == 0 || iters >= max_iter) return false;
      bool stalled = false;
      for (int64_t c = 0; c < k; ++c)
        if (h_act[c] && stall[c] >= 2) stalled = true;
      if (stalled) {
        if (!fast) return true;
        fast = false;  // perhaps at the working residual's rounding level
        std::fill(stall.begin(), stall.end(), 0);
      }
      if (changed && !upload(act, h_act)) return false;
      launch_copy(r, n, z, n, n, k, s);
      msolve(z);
      launch_axpby(z, n, X, ldx, n, k, nullptr, 1.0, nullptr, act, s);  // x += d
      ++iters;
      if (rc) return false;
    }
  }

  // CG preconditioned with M = F F^T from the current x, for the active
  // columns, with the true residual every `recompute` iterations and before
  // a column is declared converged.
  void run_pcg(int max_iter, int64_t recompute) {
    residual(X, ldx, r);
    if (!norms(false)) return;
    for (int64_t c = 0; c < k; ++c)
      if (h_act[c]) {
        cert[c] = cert_of(c);
        if (passes(c)) h_act[c] = 0;
      }
    if (active_count() == 0 || !upload(act, h_act)) return;
    launch_copy(r, n, z, n, n, k, s);
    msolve(z);
    launch_copy(z, n, p, n, n, k, s);
    launch_col_dot(r, n, z, n, n, k, rho, partial, s);
    for (int64_t it = 1; iters < max_iter; ++it) {
      residual(p, n, q, false, k == 1);                                // q = -A p
      launch_col_dot(p, n, q, n, n, k, pq, partial, s);
      launch_pcg_alpha(rho, pq, act, alpha, k, s);                     // rho / p.Ap
      launch_axpby(p, n, X, ldx, n, k, alpha, 1.0, nullptr, act, s);  // x += alpha p
      launch_axpby(q, n, r, n, n, k, alpha, 1.0, nullptr, act, s);     // r -= alpha A p
      ++iters;
      if (recompute > 0 && it % recompute == 0) {
        residual(X, ldx, t);
        launch_copy_masked(t, n, r, n, n, k, act, s);
      }
      if (!norms(false)) return;
      bool any = false;
      for (int64_t c = 0; c < k; ++c) {
        h_msk[c] = 0;
        if (!h_act[c]) continue;
        cert[c] = cert_of(c);
        if (passes(c)) h_msk[c] = 1, any = true;
      }
      if (any) {
        // confirm on the true residual; a column that fails keeps it as r
        residual(X, ldx, t);
        if (!upload(msk, h_msk)) return;
        launch_copy_masked(t, n, r, n, n, k, msk, s);
        if (!norms(false)) return;
        bool changed = false;
        for (int64_t c = 0; c < k; ++c)
          if (h_msk[c]) {
            cert[c] = cert_of(c);
            if (passes(c)) h_act[c] = 0, changed = true;
          }
        if (active_count() == 0) return;
        if (changed && !upload(act, h_act)) return;
      }
      launch_copy(r, n, z, n, n, k, s);
      msolve(z);
      launch_col_dot(r, n, z, n, n, k, rho_new, partial, s);
      launch_pcg_beta(rho_new, rho, act, beta, k, s);                 // beta; rho <- rho_new
      launch_axpby(z, n, p, n, n, k, nullptr, 1.0, beta, act, s);     // p = z + beta p
      if (rc) return;
    }
  }
};

}  // namespace

int chol_refine_solve(chol_handle F, const double *A, int64_t lda, const double *Xf, int64_t d,
                      int64_t ldxf, double lengthscale, double variance, double noise,
                      const double *B, int64_t ldb, double *X, int64_t ldxs, int64_t nrhs,
                      double tol, int max_iter, int method, void *workspace, size_t ws_bytes,
                      chol_refine_report *rep, void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!F) return CHOL_ERR_BAD_HANDLE;
  const int64_t n = F->n;
  if (A && lda < (n > 1 ? n : 1)) return -3;
  if (!A && (!Xf || d < 1 || ldxf < d || !(lengthscale > 0.0))) return -4;
  if (nrhs > 0 && (!B || !X)) return -10;
  if (ldb < (n > 1 ? n : 1)) return -11;
  if (ldxs < (n > 1 ? n : 1)) return -13;
  if (nrhs < 0) return -14;
  if (!(tol > 0.0)) return -15;
  if (max_iter < 0) return -16;
  if (method != CHOL_REFINE_IR && method != CHOL_REFINE_PCG) return -17;
  if (ws_bytes < chol_refine_bytes(n, nrhs, method) || (!workspace && nrhs > 0) ||
      ((uintptr_t)workspace & 7))
    return CHOL_ERR_WORKSPACE;
  if (F->info < 0) {
    int64_t inf;
    int rc = chol_get_info(F, &inf);
    if (rc) return rc;
  }
  if (F->info > 0) return CHOL_ERR_NOT_SPD;
  if (rep) memset(rep, 0, sizeof(*rep));
  if (n == 0 || nrhs == 0) {
    if (rep) rep->converged = 1, rep->fallback_used = F->fallback;
    return CHOL_OK;
  }
  Refiner R{};
  R.F = F;
  R.A = A;
  R.lda = lda;
  R.Xf = Xf;
  R.d = d;
  R.ldxf = ldxf;
  R.two_l2 = 2.0 * lengthscale * lengthscale;
  R.var = variance;
  R.noise = noise;
  R.B = B;
  R.ldb = ldb;
  R.X = X;
  R.ldx = ldxs;
  R.n = n;
  R.k = nrhs;
  R.tol = tol;
  R.lam = noise;
  R.certify = noise > 0.0;
  R.s = (hipStream_t)stream;
  R.setup(workspace);
  if (!R.certify) {
    // ||b|| for the relative-residual test of PCG without an eigenvalue bound
    launch_col_dot(B, ldb, B, ldb, n, nrhs, R.bb, R.partial, R.s);
    if (!R.ok(hipMemcpyAsync(R.h_bb.data(), R.bb, nrhs * sizeof(double), hipMemcpyDeviceToHost,
                             R.s)))
      return R.rc;
  }
  // x0 = M^{-1} b
  launch_copy(B, ldb, X, ldxs, n, nrhs, R.s);
  R.msolve(X);
  if (R.rc) return R.rc;
  if (method == CHOL_REFINE_IR) {
    if (R.run_ir(max_iter) && R.rc == CHOL_OK) {
      R.fallback |= CHOL_FALLBACK_PCG;
      R.run_pcg(max_iter, g_opt.pcg_recompute.load());
    }
  } else {
    R.run_pcg(max_iter, g_opt.pcg_recompute.load());
  }
  if (R.rc) return R.rc;
  HIP_OK(hipStreamSynchronize(R.s));
  bool conv = true;
  double cert_max = 0.0;
  for (int64_t c = 0; c < nrhs; ++c) {
    conv = conv && R.passes(c);
    cert_max = std::fmax(cert_max, R.cert[c]);
  }
  double res_max = 0.0;
  for (int64_t c = 0; c < nrhs; ++c) res_max = std::fmax(res_max, std::sqrt(R.h_nrm[c]));
  if (rep) {
    rep->iters = R.iters;
    rep->converged = conv ? 1 : 0;
    rep->cert = cert_max;
    rep->resid_norm = res_max;
    rep->fallback_used = F->fallback | R.fallback;
    rep->time_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return conv ? CHOL_OK : CHOL_ERR_NOT_CONVERGED;
}

// ------------------------------------------- refinement without allocation ----
// A file-scope device array replaces the caller's workspace.  In host code
// `scratch` names a host-side stand-in, not device memory: its device address
// is looked up once per device with hipGetSymbolAddress (on the first call
// on that device, with the device current) and only that address is passed
// to the kernels.  Every buffer in it is written before it is read, so
// nothing needs clearing between calls.
}  // extern "C"

namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::vector<std::pair<int, void *>> g_scratch;  // (device, device address of scratch)

int scratch_address(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CHOL_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  for (const auto &e : g_scratch)
    if (e.first == dev) {
      *out = e.second;
      return CHOL_OK;
    }
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CHOL_ERR_HIP;
  g_scratch.emplace_back(dev, p);
  *out = p;
  return CHOL_OK;
}
}  // namespace

extern "C" {

size_t chol_refine_noalloc_max_bytes(void) { return kScratchBytes; }

int chol_refine_solve_noalloc(chol_handle F, const double *A, int64_t lda, const double *Xf,
                              int64_t d, int64_t ldxf, double lengthscale, double variance,
                              double noise, const double *B, int64_t ldb, double *X,
                              int64_t ldxs, int64_t nrhs, double tol, int max_iter, int method,
                              chol_refine_report *rep, void *stream) {
  if (!F) return CHOL_ERR_BAD_HANDLE;
  if (nrhs < 0) return -14;
  if (method != CHOL_REFINE_IR && method != CHOL_REFINE_PCG) return -17;
  if (chol_refine_bytes(F->n, nrhs, method) > kScratchBytes) return CHOL_ERR_WORKSPACE;
  void *ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc) return rc;
  return chol_refine_solve(F, A, lda, Xf, d, ldxf, lengthscale, variance, noise, B, ldb, X, ldxs,
                           nrhs, tol, max_iter, method, ws, kScratchBytes, rep, stream);
}

}  // extern "C"
