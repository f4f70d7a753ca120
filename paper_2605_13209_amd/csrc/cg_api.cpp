// C ABI of the conjugate gradient solver (cg_workspace_bytes, cg_solve):
// argument checks, the workspace layout and the host loop that enqueues the
// iterations.  The arithmetic runs in the kernels of cg.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/chol.h"
#include "internal.hpp"

using namespace chol;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace regions, in order (each 256-byte aligned).
struct CgLayout {
  size_t tiles, part, vec, pdot, prr, scal, total;
};

CgLayout cg_layout(int64_t n, int b, int64_t K) {
  const int64_t N = (n + b - 1) / b, n_pad = N * b;
  CgLayout L{};
  size_t off = 0;
  L.tiles = off;
  off = align_up(off + (size_t)tile_count(N) * b * b * sizeof(double));
  L.part = off;
  off = align_up(off + (size_t)tile_count(N) * 2 * K * b * sizeof(double));
  L.vec = off;  // x, r, s, t, b: n_pad x K each
  off = align_up(off + (size_t)5 * n_pad * K * sizeof(double));
  L.pdot = off;
  off = align_up(off + (size_t)N * K * sizeof(double));
  L.prr = off;
  off = align_up(off + (size_t)N * K * sizeof(double));
  L.scal = off;  // u[2][16], u0[16] doubles; act[2][16], iters[16] ints
  off = align_up(off + 3 * CG_MAX_RHS * sizeof(double) + 3 * CG_MAX_RHS * sizeof(int));
  L.total = off;
  return L;
}

// Pinned host words the stopping flags are copied to (one slot per step
// parity) and two events, per (device, caller stream), kept for the process.
struct CgCtx {
  int device = -1;
  hipStream_t caller = nullptr;
  int *flags = nullptr;  // 2 * CG_MAX_RHS ints, pinned host memory
  hipEvent_t ev[2] = {nullptr, nullptr};
};
std::mutex g_cg_mu;
std::vector<CgCtx *> g_cg_ctx;

int cg_ctx(hipStream_t caller, CgCtx **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CHOL_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_cg_mu);
  for (CgCtx *c : g_cg_ctx)
    if (c->device == dev && c->caller == caller) {
      *out = c;
      return CHOL_OK;
    }
  CgCtx *c = new CgCtx();
  c->device = dev;
  c->caller = caller;
  if (hipHostMalloc((void **)&c->flags, 2 * CG_MAX_RHS * sizeof(int), hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return CHOL_ERR_HIP;
  }
  if (hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess) {
    for (hipEvent_t e : c->ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipHostFree(c->flags);
    delete c;
    return CHOL_ERR_HIP;
  }
  g_cg_ctx.push_back(c);
  *out = c;
  return CHOL_OK;
}

// The tile product, bracketed by events when profiling; its algorithmic
// work is the packed triangle's bytes (each stored tile read once).
void symv(const double *tiles, int b, int64_t N, const double *v, int64_t ld, int K, double *part,
          hipStream_t s) {
  if (!profile_option()) {
    launch_cg_symv(tiles, b, N, v, ld, K, part, s);
    return;
  }
  hipEvent_t a = profile_begin(s);
  launch_cg_symv(tiles, b, N, v, ld, K, part, s);
  profile_end(s, a, (double)tile_count(N) * b * b * sizeof(double));
}

#define CG_HIP(x)                                \
  do {                                           \
    if ((x) != hipSuccess) return CHOL_ERR_HIP;  \
  } while (0)

}  // namespace

extern "C" {

size_t cg_workspace_bytes(int64_t n, int tile, int64_t nrhs) {
  if (n < 0 || nrhs < 1 || nrhs > CG_MAX_RHS) return 0;
  if (tile == 0) tile = 128;
  if (tile != 64 && tile != 128) return 0;
  return cg_layout(n, tile, nrhs).total;
}

int cg_solve(const double *A, int64_t n, int64_t lda, int tile, const double *B, int64_t ldb,
             double *X, int64_t ldx, int64_t nrhs, double eps, int64_t max_iter,
             int64_t recompute, void *workspace, size_t ws_bytes, int64_t *iters,
             double *relres, void *stream) {
  if (n > 0 && !A) return -1;
  if (n < 0) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (tile == 0) tile = 128;
  if (tile != 64 && tile != 128) return CHOL_ERR_UNSUPPORTED;
  if (n > 0 && !B) return -5;
  if (ldb < (n > 1 ? n : 1)) return -6;
  if (n > 0 && !X) return -7;
  if (ldx < (n > 1 ? n : 1)) return -8;
  if (nrhs < 1 || nrhs > CG_MAX_RHS) return -9;
  if (!(eps >= 0.0) || !std::isfinite(eps)) return -10;
  if (max_iter < 0) return -11;
  if (recompute < 0) return -12;
  if (n > 0 && (!workspace || ((uintptr_t)workspace % kAlign) != 0)) return -13;
  const int b = tile;
  const int K = (int)nrhs;
  const CgLayout L = cg_layout(n, b, K);
  if (ws_bytes < L.total) return CHOL_ERR_WORKSPACE;
  if (n == 0) {
    for (int k = 0; k < K; ++k) {
      if (iters) iters[k] = 0;
      if (relres) relres[k] = 0.0;
    }
    return CHOL_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  CgCtx *ctx = nullptr;
  {
    const int rc = cg_ctx(s, &ctx);
    if (rc != CHOL_OK) return rc;
  }
  const int64_t N = (n + b - 1) / b, n_pad = N * b, ld = n_pad;
  char *ws = (char *)workspace;
  double *tiles = (double *)(ws + L.tiles);
  double *part = (double *)(ws + L.part);
  double *vx = (double *)(ws + L.vec);
  double *vr = vx + n_pad * K;
  double *vs = vr + n_pad * K;
  double *vt = vs + n_pad * K;
  double *vb = vt + n_pad * K;
  double *pdot = (double *)(ws + L.pdot);
  double *prr = (double *)(ws + L.prr);
  double *u = (double *)(ws + L.scal);        // u[2][CG_MAX_RHS]
  double *u0 = u + 2 * CG_MAX_RHS;            // u0[CG_MAX_RHS]
  int *act = (int *)(u0 + CG_MAX_RHS);        // act[2][CG_MAX_RHS]
  int *its = act + 2 * CG_MAX_RHS;            // iters[CG_MAX_RHS]
  const double eps2 = eps * eps;

  // set-up: packed tiles, padded copies of X and B, r = s = b - A x, u = u0
  launch_pack(A, n, lda, tiles, STORE_F64, b, N, 1.0, s);
  launch_cg_copy_in(X, ldx, n, n_pad, K, vx, ld, s);
  launch_cg_copy_in(B, ldb, n, n_pad, K, vb, ld, s);
  symv(tiles, b, N, vx, ld, K, part, s);
  launch_cg_reduce(part, b, N, K, CG_RED_INIT, nullptr, vs, vr, vb, ld, nullptr, prr, s);
  launch_cg_init(b, N, K, prr, u, u0, act, its, eps2, s);
  CG_HIP(hipGetLastError());

  // iterations: the host reads the flags of step it - 1 after enqueueing
  // step it, so the device always has the next step queued
  int64_t launched = 0;
  bool done = false;
  if (max_iter > 0) {
    CG_HIP(hipMemcpyAsync(ctx->flags + CG_MAX_RHS, act, K * sizeof(int), hipMemcpyDeviceToHost, s));
    CG_HIP(hipEventRecord(ctx->ev[1], s));
    CG_HIP(hipEventSynchronize(ctx->ev[1]));
    done = true;
    for (int k = 0; k < K; ++k) done = done && ctx->flags[CG_MAX_RHS + k] == 0;
  }
  for (int64_t it = 0; it < max_iter && !done; ++it) {
    const int p = (int)(it & 1), q = 1 - p;
    const int recompute_now = (recompute > 0 && (it + 1) % recompute == 0) ? 1 : 0;
    symv(tiles, b, N, vs, ld, K, part, s);
    launch_cg_reduce(part, b, N, K, CG_RED_T, vt, vs, nullptr, nullptr, ld, nullptr, pdot, s);
    launch_cg_xr(b, N, K, pdot, u + p * CG_MAX_RHS, act + p * CG_MAX_RHS, vx, vr, vs, vt, ld,
                 recompute_now, prr, s);
    if (recompute_now) {
      symv(tiles, b, N, vx, ld, K, part, s);
      launch_cg_reduce(part, b, N, K, CG_RED_RESID, nullptr, nullptr, vr, vb, ld,
                       act + p * CG_MAX_RHS, prr, s);
    }
    launch_cg_s(b, N, K, prr, u + p * CG_MAX_RHS, act + p * CG_MAX_RHS, u + q * CG_MAX_RHS,
                act + q * CG_MAX_RHS, u0, eps2, its, vr, vs, ld, s);
    CG_HIP(hipGetLastError());
    CG_HIP(hipMemcpyAsync(ctx->flags + q * CG_MAX_RHS, act + q * CG_MAX_RHS, K * sizeof(int),
                          hipMemcpyDeviceToHost, s));
    CG_HIP(hipEventRecord(ctx->ev[q], s));
    launched = it + 1;
    if (it >= 1) {
      // flags written by step it - 1 (slot p)
      CG_HIP(hipEventSynchronize(ctx->ev[p]));
      bool all = true;
      for (int k = 0; k < K; ++k) all = all && ctx->flags[p * CG_MAX_RHS + k] == 0;
      if (all) done = true;
    }
  }

  // results: X, iteration counts, sqrt(u / u0) from the last written slot
  launch_cg_copy_out(vx, ld, n, K, X, ldx, s);
  std::vector<double> hu(CG_MAX_RHS), hu0(CG_MAX_RHS);
  std::vector<int> hit(CG_MAX_RHS), hact(CG_MAX_RHS);
  const int last = (int)(launched & 1);
  CG_HIP(hipMemcpyAsync(hu.data(), u + last * CG_MAX_RHS, K * sizeof(double), hipMemcpyDeviceToHost,
                        s));
  CG_HIP(hipMemcpyAsync(hu0.data(), u0, K * sizeof(double), hipMemcpyDeviceToHost, s));
  CG_HIP(hipMemcpyAsync(hit.data(), its, K * sizeof(int), hipMemcpyDeviceToHost, s));
  CG_HIP(hipMemcpyAsync(hact.data(), act + last * CG_MAX_RHS, K * sizeof(int),
                        hipMemcpyDeviceToHost, s));
  CG_HIP(hipStreamSynchronize(s));
  int rc = CHOL_OK;
  for (int k = 0; k < K; ++k) {
    if (iters) iters[k] = hit[k];
    if (relres) relres[k] = hu0[k] > 0.0 ? std::sqrt(hu[k] / hu0[k]) : 0.0;
    if (hact[k] || !(hu[k] <= eps2 * hu0[k] || hu0[k] == 0.0)) rc = CHOL_ERR_NOT_CONVERGED;
  }
  return rc;
}

}  // extern "C"
