// Heterogeneous CPU + GPU conjugate gradients (the paper's heterogeneous CG:
// Implementation, "CG implementation"; Results, its workload distribution
// and heterogeneous-vs-homogeneous comparison).
//
// The packed lower-tile matrix is split horizontally at tile row S: the GPU
// owns block rows [0, S), the CPU block rows [S, N), and every vector is
// split at the same row.  The GPU streams the tiles of its leading S x S
// triangle; the CPU streams every tile of its rows, i.e. its own triangle
// and the rectangle left of it, whose transposed products belong to the
// GPU's rows: the CPU sends them over as one vector per product (its
// column sums), so that each side reads only its own tiles.  Per iteration
// (one right-hand side, the paper's algorithm step by step):
//   t = A s              both sides, their rows (the CPU's rectangle
//                        products for the GPU's rows go host -> device);
//   s.t                  a partial sum per block row on each side; the host
//                        gathers them (device -> host), completes the
//                        device's copy (host -> device) and forms alpha in
//                        the device's summation order, so both agree bitwise;
//   x += alpha s, r -= alpha t (or the true residual every `recompute`
//                        iterations, which first exchanges x);
//   r.r                  gathered the same way, beta = r.r / previous;
//   s = r + beta s       both sides, then the two halves of s are exchanged.
// The split is chosen from gpu_share, the fraction of the stored tiles in
// the GPU's triangle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/chol.h"
#include "host_tiles.hpp"
#include "internal.hpp"

using namespace chol;

namespace {

constexpr int B = 128;
constexpr int64_t TE = (int64_t)B * B;
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// GPU block rows for a share of the stored tiles: the largest S with
// S (S + 1) / 2 <= share N (N + 1) / 2.
int64_t gpu_rows(int64_t N, double share) {
  const double want = share * (double)N * (N + 1) / 2.0;
  int64_t S = (int64_t)std::floor((std::sqrt(8.0 * want + 1.0) - 1.0) / 2.0);
  while (S > 0 && (double)S * (S + 1) / 2.0 > want) --S;
  while (S < N && (double)(S + 1) * (S + 2) / 2.0 <= want) ++S;
  return std::min(S, N);
}

// Device workspace: packed tiles, partials, vectors x r s t b and the
// rectangle products for the GPU rows (n_pad each), per-row partial dots,
// scalars.
struct DevLayout {
  size_t tiles, part, vec, extra, pdot, prr, scal, total;
};
DevLayout dev_layout(int64_t n) {
  const int64_t N = (n + B - 1) / B, n_pad = N * B;
  DevLayout L{};
  size_t off = 0;
  L.tiles = off;
  off = align_up(off + (size_t)tile_count(N) * TE * sizeof(double));
  L.part = off;
  off = align_up(off + (size_t)tile_count(N) * 2 * B * sizeof(double));
  L.vec = off;
  off = align_up(off + (size_t)5 * n_pad * sizeof(double));
  L.extra = off;
  off = align_up(off + (size_t)n_pad * sizeof(double));
  L.pdot = off;
  off = align_up(off + (size_t)N * sizeof(double));
  L.prr = off;
  off = align_up(off + (size_t)N * sizeof(double));
  L.scal = off;
  off = align_up(off + 3 * CG_MAX_RHS * sizeof(double) + 3 * CG_MAX_RHS * sizeof(int));
  L.total = off;
  return L;
}

// Host workspace: the CPU's tiles (column c: rows [max(c, S), N), columns
// one after another), their row products (one block-row vector per tile),
// the column sums, and the vectors x r s t b y (n_pad each), pdot, prr.
struct HostLayout {
  int64_t S, ntiles;
  std::vector<int64_t> col_off;  // tile offset of column c
  size_t tiles, p0, side1, vec, dots, total;
};
HostLayout host_layout(int64_t n, double share) {
  const int64_t N = (n + B - 1) / B, n_pad = N * B;
  HostLayout L{};
  L.S = gpu_rows(N, share);
  L.col_off.resize(N + 1);
  int64_t t = 0;
  for (int64_t c = 0; c < N; ++c) {
    L.col_off[c] = t;
    t += N - std::max(c, L.S);
  }
  L.col_off[N] = t;
  L.ntiles = t;
  size_t off = 0;
  L.tiles = off;
  off = align_up(off + (size_t)t * TE * sizeof(double));
  L.p0 = off;
  off = align_up(off + (size_t)t * B * sizeof(double));
  L.side1 = off;
  off = align_up(off + (size_t)n_pad * sizeof(double));
  L.vec = off;
  off = align_up(off + (size_t)6 * n_pad * sizeof(double));
  L.dots = off;
  off = align_up(off + (size_t)2 * N * sizeof(double));
  L.total = off;
  return L;
}

// The device's order of summing per-row partials (strided partial sums over
// B threads, then a tree), so that host and device form the same scalars.
double device_order_sum(const double *p, int64_t N) {
  double sh[B];
  for (int t = 0; t < B; ++t) {
    double acc = 0.0;
    for (int64_t e = t; e < N; e += B) acc += p[e];
    sh[t] = acc;
  }
  for (int m = B / 2; m >= 1; m >>= 1)
    for (int t = 0; t < m; ++t) sh[t] += sh[t + m];
  return sh[0];
}

struct HetCg {
  int64_t n, N, n_pad, S;
  HostLayout HL;
  DevLayout DL;
  char *hw;  // host workspace
  char *dw;  // device workspace
  hipStream_t s;
  hipEvent_t ev;
  int rc = CHOL_OK;
  cg_hetero_report rep{};
  // host views
  double *ht, *hp0, *hside1, *hx, *hr, *hs, *htt, *hb, *hy, *hpdot, *hprr;
  // device views
  double *dtiles, *dpart, *dx, *dr, *ds, *dt, *db, *dextra, *dpdot, *dprr, *du, *du0;
  int *dact, *dits;

  bool ok(hipError_t e) {
    if (e != hipSuccess && rc == CHOL_OK) rc = CHOL_ERR_HIP;
    return rc == CHOL_OK;
  }
  void setup() {
    ht = (double *)(hw + HL.tiles);
    hp0 = (double *)(hw + HL.p0);
    hside1 = (double *)(hw + HL.side1);
    double *v = (double *)(hw + HL.vec);
    hx = v;
    hr = v + n_pad;
    hs = v + 2 * n_pad;
    htt = v + 3 * n_pad;
    hb = v + 4 * n_pad;
    hy = v + 5 * n_pad;
    hpdot = (double *)(hw + HL.dots);
    hprr = hpdot + N;
    dtiles = (double *)(dw + DL.tiles);
    dpart = (double *)(dw + DL.part);
    double *dv = (double *)(dw + DL.vec);
    dx = dv;
    dr = dv + n_pad;
    ds = dv + 2 * n_pad;
    dt = dv + 3 * n_pad;
    db = dv + 4 * n_pad;
    dextra = (double *)(dw + DL.extra);
    dpdot = (double *)(dw + DL.pdot);
    dprr = (double *)(dw + DL.prr);
    du = (double *)(dw + DL.scal);
    du0 = du + 2 * CG_MAX_RHS;
    dact = (int *)(du0 + CG_MAX_RHS);
    dits = dact + 2 * CG_MAX_RHS;
  }
  double *htile(int64_t i, int64_t c) {
    return ht + (HL.col_off[c] + (i - std::max(c, S))) * TE;
  }
  double *hp0of(int64_t i, int64_t c) { return hp0 + (HL.col_off[c] + (i - std::max(c, S))) * B; }

  // y = A v on the CPU's tiles: hy holds rows [S, N) of A v (from the CPU's
  // tiles, which are all of those rows' tiles), and rows [0, S) the
  // rectangle's transposed products (the part the GPU's tiles miss).
  void cpu_matvec(const double *v) {
    const auto t0 = clk::now();
    // column tasks: both products of every CPU tile in column c
    host::parallel_for(N, [&](int64_t c) {
      double *sc = hside1 + c * B;
      for (int r = 0; r < B; ++r) sc[r] = 0.0;
      for (int64_t i = std::max(c, S); i < N; ++i)
        host::tile_symv_pair(htile(i, c), v + c * B, v + i * B, hp0of(i, c), sc, i == c);
    });
    // row sums of the CPU rows: side-0 products of tiles (i, c), c <= i, in
    // column order, then the side-1 sum of column i
    host::parallel_for(N - S, [&](int64_t q) {
      const int64_t i = S + q;
      double *y = hy + i * B;
      for (int r = 0; r < B; ++r) y[r] = 0.0;
      for (int64_t c = 0; c <= i; ++c) {
        const double *p = hp0of(i, c);
        for (int r = 0; r < B; ++r) y[r] += p[r];
      }
      const double *sc = hside1 + i * B;
      for (int r = 0; r < B; ++r) y[r] += sc[r];
    });
    // the GPU rows' share: column sums of the rectangle
    std::memcpy(hy, hside1, (size_t)S * B * sizeof(double));
    rep.ms_cpu += ms_since(t0);
  }
  // per-block-row dots on the CPU rows into out[S .. N)
  void cpu_dots(const double *a, const double *b, double *out) {
    host::parallel_for(N - S, [&](int64_t q) {
      const int64_t i = S + q;
      double d = 0.0;
      for (int r = 0; r < B; ++r) d += a[i * B + r] * b[i * B + r];
      out[i] = d;
    });
  }
  void h2d(double *dst, const double *src, int64_t count) {
    if (count <= 0) return;
    ok(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyHostToDevice, s));
    rep.bytes_h2d += (double)count * sizeof(double);
  }
  void d2h(double *dst, const double *src, int64_t count) {
    if (count <= 0) return;
    ok(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToHost, s));
    rep.bytes_d2h += (double)count * sizeof(double);
  }
  void wait() {
    const auto t0 = clk::now();
    ok(hipEventRecord(ev, s));
    ok(hipEventSynchronize(ev));
    rep.ms_wait_gpu += ms_since(t0);
  }
  // A v on both sides: the GPU's tile products are enqueued first, so that
  // they run while the CPU computes its rows; then the rectangle products go
  // to the device and its rows are reduced in `mode`
  void matvec(const double *dv, const double *v, int mode, int act_slot) {
    launch_cg_symv(dtiles, B, N, dv, n_pad, 1, dpart, s, S);
    cpu_matvec(v);
    h2d(dextra, hy, S * B);
    launch_cg_reduce(dpart, B, N, 1, mode, dt, ds, dr, db, n_pad, dact + act_slot * CG_MAX_RHS,
                     mode == CG_RED_T ? dpdot : dprr, s, S, dextra);
  }
};

}  // namespace

extern "C" {

size_t cg_hetero_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return dev_layout(n).total;
}

size_t cg_hetero_host_bytes(int64_t n, double gpu_share) {
  if (n < 0 || !(gpu_share >= 0.0 && gpu_share <= 1.0)) return 0;
  return host_layout(n, gpu_share).total;
}

int cg_solve_hetero(const double *A, int64_t n, int64_t lda, const double *Bv, double *X,
                    double eps, int64_t max_iter, int64_t recompute, double gpu_share,
                    void *workspace, size_t ws_bytes, void *host_ws, size_t host_bytes,
                    int64_t *iters, double *relres, cg_hetero_report *rep, void *stream) {
  const auto t0 = clk::now();
  if (n > 0 && !A) return -1;
  if (n < 0) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && (!Bv || !X)) return -4;
  if (!(eps >= 0.0) || !std::isfinite(eps)) return -6;
  if (max_iter < 0) return -7;
  if (recompute < 0) return -8;
  if (!(gpu_share >= 0.0 && gpu_share <= 1.0)) return -9;
  if (n > 0 && (!workspace || ((uintptr_t)workspace % kAlign) != 0)) return -10;
  if (ws_bytes < cg_hetero_workspace_bytes(n)) return CHOL_ERR_WORKSPACE;
  if (n > 0 && (!host_ws || host_bytes < cg_hetero_host_bytes(n, gpu_share))) return -12;
  if (n == 0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return CHOL_OK;
  }
  HetCg H{};
  H.n = n;
  H.N = (n + B - 1) / B;
  H.n_pad = H.N * B;
  H.HL = host_layout(n, gpu_share);
  H.DL = dev_layout(n);
  H.S = H.HL.S;
  H.hw = (char *)host_ws;
  H.dw = (char *)workspace;
  H.s = (hipStream_t)stream;
  H.setup();
  if (hipEventCreateWithFlags(&H.ev, hipEventDisableTiming) != hipSuccess) return CHOL_ERR_HIP;
  const int64_t N = H.N, S = H.S, np = H.n_pad, SB = S * B;
  const double eps2 = eps * eps;
  hipStream_t s = H.s;
  H.rep.gpu_share_target = gpu_share;
  H.rep.gpu_rows = (int32_t)S;
  H.rep.cpu_threads = host::threads();
  H.rep.gpu_share_tiles = (double)tile_count(S) / (double)tile_count(N);

  // set-up: packed tiles on the device, the CPU's tiles copied to the host
  // (one copy per tile column), x and b on both sides
  launch_pack(A, n, lda, H.dtiles, STORE_F64, B, N, 1.0, s);
  launch_cg_copy_in(X, n, n, np, 1, H.dx, np, s);
  launch_cg_copy_in(Bv, n, n, np, 1, H.db, np, s);
  for (int64_t c = 0; c < N; ++c) {
    const int64_t r0 = std::max(c, S);
    if (r0 >= N) continue;
    const size_t bytes = (size_t)(N - r0) * TE * sizeof(double);
    H.ok(hipMemcpyAsync(H.htile(r0, c), H.dtiles + tile_index(r0, c, N) * TE, bytes,
                        hipMemcpyDeviceToHost, s));
    H.rep.bytes_d2h += (double)bytes;
  }
  H.d2h(H.hx, H.dx, np);
  H.d2h(H.hb, H.db, np);
  H.wait();

  // r = s = b - A x; u = u0 = r.r
  H.matvec(H.dx, H.hx, CG_RED_INIT, 0);
  for (int64_t e = SB; e < np; ++e) H.hr[e] = H.hs[e] = H.hb[e] - H.hy[e];
  H.cpu_dots(H.hr, H.hr, H.hprr);
  H.h2d(H.dprr + S, H.hprr + S, N - S);
  launch_cg_init(B, N, 1, H.dprr, H.du, H.du0, H.dact, H.dits, eps2, s);
  H.d2h(H.hprr, H.dprr, S);
  H.d2h(H.hs, H.ds, SB);
  H.h2d(H.ds + SB, H.hs + SB, np - SB);
  H.wait();
  double u = device_order_sum(H.hprr, N);
  const double u0 = u;
  bool active = u > eps2 * u0;
  int64_t it = 0;
  for (; it < max_iter && active && H.rc == CHOL_OK; ++it) {
    const int p = (int)(it & 1), q = 1 - p;
    const bool rec = recompute > 0 && (it + 1) % recompute == 0;
    // t = A s, s.t
    H.matvec(H.ds, H.hs, CG_RED_T, p);
    H.d2h(H.hpdot, H.dpdot, S);
    for (int64_t e = SB; e < np; ++e) H.htt[e] = H.hy[e];
    H.cpu_dots(H.hs, H.htt, H.hpdot);
    H.h2d(H.dpdot + S, H.hpdot + S, N - S);
    H.wait();
    const double alpha = u / device_order_sum(H.hpdot, N);
    // x += alpha s; r -= alpha t (or the true residual)
    launch_cg_xr(B, N, 1, H.dpdot, H.du + p * CG_MAX_RHS, H.dact + p * CG_MAX_RHS, H.dx, H.dr,
                 H.ds, H.dt, np, rec ? 1 : 0, H.dprr, s, S);
    for (int64_t e = SB; e < np; ++e) {
      H.hx[e] = std::fma(alpha, H.hs[e], H.hx[e]);
      if (!rec) H.hr[e] = std::fma(-alpha, H.htt[e], H.hr[e]);
    }
    if (rec) {
      // the true residual: both halves of x on both sides first
      H.d2h(H.hx, H.dx, SB);
      H.h2d(H.dx + SB, H.hx + SB, np - SB);
      H.wait();
      H.matvec(H.dx, H.hx, CG_RED_RESID, p);
      for (int64_t e = SB; e < np; ++e) H.hr[e] = H.hb[e] - H.hy[e];
      ++H.rep.recomputations;
    }
    H.cpu_dots(H.hr, H.hr, H.hprr);
    H.h2d(H.dprr + S, H.hprr + S, N - S);
    H.d2h(H.hprr, H.dprr, S);
    H.wait();
    const double un = device_order_sum(H.hprr, N);
    // s = r + beta s, then the halves of s change sides
    launch_cg_s(B, N, 1, H.dprr, H.du + p * CG_MAX_RHS, H.dact + p * CG_MAX_RHS,
                H.du + q * CG_MAX_RHS, H.dact + q * CG_MAX_RHS, H.du0, eps2, H.dits, H.dr, H.ds, np,
                s, S);
    const double beta = un / u;
    for (int64_t e = SB; e < np; ++e) H.hs[e] = std::fma(beta, H.hs[e], H.hr[e]);
    u = un;
    active = un > eps2 * u0;
    H.d2h(H.hs, H.ds, SB);
    H.h2d(H.ds + SB, H.hs + SB, np - SB);
    H.wait();
  }
  // x: the GPU's rows are on the device, the CPU's on the host
  H.h2d(H.dx + SB, H.hx + SB, np - SB);
  launch_cg_copy_out(H.dx, np, n, 1, X, n, s);
  H.wait();
  (void)hipEventDestroy(H.ev);
  if (H.rc != CHOL_OK) return H.rc;
  if (iters) *iters = it;
  if (relres) *relres = u0 > 0.0 ? std::sqrt(u / u0) : 0.0;
  if (rep) {
    H.rep.iterations = (int32_t)it;
    H.rep.ms_total = ms_since(t0);
    *rep = H.rep;
  }
  return active ? CHOL_ERR_NOT_CONVERGED : CHOL_OK;
}

}  // extern "C"
