// Continuous-batching factorisation engine for the serving loop: many FP32
// factorisations (tile 128) advance together, one tile column per step.  A
// step is one batched diagonal-tile factorisation (a workgroup per job), one
// batched panel solve and one batched trailing update (the FP32 matrix-core
// kernel walking a flat list of every job's trailing triangle), described by
// a device descriptor that the host rewrites before each step; the three
// launches are captured once into a HIP graph and replayed.  Jobs join and
// leave between steps, so requests that arrive while others are being
// factored share the next launches.  A job's tiles receive the same
// operations in the same order whatever else is in the batch, so its factor
// is bitwise the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/chol.h"
#include "factor_handle.hpp"
#include "internal.hpp"

using namespace chol;

namespace {
constexpr int B = 128;
constexpr int kTrsmGrid = 1024;
constexpr int kUpdGrid = 2048;
constexpr int kSuper = 8;

struct Job {
  chol_factor_s *F = nullptr;
  int64_t c = 0;  // next tile column
  bool done = false, taken = false;  // a taken slot is free for a new job
};
}  // namespace

struct chol_batch_s {
  int max_jobs = 0;
  BatchDesc *d_desc = nullptr;            // device (caller memory)
  std::vector<std::vector<char>> h_desc;  // two host staging copies
  hipEvent_t ev_copy[2] = {nullptr, nullptr};
  bool copy_pending[2] = {false, false};
  uint64_t steps = 0;
  hipStream_t stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int use_graph = 1;
  std::vector<Job> jobs;  // slot per job id
  std::mutex mu;
  ~chol_batch_s() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (hipEvent_t e : ev_copy)
      if (e) (void)hipEventDestroy(e);
    for (Job &j : jobs)
      if (!j.taken) delete j.F;
  }
};

namespace {
void enqueue_step(chol_batch_s *b, hipStream_t s) {
  launch_batch_potrf_trsm(b->d_desc, b->max_jobs, kTrsmGrid, s);
  launch_batch_update(b->d_desc, kUpdGrid, kSuper, s);
}
}  // namespace

extern "C" {

size_t chol_batch_desc_bytes(int max_jobs) {
  if (max_jobs < 1 || max_jobs > 1024) return 0;
  return batch_desc_bytes(max_jobs);
}

int chol_batch_create(int max_jobs, void *desc, size_t desc_bytes, int use_graph, void *stream,
                      chol_batch *out) {
  if (max_jobs < 1 || max_jobs > 1024) return -1;
  if (!desc || ((uintptr_t)desc & 255)) return -2;
  if (desc_bytes < batch_desc_bytes(max_jobs)) return CHOL_ERR_WORKSPACE;
  if (!out) return -6;
  if (use_graph && !stream) return -5;  // capture needs a created stream
  chol_batch_s *b = new chol_batch_s();
  b->max_jobs = max_jobs;
  b->d_desc = (BatchDesc *)desc;
  b->stream = (hipStream_t)stream;
  b->use_graph = use_graph ? 1 : 0;
  b->h_desc.assign(2, std::vector<char>(batch_desc_bytes(max_jobs), 0));
  for (hipEvent_t &e : b->ev_copy)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      delete b;
      return CHOL_ERR_HIP;
    }
  *out = b;
  return CHOL_OK;
}

void chol_batch_destroy(chol_batch b) { delete b; }

int chol_batch_add(chol_batch b, const double *A, int64_t n, int64_t lda, void *workspace,
                   size_t ws_bytes, int64_t *job) {
  if (!b) return CHOL_ERR_BAD_HANDLE;
  if (n > 0 && !A) return -2;
  if (n < 1) return -3;
  if (lda < n) return -4;
  if (!workspace || ((uintptr_t)workspace & 255)) return -5;
  if (ws_bytes < chol_factor_bytes(n, CHOL_FP32, B)) return CHOL_ERR_WORKSPACE;
  if (!job) return -7;
  std::lock_guard<std::mutex> lk(b->mu);
  int active = 0;
  for (const Job &j : b->jobs) active += !j.done && !j.taken;
  if (active >= b->max_jobs) return CHOL_ERR_WORKSPACE;
  chol_factor_s *F = new chol_factor_s();
  F->n = n;
  F->b = B;
  F->N = (n + B - 1) / B;
  F->precision = CHOL_FP32;
  (void)hipGetDevice(&F->device);
  F->d_info = (int64_t *)workspace;
  F->sync = (int *)((char *)workspace + kSolveSyncOff);
  F->tiles = (char *)workspace + kHeader;
  F->dinv = (char *)F->tiles + (size_t)tile_count(F->N) * B * B * sizeof(float);
  F->stream = b->stream;
  if (hipEventCreateWithFlags(&F->ev_solve, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&F->ev_ready, hipEventDisableTiming) != hipSuccess) {
    delete F;
    return CHOL_ERR_HIP;
  }
  // cleared info and packed tiles, ordered before the job's first step
  launch_clear_i64(F->d_info, 1, b->stream);
  launch_pack(A, n, lda, F->tiles, STORE_F32, B, F->N, 1.0, b->stream);
  if (hipGetLastError() != hipSuccess) {
    delete F;
    return CHOL_ERR_HIP;
  }
  Job j;
  j.F = F;
  size_t slot = 0;
  while (slot < b->jobs.size() && !b->jobs[slot].taken) ++slot;
  if (slot == b->jobs.size())
    b->jobs.push_back(j);
  else
    b->jobs[slot] = j;
  *job = (int64_t)slot;
  return CHOL_OK;
}

int chol_batch_step(chol_batch b, int *active_out, int *finished_out) {
  if (!b) return CHOL_ERR_BAD_HANDLE;
  std::lock_guard<std::mutex> lk(b->mu);
  hipStream_t s = b->stream;
  const int slot = (int)(b->steps & 1);
  if (b->copy_pending[slot]) {
    // the host copy used two steps ago must have reached the device
    if (hipEventSynchronize(b->ev_copy[slot]) != hipSuccess) return CHOL_ERR_HIP;
    b->copy_pending[slot] = false;
  }
  BatchDesc *h = (BatchDesc *)b->h_desc[slot].data();
  int64_t nj = 0, tp = 0, up = 0;
  std::vector<size_t> in_step;
  for (size_t id = 0; id < b->jobs.size(); ++id) {
    Job &j = b->jobs[id];
    if (j.done || j.taken) continue;
    BatchJob &J = h->jobs[nj++];
    J.tiles = j.F->tiles;
    J.info = j.F->d_info;
    J.N = j.F->N;
    J.c = j.c;
    J.trsm_begin = tp;
    J.upd_begin = up;
    const int64_t R = j.F->N - j.c - 1;
    tp += R;
    up += R * (R + 1) / 2;
    in_step.push_back(id);
  }
  if (active_out) *active_out = (int)nj;
  if (finished_out) *finished_out = 0;
  if (nj == 0) return CHOL_OK;
  h->njobs = nj;
  h->trsm_total = tp;
  h->upd_total = up;
  if (hipMemcpyAsync(b->d_desc, h, batch_desc_bytes((int)nj), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipEventRecord(b->ev_copy[slot], s) != hipSuccess)
    return CHOL_ERR_HIP;
  b->copy_pending[slot] = true;
  if (b->use_graph) {
    if (!b->graph) {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return CHOL_ERR_HIP;
      enqueue_step(b, s);
      if (hipStreamEndCapture(s, &g) != hipSuccess) return CHOL_ERR_HIP;
      const hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        b->graph = nullptr;
        return CHOL_ERR_HIP;
      }
    }
    if (hipGraphLaunch(b->graph, s) != hipSuccess) return CHOL_ERR_HIP;
  } else {
    enqueue_step(b, s);
    if (hipGetLastError() != hipSuccess) return CHOL_ERR_HIP;
  }
  ++b->steps;
  int fin = 0;
  for (size_t id : in_step) {
    Job &j = b->jobs[id];
    if (++j.c == j.F->N) {
      j.done = true;
      ++fin;
      launch_diag_inverse(j.F->tiles, STORE_F32, B, j.F->N, j.F->dinv, j.F->d_info, s);
      if (hipEventRecord(j.F->ev_ready, s) != hipSuccess) return CHOL_ERR_HIP;
    }
  }
  if (finished_out) *finished_out = fin;
  return hipGetLastError() == hipSuccess ? CHOL_OK : CHOL_ERR_HIP;
}

int chol_batch_status(chol_batch b, int64_t job, int *done) {
  if (!b) return CHOL_ERR_BAD_HANDLE;
  std::lock_guard<std::mutex> lk(b->mu);
  if (job < 0 || job >= (int64_t)b->jobs.size() || b->jobs[job].taken) return -2;
  if (done) *done = b->jobs[job].done ? 1 : 0;
  return CHOL_OK;
}

int chol_batch_take(chol_batch b, int64_t job, chol_handle *F) {
  if (!b) return CHOL_ERR_BAD_HANDLE;
  if (!F) return -3;
  std::lock_guard<std::mutex> lk(b->mu);
  if (job < 0 || job >= (int64_t)b->jobs.size() || b->jobs[job].taken) return -2;
  Job &j = b->jobs[job];
  if (!j.done) return CHOL_ERR_NOT_CONVERGED;
  j.taken = true;
  *F = j.F;
  return CHOL_OK;
}

}  // extern "C"
