// The host handle of a factorisation (chol_handle) and the layout of the
// factor workspace, shared by the drivers (chol_api.cpp, hetero.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>

namespace chol {
// Start of the factor workspace: the info word (offset 0), the largest
// diagonal entry for the FP16 form's scaling (offset 64), and the solves'
// synchronisation words (offset kSolveSyncOff, kSolveSyncWords ints: an
// abort word and per-chunk progress counters, cleared by a kernel before
// every solve).
constexpr size_t kHeader = 512;
constexpr size_t kSolveSyncOff = 256;
constexpr int64_t kSolveSyncWords = 64;
}  // namespace chol

struct chol_factor_s {
  int64_t n = 0, N = 0;
  int b = 0, precision = 0, device = 0;
  void *tiles = nullptr;
  void *dinv = nullptr;  // inverted diagonal blocks L_cc^{-T} (the solves)
  void *p16 = nullptr;   // CHOL_FP16_SCALED: two FP16 panel buffers (alternating panels)
  int64_t *d_info = nullptr;
  int *sync = nullptr;   // the solves' synchronisation words (workspace header)
  double scale = 1.0;  // CHOL_FP16_SCALED: the factor of A / scale (+ shift I) is stored
  double shift = 0.0;  // CHOL_FP16_SCALED retry: diagonal shift added to A / scale
  int fallback = 0;    // CHOL_FALLBACK_SHIFT / CHOL_FALLBACK_FP32 taken by chol_factor
  hipStream_t stream = nullptr;
  int64_t info = -1;  // host copy once known
  // Solves share the synchronisation words: a solve on another stream than
  // the previous one waits for it (event recorded after every solve).
  // The mutex makes that check, the launches and the record one step when
  // several host threads solve with the handle.
  std::mutex solve_mu;
  hipEvent_t ev_solve = nullptr;
  hipStream_t last_solve = nullptr;
  bool solved = false;
  int inpanel = 0;            // in-panel updates: 0 right-looking, 1 left-looking, 2 recursive
  bool potrf_la = false;      // diagonal factorisations with the fifth-wave lookahead
  // Set by the batched engine: recorded after the factor's last kernel on a
  // stream shared with other work; chol_get_info waits for it instead of
  // the whole stream.
  hipEvent_t ev_ready = nullptr;
  ~chol_factor_s() {
    if (ev_solve) (void)hipEventDestroy(ev_solve);
    if (ev_ready) (void)hipEventDestroy(ev_ready);
  }
};

namespace chol {
// The plain schedule from tile column c_start on (see chol_api.cpp).
int enqueue_factor_tail(chol_factor_s *F, int64_t c_start, int64_t w, int S, hipStream_t s);
}  // namespace chol
