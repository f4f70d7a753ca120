// Linear work index -> tile of a Step-3 update region.  Plain C++ usable on
// the host (for tests) and on the device.
//
// Triangle region: relative tiles (ir, kr), 0 <= kr <= ir < R, R(R+1)/2 of
// them, walked in S x S super-tiles: super-rows top to bottom, inside a
// super-row the super-tiles left to right (the diagonal one last, lower
// triangle only), row-major inside a super-tile.  With P = ceil(R/S)
// super-rows, every super-row but the last has S rows, so the number of tiles
// before super-row I (I <= P-1) is S^2 I(I-1)/2 + I S(S+1)/2, whose inverse
// gives I in closed form.
//
// Band region: relative tiles (ir, kr), kr < K, kr <= ir < R, row-major:
// K(K+1)/2 tiles in the first K rows, then K per row.
#pragma once

#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#define CHOL_HD __host__ __device__
#else
#define CHOL_HD
#endif

namespace chol {

CHOL_HD inline int64_t tri_row(int64_t v) {  // largest r with r(r+1)/2 <= v
  int64_t r = (int64_t)((sqrt(8.0 * (double)v + 1.0) - 1.0) * 0.5);
  while (r > 0 && r * (r + 1) / 2 > v) --r;
  while ((r + 1) * (r + 2) / 2 <= v) ++r;
  return r;
}

CHOL_HD inline int64_t super_prefix(int64_t I, int64_t S) {
  return S * S * I * (I - 1) / 2 + I * S * (S + 1) / 2;
}

CHOL_HD inline void map_triangle(int64_t t, int64_t R, int64_t S, int64_t &ir, int64_t &kr) {
  const int64_t P = (R + S - 1) / S;
  int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) / (2.0 * (double)S));
  if (I > P - 1) I = P - 1;
  if (I < 0) I = 0;
  while (I > 0 && super_prefix(I, S) > t) --I;
  while (I + 1 <= P - 1 && super_prefix(I + 1, S) <= t) ++I;
  const int64_t rows = (R - I * S < S) ? R - I * S : S;
  const int64_t u = t - super_prefix(I, S);
  if (u < I * rows * S) {
    const int64_t kc = u / (rows * S), v = u % (rows * S);
    ir = I * S + v / S;
    kr = kc * S + v % S;
  } else {
    const int64_t v = u - I * rows * S;
    const int64_t r = tri_row(v);
    ir = I * S + r;
    kr = I * S + (v - r * (r + 1) / 2);
  }
}

CHOL_HD inline void map_band(int64_t t, int64_t K, int64_t &ir, int64_t &kr) {
  const int64_t head = K * (K + 1) / 2;
  if (t < head) {
    const int64_t r = tri_row(t);
    ir = r;
    kr = t - r * (r + 1) / 2;
  } else {
    const int64_t u = t - head;
    ir = K + u / K;
    kr = u % K;
  }
}

CHOL_HD inline int64_t triangle_count(int64_t R) { return R * (R + 1) / 2; }
CHOL_HD inline int64_t band_count(int64_t R, int64_t K) {
  return K * (K + 1) / 2 + (R - K) * K;
}

}  // namespace chol
