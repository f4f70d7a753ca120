// Step 3 of the blocked right-looking Cholesky factorisation (the paper's
// algorithm figure, right column, the symmetric and general matrix-matrix
// updates of the trailing blocks):
//   A_ik -= sum_{p in panel} L_ip L_kp^T      for the tiles (i, k), k <= i,
// of a region of the trailing lower triangle.  Diagonal tiles (i == k, the
// symmetric update) are computed in full; their strict upper part is never
// read.  This is where almost all of the n^3/3 flops are spent.
//
// gfx950 design
// -------------
// * One workgroup (4 waves, 2 x 2) per 128 x 128 output tile; each wave owns
//   a 64 x 64 block as 4 x 4 MFMA 16x16 blocks (FP64: v_mfma_f64_16x16x4,
//   FP32: v_mfma_f32_16x16x4; FP16 operands: v_mfma_f32_16x16x32_f16).
//   The accumulators are initialised with the C tile itself and the panel
//   operand A is negated when staged, so each MFMA performs C -= a b^T.
// * Rows are interleaved across the 4 MFMA blocks of a wave so that a lane's
//   four A (or B) fragments come from one or two 16-byte LDS reads that are
//   contiguous across lanes (conflict-free), and a lane's accumulators form
//   16-byte runs of C columns (vector loads/stores of C straight to and from
//   HBM).  See the row-interleave comment in update_kernel.
// * The panel is streamed through LDS in chunks of KC columns (128 bytes per
//   tile row), double-buffered; global loads of chunk s+1 are in flight while
//   chunk s is multiplied.  LDS rows are padded to avoid bank conflicts.
// * Work mapping: the tile region is walked in super-tiles of S x S tiles
//   and the linear order is split into 8 contiguous ranges, one per XCD
//   (workgroup w runs on XCD w mod 8), so the workgroups that share an L2
//   also share panel rows.
#include "internal.hpp"
#include "tile_map.hpp"

namespace chol {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int BT = 128;  // tile side handled by this kernel

// Storage element type, MFMA accumulator type and chunk depth per mode.
template <int MODE> struct Cfg;
// MODE 0: FP64 storage and arithmetic.
template <> struct Cfg<0> {
  using T = double;
  using acc_t = v4d;
  static constexpr int KC = 16;   // columns per LDS chunk (16 * 8 B = 128 B)
  static constexpr int PAD = 4;   // LDS row padding (elements)
};
// MODE 1: FP32 storage and arithmetic.
template <> struct Cfg<1> {
  using T = float;
  using acc_t = v4f;
  static constexpr int KC = 32;
  static constexpr int PAD = 8;
};

__device__ inline uint4 neg_f64x2(uint4 v) {
  v.y ^= 0x80000000u;
  v.w ^= 0x80000000u;
  return v;
}
__device__ inline uint4 neg_f32x4(uint4 v) {
  v.x ^= 0x80000000u;
  v.y ^= 0x80000000u;
  v.z ^= 0x80000000u;
  v.w ^= 0x80000000u;
  return v;
}

// ------------------------------------------------------------ FP64 / FP32 --
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_kernel(
    typename Cfg<MODE>::T *__restrict__ tiles, int64_t N, int64_t p0, int pw, int64_t k0,
    int64_t K, int mode, int S, int64_t G, int64_t G8, const int64_t *__restrict__ info) {
  using C_ = Cfg<MODE>;
  using T = typename C_::T;
  using acc_t = typename C_::acc_t;
  constexpr int KC = C_::KC;
  constexpr int LDP = BT + C_::PAD;
  constexpr int VE = 16 / sizeof(T);            // elements per 16-byte vector
  constexpr int NV = KC * BT / VE / 256;        // 16-byte vectors per thread per operand
  if (*info != 0) return;

  const int64_t bid = blockIdx.x;
  const int64_t t = (bid % 8) * G8 + bid / 8;
  if (t >= G) return;
  int64_t ir, kr;
  if (mode == 0)
    map_triangle(t, N - k0, S, ir, kr);
  else
    map_band(t, K, ir, kr);
  const int64_t i = k0 + ir, k = k0 + kr;

  __shared__ __attribute__((aligned(16))) T lds[2][2][KC * LDP];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;

  T *C = tiles + tile_index(i, k, N) * (int64_t)(BT * BT);

  // Row interleave.  MFMA block s (of 4 per wave and dimension) takes, for
  // its MFMA row index i, the wave-local row
  //   FP64: 2i + (s & 1) + 32 (s >> 1)   -> a lane's fragments are rows
  //         {2q, 2q+1} and {2q+32, 2q+33}: two 16-byte LDS reads that are
  //         contiguous across the 16 lanes of a group (no bank conflicts);
  //   FP32: 4i + s                       -> one 16-byte read {4q..4q+3}.
  // Columns (the B operand) use the same map.  With the MFMA output layouts
  // (lane (g,q), register e holds MFMA row g+4e for f64, 4g+e for f32, and
  // MFMA column q), accumulator acc[s][u][e] is C element
  //   row 64wm + crow(s, e),  column 64wn + ccol(u)
  // with crow = 2g + 8e + (s&1) + 32(s>>1) (FP64) or 16g + 4e + s (FP32),
  // ccol = 2q + (u&1) + 32(u>>1) (FP64) or 4q + u (FP32).  Consecutive s
  // give consecutive rows, so C moves in 16-byte vectors.
  auto crow = [&](int s4, int e) -> int {
    return (MODE == 0) ? 2 * g + 8 * e + (s4 & 1) + 32 * (s4 >> 1) : 16 * g + 4 * e + s4;
  };
  auto ccol = [&](int u) -> int { return (MODE == 0) ? 2 * q + (u & 1) + 32 * (u >> 1) : 4 * q + u; };
  constexpr int SPV = (MODE == 0) ? 2 : 4;  // consecutive s per 16-byte vector

  acc_t acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const T *col = C + (64 * wn + ccol(u)) * BT + 64 * wm;
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int s0 = 0; s0 < 4; s0 += SPV) {
        T v[SPV];
        *(uint4 *)&v[0] = *(const uint4 *)(col + crow(s0, e));
#pragma unroll
        for (int y = 0; y < SPV; ++y) acc[s0 + y][u][e] = v[y];
      }
  }

  const int nstage = pw * (BT / KC);
  uint4 ra[NV], rb[NV];
  auto gload = [&](int s) {
    const int64_t p = p0 + (s * KC) / BT;
    const int col0 = (s * KC) % BT;
    const T *pa = tiles + tile_index(i, p, N) * (int64_t)(BT * BT) + col0 * BT;
    const T *pb = tiles + tile_index(k, p, N) * (int64_t)(BT * BT) + col0 * BT;
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      const int v = tid + 256 * x;
      ra[x] = *(const uint4 *)(pa + v * VE);
      rb[x] = *(const uint4 *)(pb + v * VE);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      const int e = (tid + 256 * x) * VE;
      const int kk = e / BT, r = e % BT;
      uint4 na = (sizeof(T) == 8) ? neg_f64x2(ra[x]) : neg_f32x4(ra[x]);
      *(uint4 *)&lds[buf][0][kk * LDP + r] = na;
      *(uint4 *)&lds[buf][1][kk * LDP + r] = rb[x];
    }
  };
  // fragments of k-step kk for this lane: a[s], b[u]
  auto frag = [&](const T *la, const T *lb, int kk, T (&a)[4], T (&b)[4]) {
    if constexpr (MODE == 0) {
      *(uint4 *)&a[0] = *(const uint4 *)(la + kk * LDP + 64 * wm + 2 * q);
      *(uint4 *)&a[2] = *(const uint4 *)(la + kk * LDP + 64 * wm + 2 * q + 32);
      *(uint4 *)&b[0] = *(const uint4 *)(lb + kk * LDP + 64 * wn + 2 * q);
      *(uint4 *)&b[2] = *(const uint4 *)(lb + kk * LDP + 64 * wn + 2 * q + 32);
    } else {
      *(uint4 *)&a[0] = *(const uint4 *)(la + kk * LDP + 64 * wm + 4 * q);
      *(uint4 *)&b[0] = *(const uint4 *)(lb + kk * LDP + 64 * wn + 4 * q);
    }
  };

  gload(0);
  lstore(0);
  __syncthreads();
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstage) gload(s + 1);
    const T *la = &lds[buf][0][0];
    const T *lb = &lds[buf][1][0];
    T a[2][4], b[2][4];
    frag(la, lb, g, a[0], b[0]);
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int cur = ks & 1;
      if (ks + 1 < KC / 4) frag(la, lb, (ks + 1) * 4 + g, a[cur ^ 1], b[cur ^ 1]);
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if constexpr (MODE == 0)
            acc[s2][u] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][s2], b[cur][u], acc[s2][u], 0, 0, 0);
          else
            acc[s2][u] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(a[cur][s2], b[cur][u], acc[s2][u], 0, 0, 0);
        }
    }
    if (s + 1 < nstage) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int u = 0; u < 4; ++u) {
    T *col = C + (64 * wn + ccol(u)) * BT + 64 * wm;
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int s0 = 0; s0 < 4; s0 += SPV) {
        T v[SPV];
#pragma unroll
        for (int y = 0; y < SPV; ++y) v[y] = acc[s0 + y][u][e];
        *(uint4 *)(col + crow(s0, e)) = *(const uint4 *)&v[0];
      }
  }
}

// ---------------------------------------------------------- FP64, 4x4x4 --
// FP64 update on v_mfma_f64_4x4x4_4b_f64, which on gfx950 sustains the full
// FP64 matrix rate (the 16x16x4 form issues far less often).  Operand
// layout of the instruction (lane l = 16 g + q): the lane supplies A[q][g]
// and B[g][q] of a 16x4 / 4x16 pair, and only the four diagonal 4x4 blocks
// of the 16x16 product are formed: lane l receives D[4 (q/4) + g][q].  So
// block bq = q/4 multiplies A-operand rows 4bq..4bq+3 with B-operand
// columns 4bq..4bq+3.
//
// Each wave owns a 64 x 64 block of the 128 x 128 tile and issues, per
// k-step of 4, 64 instructions (x, y), x < 4, y < 16.  Instruction (x, y)
// feeds A-operand row i with tile row  rho(x, i) = 2i + (x&1) + 32(x>>1)
// and B-operand column j with tile column  sigma(y, j) = 4y + (j mod 4).
// Hence lane (g, q) holds acc[x][y] = C(row 8 bq + 2g + (x&1) + 32(x>>1),
// column 4y + (q mod 4)), every (row, column) of the 64 x 64 block exactly
// once; its A fragments are rows {2q, 2q+1} and {2q+32, 2q+33} (two 16-byte
// LDS reads, contiguous across lanes), its B fragments 16 single elements
// that four lanes share (broadcast reads), and each C column is touched as
// two 16-byte vectors.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_f64_kernel(
    double *__restrict__ tiles, int64_t N, int64_t p0, int pw, int64_t k0, int64_t K, int mode,
    int S, int64_t G, int64_t G8, const int64_t *__restrict__ info) {
  constexpr int KC = 16;          // panel columns per LDS chunk (128 bytes per tile row)
  constexpr int LDP = BT + 4;     // LDS row pitch (doubles)
  constexpr int NV = KC * BT / 2 / 256;  // 16-byte vectors per thread per operand
  if (*info != 0) return;
  const int64_t bid = blockIdx.x;
  const int64_t t = (bid % 8) * G8 + bid / 8;
  if (t >= G) return;
  int64_t ir, kr;
  if (mode == 0)
    map_triangle(t, N - k0, S, ir, kr);
  else
    map_band(t, K, ir, kr);
  const int64_t i = k0 + ir, k = k0 + kr;

  __shared__ __attribute__((aligned(16))) double lds[2][2][KC * LDP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15, bq = q >> 2, jq = q & 3;
  const int wm = wave >> 1, wn = wave & 1;
  double *C = tiles + tile_index(i, k, N) * (int64_t)(BT * BT);

  // acc[x][y] <-> C(64wm + 8bq + 2g + (x&1) + 32(x>>1), 64wn + 4y + jq)
  double acc[4][16];
#pragma unroll
  for (int y = 0; y < 16; ++y) {
    const double *col = C + (64 * wn + 4 * y + jq) * BT + 64 * wm + 8 * bq + 2 * g;
#pragma unroll
    for (int xh = 0; xh < 2; ++xh) {
      double v[2];
      *(uint4 *)&v[0] = *(const uint4 *)(col + 32 * xh);
      acc[2 * xh][y] = v[0];
      acc[2 * xh + 1][y] = v[1];
    }
  }

  const int nstage = pw * (BT / KC);
  uint4 ra[NV], rb[NV];
  auto gload = [&](int s) {
    const int64_t p = p0 + (s * KC) / BT;
    const int col0 = (s * KC) % BT;
    const double *pa = tiles + tile_index(i, p, N) * (int64_t)(BT * BT) + col0 * BT;
    const double *pb = tiles + tile_index(k, p, N) * (int64_t)(BT * BT) + col0 * BT;
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      const int v = tid + 256 * x;
      ra[x] = *(const uint4 *)(pa + v * 2);
      rb[x] = *(const uint4 *)(pb + v * 2);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      const int e = (tid + 256 * x) * 2;
      const int kk = e / BT, r = e % BT;
      *(uint4 *)&lds[buf][0][kk * LDP + r] = neg_f64x2(ra[x]);
      *(uint4 *)&lds[buf][1][kk * LDP + r] = rb[x];
    }
  };

  gload(0);
  lstore(0);
  __syncthreads();
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstage) gload(s + 1);
    const double *la = &lds[buf][0][64 * wm + 2 * q];
    const double *lb = &lds[buf][1][64 * wn + jq];
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = ks * 4 + g;
      double a[4], b[16];
      *(uint4 *)&a[0] = *(const uint4 *)(la + kk * LDP);
      *(uint4 *)&a[2] = *(const uint4 *)(la + kk * LDP + 32);
#pragma unroll
      for (int y = 0; y < 16; ++y) b[y] = lb[kk * LDP + 4 * y];
#pragma unroll
      for (int y = 0; y < 16; ++y)
#pragma unroll
        for (int x = 0; x < 4; ++x)
          acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (s + 1 < nstage) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int y = 0; y < 16; ++y) {
    double *col = C + (64 * wn + 4 * y + jq) * BT + 64 * wm + 8 * bq + 2 * g;
#pragma unroll
    for (int xh = 0; xh < 2; ++xh) {
      double v[2] = {acc[2 * xh][y], acc[2 * xh + 1][y]};
      *(uint4 *)(col + 32 * xh) = *(const uint4 *)&v[0];
    }
  }
}

// --------------------------------------------------- FP16 operands (FP32 C) --
// Panel tiles are FP32 in memory; each chunk is rounded to FP16 when staged.
// v_mfma_f32_16x16x32_f16: lane (g, q) supplies A[row q][k = 8g .. 8g+7] and
// B[k = 8g .. 8g+7][col q]; LDS keeps the chunk k-contiguous per row
// ([row][k], KC16 = 32 halves = 64 bytes per row, padded), so each fragment
// is one 16-byte read.  Rows are interleaved across MFMA blocks as above.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_f16_kernel(
    float *__restrict__ tiles, int64_t N, int64_t p0, int pw, int64_t k0, int64_t K, int mode,
    int S, int64_t G, int64_t G8, const int64_t *__restrict__ info) {
  constexpr int KC16 = 32;            // k per chunk
  constexpr int RP = KC16 + 8;        // LDS row pitch in halves (80 bytes)
  if (*info != 0) return;
  const int64_t bid = blockIdx.x;
  const int64_t t = (bid % 8) * G8 + bid / 8;
  if (t >= G) return;
  int64_t ir, kr;
  if (mode == 0)
    map_triangle(t, N - k0, S, ir, kr);
  else
    map_band(t, K, ir, kr);
  const int64_t i = k0 + ir, k = k0 + kr;

  __shared__ __attribute__((aligned(16))) _Float16 lds[2][2][BT * RP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  float *C = tiles + tile_index(i, k, N) * (int64_t)(BT * BT);

  v4f acc[4][4];
  {
    const int r0 = 64 * wm + 16 * g;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float *src = C + (64 * wn + 4 * q + u) * BT + r0;
      float v[16];
#pragma unroll
      for (int x = 0; x < 4; ++x) *(uint4 *)&v[x * 4] = *(const uint4 *)(src + x * 4);
#pragma unroll
      for (int rho = 0; rho < 16; ++rho) acc[rho & 3][u][rho >> 2] = v[rho];
    }
  }
  // Chunk = 32 columns x 128 rows of FP32 = 4096 floats = 1024 float4 per operand;
  // each thread loads 4 float4 of A and of B.  Thread -> (column kk, rows r..r+3).
  const int nstage = pw * (BT / KC16);
  float4 ra[4], rb[4];
  auto gload = [&](int s) {
    const int64_t p = p0 + (s * KC16) / BT;
    const int col0 = (s * KC16) % BT;
    const float *pa = tiles + tile_index(i, p, N) * (int64_t)(BT * BT) + col0 * BT;
    const float *pb = tiles + tile_index(k, p, N) * (int64_t)(BT * BT) + col0 * BT;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int v = tid + 256 * x;
      ra[x] = *(const float4 *)(pa + v * 4);
      rb[x] = *(const float4 *)(pb + v * 4);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int e = (tid + 256 * x) * 4;
      const int kk = e / BT, r = e % BT;
      const float av[4] = {ra[x].x, ra[x].y, ra[x].z, ra[x].w};
      const float bv[4] = {rb[x].x, rb[x].y, rb[x].z, rb[x].w};
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        lds[buf][0][(r + y) * RP + kk] = (_Float16)(-av[y]);
        lds[buf][1][(r + y) * RP + kk] = (_Float16)bv[y];
      }
    }
  };
  gload(0);
  lstore(0);
  __syncthreads();
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstage) gload(s + 1);
    const _Float16 *la = &lds[buf][0][0];
    const _Float16 *lb = &lds[buf][1][0];
    v8h a[4], b[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      a[s2] = *(const v8h *)(la + (64 * wm + 4 * q + s2) * RP + 8 * g);
      b[s2] = *(const v8h *)(lb + (64 * wn + 4 * q + s2) * RP + 8 * g);
    }
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[s2][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[s2], b[u], acc[s2][u], 0, 0, 0);
    if (s + 1 < nstage) lstore(buf ^ 1);
    __syncthreads();
  }
  {
    const int r0 = 64 * wm + 16 * g;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float *dst = C + (64 * wn + 4 * q + u) * BT + r0;
      float v[16];
#pragma unroll
      for (int rho = 0; rho < 16; ++rho) v[rho] = acc[rho & 3][u][rho >> 2];
#pragma unroll
      for (int x = 0; x < 4; ++x) *(uint4 *)(dst + x * 4) = *(const uint4 *)&v[x * 4];
    }
  }
}

// Portable fallback for tile side 64 (small problems): one workgroup of 256
// threads per 64 x 64 tile, plain FP64 FMAs, panel read through LDS.
template <typename T>
__global__ __launch_bounds__(256) void update64_kernel(T *__restrict__ tiles, int64_t N,
                                                       int64_t p0, int pw, int64_t k0, int64_t K,
                                                       int mode, int S, int64_t G,
                                                       const int64_t *__restrict__ info) {
  constexpr int B = 64;
  if (*info != 0) return;
  const int64_t t = blockIdx.x;
  if (t >= G) return;
  int64_t ir, kr;
  if (mode == 0)
    map_triangle(t, N - k0, S, ir, kr);
  else
    map_band(t, K, ir, kr);
  const int64_t i = k0 + ir, k = k0 + kr;
  __shared__ double la[16][B + 1], lb[16][B + 1];
  T *C = tiles + tile_index(i, k, N) * (int64_t)(B * B);
  const int tid = threadIdx.x;
  const int r = tid & 63, cg = tid >> 6;  // row r, columns cg + 4m
  double acc[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) acc[m] = (double)C[(cg + 4 * m) * B + r];
  for (int p = 0; p < pw; ++p) {
    const T *pa = tiles + tile_index(i, p0 + p, N) * (int64_t)(B * B);
    const T *pb = tiles + tile_index(k, p0 + p, N) * (int64_t)(B * B);
    for (int kc = 0; kc < B; kc += 16) {
      __syncthreads();
      for (int e = tid; e < 16 * B; e += 256) {
        const int kk = e / B, rr = e % B;
        la[kk][rr] = (double)pa[(kc + kk) * B + rr];
        lb[kk][rr] = (double)pb[(kc + kk) * B + rr];
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double av = la[kk][r];
#pragma unroll
        for (int m = 0; m < 16; ++m) acc[m] -= av * lb[kk][cg + 4 * m];
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 16; ++m) C[(cg + 4 * m) * B + r] = (T)acc[m];
}

}  // namespace

void launch_update(void *tiles, int store, int b, int64_t N, int64_t p0, int pw, int64_t k0,
                   int64_t k1, int mode, int super_tile, int fp16, const int64_t *info,
                   hipStream_t s) {
  const int64_t R = N - k0;
  if (R <= 0 || pw <= 0) return;
  const int64_t K = k1 - k0;
  int64_t G;
  if (mode == 0) {
    G = triangle_count(R);
  } else {
    if (K <= 0 || K > R) return;
    G = band_count(R, K);
  }
  if (G <= 0) return;
  if (b == BT) {
    const int64_t G8 = (G + 7) / 8;
    const dim3 grid((unsigned)(8 * G8));
    if (fp16)
      hipLaunchKernelGGL(update_f16_kernel, grid, dim3(256), 0, s, (float *)tiles, N, p0, pw, k0,
                         K, mode, super_tile, G, G8, info);
    else if (store == STORE_F64)
      hipLaunchKernelGGL(update_f64_kernel, grid, dim3(256), 0, s, (double *)tiles, N, p0, pw, k0,
                         K, mode, super_tile, G, G8, info);
    else
      hipLaunchKernelGGL(update_kernel<1>, grid, dim3(256), 0, s, (float *)tiles, N, p0, pw, k0,
                         K, mode, super_tile, G, G8, info);
  } else {
    const dim3 grid((unsigned)G);
    if (store == STORE_F64)
      hipLaunchKernelGGL(update64_kernel<double>, grid, dim3(256), 0, s, (double *)tiles, N, p0,
                         pw, k0, K, mode, super_tile, G, info);
    else
      hipLaunchKernelGGL(update64_kernel<float>, grid, dim3(256), 0, s, (float *)tiles, N, p0, pw,
                         k0, K, mode, super_tile, G, info);
  }
}

}  // namespace chol
