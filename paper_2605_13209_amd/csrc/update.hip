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
//   a 64 x 64 block (FP64: v_mfma_f64_4x4x4_4b_f64, FP32:
//   v_mfma_f32_16x16x4_f32, FP16 operands: v_mfma_f32_16x16x32_f16).
//   The accumulators start at -C and the tile is negated back on store, so
//   the panel operands are used unmodified and each MFMA adds a b^T.
// * Rows are interleaved across the MFMA blocks of a wave so that a lane's
//   A (or B) fragments come from 16-byte LDS reads that are contiguous
//   across lanes, and a lane's accumulators form runs of C columns moved
//   with vector loads/stores straight to and from HBM (FP32 C: exchanged
//   between lanes first, so that every access covers whole 64-byte pieces).
// * FP64 / FP32: the panel is streamed through LDS in chunks of 128 bytes per
//   tile row by LDS DMA (global_load_lds_dwordx4), two chunks ahead, and the
//   fragments of the next k-step are read while the MFMAs of the current one
//   run; one barrier per chunk.  FP16 operands are rounded when staged.
// * Work mapping: the tile region is walked in super-tiles of S x S tiles
//   and the linear order is split into 8 contiguous ranges, one per XCD
//   (workgroup w runs on XCD w mod 8), so the workgroups that share an L2
//   also share panel rows.  Workgroups are persistent: a grid smaller than
//   the tile count walks the range.
#include "internal.hpp"
#include "tile_map.hpp"

namespace chol {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int BT = 128;  // tile side handled by the matrix-core kernels

// LDS DMA: global_load_lds_dwordx4 moves 16 bytes per lane from global
// memory straight into LDS, lane l writing bytes [16 l, 16 l + 16) after the
// wave-uniform LDS address held in M0; the global address is a scalar base
// plus a per-lane 32-bit byte offset.  It is issued as inline asm so that the
// compiler, which cannot tell which LDS bytes an outstanding DMA writes, does
// not wait for all of them before every LDS read; callers wait explicitly
// (wait_vmem) before the barrier that publishes the data.
template <typename T> __device__ inline T *uniform_ptr(T *p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
typedef __attribute__((address_space(3))) void lds_void_t;
__device__ inline void lds_dma16(const void *base, uint32_t voff, void *lds_dst) {
  const uint32_t m0v = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)lds_dst);
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, %2" ::"s"(m0v), "v"(voff),
               "s"(uniform_ptr(base))
               : "memory", "m0");
}
__device__ inline void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// C runs of the FP32-accumulating kernels.  In the MFMA output layout lane
// (g, q) of a wave holds, for one output column, the 16 rows 16 g + 4 e + s2
// of a 64-row block (register e, component s2): 64 contiguous bytes per lane.
// Moved as is, one 16-byte access per e would touch four 16-byte pieces 64
// bytes apart per column, and partly written lines leave L2 as partial
// writes (counted: 1.45x the C bytes).  Instead the four lanes g = 0..3 of a
// column exchange their registers as a 4 x 4 transpose (two lane-swap
// stages: rows of 32 lanes, then rows of 16), after which access e of the
// four lanes covers the 64 contiguous bytes of rows 16 e .. 16 e + 15.  The
// transpose is its own inverse, so loads apply it after, stores before.
__device__ inline void xpose_g(v4f *x) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[e][c]),
                                                      __float_as_uint(x[e + 2][c]), false, false);
      x[e][c] = __uint_as_float(t[0]);
      x[e + 2][c] = __uint_as_float(t[1]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int e = 0; e < 4; e += 2) {
      const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(x[e][c]),
                                                      __float_as_uint(x[e + 1][c]), false, false);
      x[e][c] = __uint_as_float(t[0]);
      x[e + 1][c] = __uint_as_float(t[1]);
    }
  }
}
// c: the 64-row block of the lane's column; x[e][s2] = row 16 g + 4 e + s2.
// Every lane of the wave must take part (cross-lane exchange).
__device__ inline void load_c_run(const float *c, int g, v4f *x) {
#pragma unroll
  for (int e = 0; e < 4; ++e) x[e] = *(const v4f *)(c + 16 * e + 4 * g);
  xpose_g(x);
}
__device__ inline void store_c_run(float *c, int g, v4f *x) {
  xpose_g(x);
#pragma unroll
  for (int e = 0; e < 4; ++e) *(v4f *)(c + 16 * e + 4 * g) = x[e];
}

// ------------------------------------------------------------------ FP32 --
// FP32 storage and arithmetic on v_mfma_f32_16x16x4_f32.  Each wave owns a
// 64 x 64 block as 4 x 4 MFMA blocks (s2, u).  MFMA row i of block s2 is
// wave-local row 4i + s2 (and likewise column 4j + u), so a lane's four A
// fragments (rows 4q .. 4q+3 at k = 4 ks + g) and four B fragments are one
// 16-byte LDS read each, contiguous across lanes.  With the MFMA output
// layout (lane (g, q), register e holds MFMA row 4g + e, column q) the
// accumulator acc[s2][u][e] is C(64 wm + 16g + 4e + s2, 64 wn + 4q + u):
// C moves as 16-byte vectors, through load_c_run / store_c_run.  Chunks of 32 panel columns (128 bytes per tile
// row) are DMA'd into unpadded LDS (the 16-byte fragment reads are
// conflict-free without padding), two chunks ahead, with the same one-barrier
// protocol as the FP64 kernel below (barrier after the second-to-last k-step
// of a chunk).
// REGION 3 (the serving engine's batched column step): the work list of a
// BatchDesc (passed as `tiles`), whose job j contributes the trailing
// triangle of its column c_j (panel width 1); G and G8 are read from it.
template <int REGION>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_f32_kernel(
    float *__restrict__ tiles, int64_t N, int64_t p0, int pw, int64_t k0, int64_t K, int S,
    int64_t G, int64_t G8, const int64_t *__restrict__ info) {
  constexpr int KC = 32;        // panel columns per chunk
  constexpr int NKS = KC / 4;   // k-steps per chunk
  const BatchDesc *bd = (const BatchDesc *)tiles;
  if (REGION == 3) {
    G = bd->upd_total;
    G8 = (G + 7) / 8;
  } else if (*info != 0) {
    return;
  }
  __shared__ __attribute__((aligned(16))) float lds[2][2][KC * BT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  const int wu = __builtin_amdgcn_readfirstlane(wave);
  const int64_t per = gridDim.x / 8;  // persistent, as in the FP64 kernel
  for (int64_t pos = blockIdx.x / 8; pos < G8; pos += per) {
    const int64_t t = (blockIdx.x % 8) * G8 + pos;
    if (t >= G) break;
    float *tl = tiles;
    int64_t NN = N, P0 = p0, i, k;
    if (REGION == 3) {
      int64_t j = 0;
      const int64_t nj = bd->njobs;
      while (j + 1 < nj && bd->jobs[j + 1].upd_begin <= t) ++j;
      const BatchJob &J = bd->jobs[j];
      if (*J.info != 0) continue;  // uniform over the workgroup
      int64_t ir, kr;
      map_triangle(t - J.upd_begin, J.N - J.c - 1, S, ir, kr);
      tl = (float *)J.tiles;
      NN = J.N;
      P0 = J.c;
      i = J.c + 1 + ir;
      k = J.c + 1 + kr;
    } else {
      int64_t ir, kr;
      if (REGION == 0)
        map_triangle(t, N - k0, S, ir, kr);
      else
        map_band(t, K, ir, kr);
      i = k0 + ir;
      k = k0 + kr;
    }
    float *C = tl + tile_index(i, k, NN) * (int64_t)(BT * BT);
    const int nstage = pw * (BT / KC);

    // chunk s: 32 columns = 16 KB per operand = 16 one-KB column pairs;
    // wave w moves pairs w, w+4, w+8, w+12 of both operands
    auto dma = [&](int s) {
      const int64_t p = P0 + (s * KC) / BT;
      const int col0 = (s * KC) % BT;
      const float *pa = tl + tile_index(i, p, NN) * (int64_t)(BT * BT) + col0 * BT;
      const float *pb = tl + tile_index(k, p, NN) * (int64_t)(BT * BT) + col0 * BT;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int off = (wu + 4 * c) * 2 * BT;
        lds_dma16(pa + off, lane * 16, &lds[s & 1][0][off]);
        lds_dma16(pb + off, lane * 16, &lds[s & 1][1][off]);
      }
    };

    v4f acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v4f x[4];
      load_c_run(C + (64 * wn + 4 * q + u) * BT + 64 * wm, g, x);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) acc[s2][u][e] = -x[e][s2];
    }
    dma(0);
    if (nstage > 1) dma(1);
    wait_vmem();
    __syncthreads();

    float fa[2][4], fb[2][4];
    *(uint4 *)&fa[0][0] = *(const uint4 *)&lds[0][0][g * BT + 64 * wm + 4 * q];
    *(uint4 *)&fb[0][0] = *(const uint4 *)&lds[0][1][g * BT + 64 * wn + 4 * q];
    const int nk = nstage * NKS;
    auto step = [&](int kt, int cur) {
      const int s = kt / NKS, ks = kt % NKS;
      const int nbuf = ((kt + 1) / NKS) & 1, nks = (kt + 1) % NKS;
      // next k-step's fragments (stale but in-bounds after the last step)
      *(uint4 *)&fa[cur ^ 1][0] = *(const uint4 *)&lds[nbuf][0][(4 * nks + g) * BT + 64 * wm + 4 * q];
      *(uint4 *)&fb[cur ^ 1][0] = *(const uint4 *)&lds[nbuf][1][(4 * nks + g) * BT + 64 * wn + 4 * q];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc[s2][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[cur][s2], fb[cur][u], acc[s2][u], 0, 0, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
      __builtin_amdgcn_sched_barrier(0);
      if (ks == NKS - 2) {
        wait_vmem();
        __syncthreads();
        if (s + 2 < nstage) dma(s + 2);
      }
    };
    for (int kt = 0; kt < nk; kt += 2) {
      step(kt, 0);
      step(kt + 1, 1);
    }

#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v4f x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) x[e][s2] = -acc[s2][u][e];
      store_c_run(C + (64 * wn + 4 * q + u) * BT + 64 * wm, g, x);
    }
  }  // tiles of this workgroup
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
//
// Staging: the panel chunks go from HBM straight into LDS with
// global_load_lds_dwordx4 (no VGPR round trip, which frees the registers
// for a second set of fragments), two chunks ahead.  The accumulators start
// at -C and the tile is negated back on store, so the operands are staged
// unmodified and every MFMA adds a b^T.  With fragments for k-step t+1 read
// from LDS while the MFMAs of step t run, one barrier per chunk suffices,
// placed after the third of its four k-steps:
//   step 2 of chunk s: wait for this wave's DMA of chunk s+1, barrier B_s
//                      (all waves have read chunk s's fragments and all DMA
//                      of chunk s+1 has landed), then DMA chunk s+2 into
//                      the buffer chunk s used;
//   step 3 of chunk s: read the first fragments of chunk s+1.
// REGION 2 (rectangle, used by the heterogeneous factorisation): tiles
// (k0 + S + t / K, k0 + t mod K), i.e. rows [k0 + S, N) by columns
// [k0, k0 + K), S then being the row offset instead of the super-tile side.
template <int REGION>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_f64_kernel(
    double *__restrict__ tiles, int64_t N, int64_t p0, int pw, int64_t k0, int64_t K, int S,
    int64_t G, int64_t G8, const int64_t *__restrict__ info) {
  constexpr int KC = 16;       // panel columns per LDS chunk (128 bytes per tile row)
  constexpr int LDP = BT + 4;  // LDS row pitch (doubles)
  if (*info != 0) return;
  __shared__ __attribute__((aligned(16))) double lds[2][2][KC * LDP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15, bq = q >> 2, jq = q & 3;
  const int wm = wave >> 1, wn = wave & 1;
  const int wu = __builtin_amdgcn_readfirstlane(wave);
  // Persistent: workgroup w walks the tiles of XCD range w mod 8 (positions
  // w/8, w/8 + per, ...), so the grid may be smaller than the tile count.
  const int64_t per = gridDim.x / 8;
  for (int64_t pos = blockIdx.x / 8; pos < G8; pos += per) {
    const int64_t t = (blockIdx.x % 8) * G8 + pos;
    if (t >= G) break;
    int64_t ir, kr;
    if (REGION == 0) {
      map_triangle(t, N - k0, S, ir, kr);
    } else if (REGION == 1) {
      map_band(t, K, ir, kr);
    } else {
      ir = S + t / K;
      kr = t % K;
    }
    const int64_t i = k0 + ir, k = k0 + kr;
    double *C = tiles + tile_index(i, k, N) * (int64_t)(BT * BT);
    const int nstage = pw * (BT / KC);

    // chunk s = columns [16 s mod 128, +16) of panel tile p0 + 16 s / 128;
    // wave w moves columns w, w+4, w+8, w+12 of both operands (1 KB each)
    auto dma = [&](int s) {
      const int64_t p = p0 + (s * KC) / BT;
      const int col0 = (s * KC) % BT;
      const double *pa = tiles + tile_index(i, p, N) * (int64_t)(BT * BT) + col0 * BT;
      const double *pb = tiles + tile_index(k, p, N) * (int64_t)(BT * BT) + col0 * BT;
#pragma unroll
      for (int c = 0; c < KC / 4; ++c) {
        const int kk = wu + 4 * c;
        lds_dma16(pa + kk * BT, lane * 16, &lds[s & 1][0][kk * LDP]);
        lds_dma16(pb + kk * BT, lane * 16, &lds[s & 1][1][kk * LDP]);
      }
    };

    // acc[x][y] <-> -C(64wm + 8bq + 2g + (x&1) + 32(x>>1), 64wn + 4y + jq)
    double acc[4][16];
#pragma unroll
    for (int y = 0; y < 16; ++y) {
      const double *col = C + (64 * wn + 4 * y + jq) * BT + 64 * wm + 8 * bq + 2 * g;
#pragma unroll
      for (int xh = 0; xh < 2; ++xh) {
        double v[2];
        *(uint4 *)&v[0] = *(const uint4 *)(col + 32 * xh);
        acc[2 * xh][y] = -v[0];
        acc[2 * xh + 1][y] = -v[1];
      }
    }
    dma(0);
    if (nstage > 1) dma(1);
    wait_vmem();
    __syncthreads();

    // fa[buf]: A fragments of the current / next k-step; fb: B fragments,
    // each overwritten with the next step's value once its 4 MFMAs are issued
    double fa[2][4], fb[16];
    {
      const double *la = &lds[0][0][64 * wm + 2 * q + g * LDP];
      const double *lb = &lds[0][1][64 * wn + jq + g * LDP];
      *(uint4 *)&fa[0][0] = *(const uint4 *)(la);
      *(uint4 *)&fa[0][2] = *(const uint4 *)(la + 32);
#pragma unroll
      for (int y = 0; y < 16; ++y) fb[y] = lb[4 * y];
    }
    const int nk = nstage * (KC / 4);
    auto step = [&](int kt, int cur) {
      const int s = kt >> 2, ks = kt & 3;
      // next k-step's fragments (after the last step this reads stale but
      // in-bounds LDS; the values are not used)
      const int nbuf = ((kt + 1) >> 2) & 1, nks = (kt + 1) & 3;
      const double *la = &lds[nbuf][0][64 * wm + 2 * q + (nks * 4 + g) * LDP];
      const double *lb = &lds[nbuf][1][64 * wn + jq + (nks * 4 + g) * LDP];
      *(uint4 *)&fa[cur ^ 1][0] = *(const uint4 *)(la);
      *(uint4 *)&fa[cur ^ 1][2] = *(const uint4 *)(la + 32);
#pragma unroll
      for (int y = 0; y < 16; ++y) {
#pragma unroll
        for (int x = 0; x < 4; ++x)
          acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[cur][x], fb[y], acc[x][y], 0, 0, 0);
        fb[y] = lb[4 * y];
      }
      // interleave: the two A reads first, then one B read per 4 MFMAs
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (ks == 2) {
        wait_vmem();
        __syncthreads();
        if (s + 2 < nstage) dma(s + 2);
      }
    };
    for (int kt = 0; kt < nk; kt += 2) {
      step(kt, 0);
      step(kt + 1, 1);
    }

#pragma unroll
    for (int y = 0; y < 16; ++y) {
      double *col = C + (64 * wn + 4 * y + jq) * BT + 64 * wm + 8 * bq + 2 * g;
#pragma unroll
      for (int xh = 0; xh < 2; ++xh) {
        double v[2] = {-acc[2 * xh][y], -acc[2 * xh + 1][y]};
        *(uint4 *)(col + 32 * xh) = *(const uint4 *)&v[0];
      }
    }
  }  // tiles of this workgroup
}

// --------------------------------------------------- FP16 operands (FP32 C) --
// The FP16 form's panel solve writes each finished tile column once more in
// FP16, into the panel buffer in the layout of p16_pos (internal.hpp): the
// update kernels DMA its 16 KB chunks straight into LDS, where their fragment
// reads are conflict-free, and no transpose is left in the inner loop.
constexpr int P16_CHMAX = kP16ChunksPerTileRow;  // chunks of 64 columns per tile row
constexpr int P16_CHUNK = BT * 64;               // halves per chunk

// Trailing update with FP16 operands from the converted panel and FP32 C
// (accumulators start at -C).  Same structure as the FP32 kernel: chunks of
// 64 panel columns DMA'd two ahead, next k-step's fragments read during the
// current MFMAs, one barrier per chunk (after its first of two k-steps).
template <int REGION>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_f16_kernel(
    float *__restrict__ tiles, const _Float16 *__restrict__ p16, int64_t N, int pw, int64_t k0,
    int64_t K, int S, int64_t G, int64_t G8, const int64_t *__restrict__ info) {
  constexpr int NKS = 2;  // k-steps of 32 per chunk
  if (*info != 0) return;
  __shared__ __attribute__((aligned(16))) _Float16 lds[2][2][P16_CHUNK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  const int wu = __builtin_amdgcn_readfirstlane(wave);
  const int64_t per = gridDim.x / 8;  // persistent, as in the FP64 kernel
  for (int64_t pos = blockIdx.x / 8; pos < G8; pos += per) {
    const int64_t t = (blockIdx.x % 8) * G8 + pos;
    if (t >= G) break;
    int64_t ir, kr;
    if (REGION == 0)
      map_triangle(t, N - k0, S, ir, kr);
    else
      map_band(t, K, ir, kr);
    const int64_t i = k0 + ir, k = k0 + kr;
    float *C = tiles + tile_index(i, k, N) * (int64_t)(BT * BT);
    const int nstage = 2 * pw;
    // chunk s: 16 KB per operand; wave w moves KB w*4 .. w*4+3 of both
    auto dma = [&](int s) {
      const _Float16 *pa = p16 + (i * P16_CHMAX + s) * (int64_t)P16_CHUNK;
      const _Float16 *pb = p16 + (k * P16_CHMAX + s) * (int64_t)P16_CHUNK;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int off = (wu * 4 + c) * 512;  // halves (1 KB)
        lds_dma16(pa + off, lane * 16, &lds[s & 1][0][off]);
        lds_dma16(pb + off, lane * 16, &lds[s & 1][1][off]);
      }
    };
    v4f acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v4f x[4];
      load_c_run(C + (64 * wn + 4 * q + u) * BT + 64 * wm, g, x);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) acc[s2][u][e] = -x[e][s2];
    }
    dma(0);
    if (nstage > 1) dma(1);
    wait_vmem();
    __syncthreads();
    // fragment of wave-local row 4q + s2 (operand base row r0), k-step ks
    auto frag = [&](const _Float16 *l, int r0, int s2, int ks) -> v8h {
      return *(const v8h *)(l + p16_pos(r0 + 4 * q + s2, 4 * ks + g));
    };
    v8h fa[2][4], fb[2][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      fa[0][x] = frag(lds[0][0], 64 * wm, x, 0);
      fb[0][x] = frag(lds[0][1], 64 * wn, x, 0);
    }
    const int nk = nstage * NKS;
    auto step = [&](int kt, int cur) {
      const int s = kt / NKS, ks = kt % NKS;
      const int nbuf = ((kt + 1) / NKS) & 1, nks = (kt + 1) % NKS;
#pragma unroll
      for (int x = 0; x < 4; ++x) {  // next k-step (stale but in-bounds after the last)
        fa[cur ^ 1][x] = frag(lds[nbuf][0], 64 * wm, x, nks);
        fb[cur ^ 1][x] = frag(lds[nbuf][1], 64 * wn, x, nks);
      }
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          acc[s2][u] =
              __builtin_amdgcn_mfma_f32_16x16x32_f16(fa[cur][s2], fb[cur][u], acc[s2][u], 0, 0, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
      __builtin_amdgcn_sched_barrier(0);
      if (ks == NKS - 2) {
        wait_vmem();
        __syncthreads();
        if (s + 2 < nstage) dma(s + 2);
      }
    };
    for (int kt = 0; kt < nk; kt += 2) {
      step(kt, 0);
      step(kt + 1, 1);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v4f x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) x[e][s2] = -acc[s2][u][e];
      store_c_run(C + (64 * wn + 4 * q + u) * BT + 64 * wm, g, x);
    }
  }  // tiles of this workgroup
}

// The same update over the whole trailing triangle with 2 x 2 tiles per
// workgroup (256 x 256 outputs, 8 waves of 128 x 64): every panel chunk
// staged in LDS serves twice the flops of the one-tile kernel, halving the
// L2 -> LDS operand traffic per flop, which bounds the FP16 form once the
// pass is wide.  Super-tile (I, K) covers tile rows 2I, 2I+1 and tile
// columns 2K, 2K+1 of the region; quadrants above the diagonal or past the
// matrix are computed on whatever the LDS holds and never loaded or stored.
// LDS per stage: the two A row chunks and the two B row chunks (64 KB).
__global__ __launch_bounds__(512) void update_f16_wide_kernel(
    float *__restrict__ tiles, const _Float16 *__restrict__ p16, int64_t N, int pw, int64_t k0,
    int S, int64_t G, int64_t G8, const int64_t *__restrict__ info) {
  constexpr int NKS = 2;  // k-steps of 32 per chunk
  if (*info != 0) return;
  __shared__ __attribute__((aligned(16))) _Float16 lds[2][4][P16_CHUNK];  // A0 A1 B0 B1
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int wm = wave >> 2, wn = wave & 3;  // tile row 2I + wm; tile column 2K + wn/2
  const int wu = __builtin_amdgcn_readfirstlane(wave);
  const int64_t R2 = (N - k0 + 1) / 2;
  const int64_t per = gridDim.x / 8;
  for (int64_t pos = blockIdx.x / 8; pos < G8; pos += per) {
    const int64_t t = (blockIdx.x % 8) * G8 + pos;
    if (t >= G) break;
    int64_t IR, KR;
    map_triangle(t, R2, S, IR, KR);
    const int64_t ib = k0 + 2 * IR, kb = k0 + 2 * KR;  // first tile row / column
    const int64_t i = ib + wm, k = kb + (wn >> 1);
    const bool valid = i < N && k <= i;  // wave-uniform
    const int cb = 64 * (wn & 1);        // the wave's first column in tile (i, k)
    float *C = valid ? tiles + tile_index(i, k, N) * (int64_t)(BT * BT) : nullptr;
    const int nstage = 2 * pw;
    // chunk s: wave w moves 8 KB of operand chunk w / 2 (A0, A1, B0, B1)
    const int op = wu >> 1;
    const int64_t orow = (op < 2 ? ib : kb) + (op & 1);  // tile row of that operand chunk
    auto dma = [&](int s) {
      if (orow >= N) return;  // rows past the matrix: nothing to stage
      const _Float16 *src = p16 + (orow * P16_CHMAX + s) * (int64_t)P16_CHUNK;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int off = ((wu & 1) * 8 + c) * 512;  // halves (1 KB)
        lds_dma16(src + off, lane * 16, &lds[s & 1][op][off]);
      }
    };
    v4f acc[2][4][4];  // [row half][s2][u]
    if (valid) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v4f x[4];
          load_c_run(C + (cb + 4 * q + u) * BT + 64 * h, g, x);
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) acc[h][s2][u][e] = -x[e][s2];
        }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[h][s2][u] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    dma(0);
    if (nstage > 1) dma(1);
    wait_vmem();
    __syncthreads();
    auto frag = [&](const _Float16 *l, int r0, int s2, int ks) -> v8h {
      return *(const v8h *)(l + p16_pos(r0 + 4 * q + s2, 4 * ks + g));
    };
    v8h fa[2][8], fb[2][4];
#pragma unroll
    for (int x = 0; x < 8; ++x) fa[0][x] = frag(lds[0][wm], 64 * (x >> 2), x & 3, 0);
#pragma unroll
    for (int x = 0; x < 4; ++x) fb[0][x] = frag(lds[0][2 + (wn >> 1)], cb, x, 0);
    const int nk = nstage * NKS;
    auto step = [&](int kt, int cur) {
      const int s = kt / NKS, ks = kt % NKS;
      const int nbuf = ((kt + 1) / NKS) & 1, nks = (kt + 1) % NKS;
#pragma unroll
      for (int x = 0; x < 8; ++x)  // next k-step (stale but in-bounds after the last)
        fa[cur ^ 1][x] = frag(lds[nbuf][wm], 64 * (x >> 2), x & 3, nks);
#pragma unroll
      for (int x = 0; x < 4; ++x) fb[cur ^ 1][x] = frag(lds[nbuf][2 + (wn >> 1)], cb, x, nks);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[h][s2][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa[cur][4 * h + s2], fb[cur][u],
                                                                    acc[h][s2][u], 0, 0, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 32, 0);
      __builtin_amdgcn_sched_barrier(0);
      if (ks == NKS - 2) {
        wait_vmem();
        __syncthreads();
        if (s + 2 < nstage) dma(s + 2);
      }
    };
    for (int kt = 0; kt < nk; kt += 2) {
      step(kt, 0);
      step(kt + 1, 1);
    }
    if (valid) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v4f x[4];
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) x[e][s2] = -acc[h][s2][u][e];
          store_c_run(C + (cb + 4 * q + u) * BT + 64 * h, g, x);
        }
    }
    __syncthreads();  // every wave's last LDS read before the next super-tile's DMA
  }  // super-tiles of this workgroup
}

// Tile side 64 (small problems), on the matrix cores: one wave per 64 x 64
// output tile, four independent waves per workgroup (tile 4 w + wave), so a
// wave's whole 64 x 64 block is the tile and no workgroup barrier is needed.
// Each wave stages its own two panel slices through its own LDS (global
// loads, then LDS writes, then the fragment reads of the chunk), one chunk
// of KC panel columns at a time.
//   FP64 storage: v_mfma_f64_4x4x4_4b_f64 with the lane layout of the
//     128-tile FP64 kernel (acc[x][y] = -C(8 bq + 2g + (x&1) + 32(x>>1),
//     4y + jq)); chunks of 16 columns, LDS column pitch 68 doubles.
//   FP32 storage: v_mfma_f32_16x16x4_f32 with the layout of the 128-tile
//     FP32 kernel (acc[s2][u][e] = -C(16g + 4e + s2, 4q + u)), FP32
//     accumulation; chunks of 32 columns, unpadded LDS.
// The panel columns enter the accumulators in increasing order, so splitting
// a panel over several launches gives the bitwise same tile.
template <typename T>
__global__ __launch_bounds__(256) void update64_kernel(T *__restrict__ tiles, int64_t N,
                                                       int64_t p0, int pw, int64_t k0, int64_t K,
                                                       int mode, int S, int64_t G,
                                                       const int64_t *__restrict__ info) {
  constexpr int B = 64;
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int KC = F64 ? 16 : 32;     // panel columns per chunk (8 KB per operand)
  constexpr int LDP = F64 ? B + 4 : B;  // LDS column pitch (elements)
  if (*info != 0) return;
  __shared__ __attribute__((aligned(16))) T lds[4][2][KC * LDP];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t t = 4 * (int64_t)blockIdx.x + wv;
  if (t >= G) return;  // the whole wave
  int64_t ir, kr;
  if (mode == 0)
    map_triangle(t, N - k0, S, ir, kr);
  else
    map_band(t, K, ir, kr);
  const int64_t i = k0 + ir, k = k0 + kr;
  T *C = tiles + tile_index(i, k, N) * (int64_t)(B * B);
  T *la = lds[wv][0], *lb = lds[wv][1];
  const int g = lane >> 4, q = lane & 15;
  const int nch = pw * (B / KC);
  // chunk s: columns [KC s mod 64, +KC) of panel tile p0 + KC s / 64; lane
  // moves eight 16-byte pieces of each operand (column e / (64 / VE), rows
  // VE (e mod (64 / VE)) .. +VE-1 for piece e = 64 c + lane)
  auto stage = [&](int s) {
    constexpr int VE = 16 / sizeof(T), PPC = B / VE;  // elements per piece, pieces per column
    const int64_t p = p0 + (s * KC) / B;
    const int col0 = (s * KC) % B;
    const T *pa = tiles + tile_index(i, p, N) * (int64_t)(B * B) + col0 * B;
    const T *pb = tiles + tile_index(k, p, N) * (int64_t)(B * B) + col0 * B;
    v4u va[8], vb[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int e = 64 * c + lane, col = e / PPC, row = VE * (e % PPC);
      va[c] = *(const v4u *)(pa + col * B + row);
      vb[c] = *(const v4u *)(pb + col * B + row);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int e = 64 * c + lane, col = e / PPC, row = VE * (e % PPC);
      *(v4u *)(la + col * LDP + row) = va[c];
      *(v4u *)(lb + col * LDP + row) = vb[c];
    }
  };
  if constexpr (F64) {
    const int bq = q >> 2, jq = q & 3;
    double acc[4][16];
#pragma unroll
    for (int y = 0; y < 16; ++y) {
      const double *col = C + (4 * y + jq) * B + 8 * bq + 2 * g;
#pragma unroll
      for (int xh = 0; xh < 2; ++xh) {
        double v[2];
        *(uint4 *)&v[0] = *(const uint4 *)(col + 32 * xh);
        acc[2 * xh][y] = -v[0];
        acc[2 * xh + 1][y] = -v[1];
      }
    }
    for (int s = 0; s < nch; ++s) {
      stage(s);
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        const double *a = la + (4 * ks + g) * LDP + 2 * q;
        const double *b = lb + (4 * ks + g) * LDP + jq;
        double fa[4], fb[16];
        *(uint4 *)&fa[0] = *(const uint4 *)(a);
        *(uint4 *)&fa[2] = *(const uint4 *)(a + 32);
#pragma unroll
        for (int y = 0; y < 16; ++y) fb[y] = b[4 * y];
#pragma unroll
        for (int y = 0; y < 16; ++y)
#pragma unroll
          for (int x = 0; x < 4; ++x)
            acc[x][y] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[x], fb[y], acc[x][y], 0, 0, 0);
      }
    }
#pragma unroll
    for (int y = 0; y < 16; ++y) {
      double *col = C + (4 * y + jq) * B + 8 * bq + 2 * g;
#pragma unroll
      for (int xh = 0; xh < 2; ++xh) {
        double v[2] = {-acc[2 * xh][y], -acc[2 * xh + 1][y]};
        *(uint4 *)(col + 32 * xh) = *(const uint4 *)&v[0];
      }
    }
  } else {
    v4f acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v4f x[4];
      load_c_run(C + (4 * q + u) * B, g, x);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) acc[s2][u][e] = -x[e][s2];
    }
    for (int s = 0; s < nch; ++s) {
      stage(s);
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        float fa[4], fb[4];
        *(uint4 *)&fa[0] = *(const uint4 *)(la + (4 * ks + g) * LDP + 4 * q);
        *(uint4 *)&fb[0] = *(const uint4 *)(lb + (4 * ks + g) * LDP + 4 * q);
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[s2][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s2], fb[u], acc[s2][u], 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v4f x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) x[e][s2] = -acc[s2][u][e];
      store_c_run(C + (4 * q + u) * B, g, x);
    }
  }
}

}  // namespace

// 1: the FP16 form's whole-triangle updates use the 2 x 2-tile kernel
// (bitwise the same result as the one-tile kernel).
static int g_f16_wide = 1;
void set_f16_wide(int on) { g_f16_wide = on ? 1 : 0; }

void launch_update(void *tiles, int store, int b, int64_t N, int64_t p0, int pw, int64_t k0,
                   int64_t k1, int mode, int super_tile, int fp16, const int64_t *info,
                   hipStream_t s, int64_t max_wg, const void *p16, int64_t r0) {
  const int64_t R = N - k0;
  if (R <= 0 || pw <= 0) return;
  const int64_t K = k1 - k0;
  if (mode == 2) {
    // rectangle rows [r0, N) x columns [k0, k1), FP64 tile 128 only
    if (K <= 0 || r0 < k1 || r0 >= N || b != BT || store != STORE_F64 || fp16) return;
    const int64_t G = (N - r0) * K, G8 = (G + 7) / 8;
    hipLaunchKernelGGL(update_f64_kernel<2>, dim3((unsigned)(8 * G8)), dim3(256), 0, s,
                       (double *)tiles, N, p0, pw, k0, K, (int)(r0 - k0), G, G8, info);
    return;
  }
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
    int64_t nwg = 8 * G8;
    if (max_wg >= 8 && nwg > max_wg) nwg = (max_wg / 8) * 8;  // persistent: fewer workgroups
    const dim3 grid((unsigned)nwg);
    if (fp16 && !p16) return;  // the FP16 form needs its converted panel
    if (fp16 && mode == 0 && R >= 16 && g_f16_wide) {
      // 2 x 2 tiles per workgroup over the super-tile triangle
      const int64_t R2 = (R + 1) / 2, G2 = triangle_count(R2), G28 = (G2 + 7) / 8;
      int64_t nw = 8 * G28;
      if (max_wg >= 8 && nw > max_wg) nw = (max_wg / 8) * 8;
      const int S2 = super_tile > 1 ? super_tile / 2 : 1;
      hipLaunchKernelGGL(update_f16_wide_kernel, dim3((unsigned)nw), dim3(512), 0, s,
                         (float *)tiles, (const _Float16 *)p16, N, pw, k0, S2, G2, G28, info);
    } else if (fp16 && mode == 0)
      hipLaunchKernelGGL(update_f16_kernel<0>, grid, dim3(256), 0, s, (float *)tiles,
                         (const _Float16 *)p16, N, pw, k0, K, super_tile, G, G8, info);
    else if (fp16)
      hipLaunchKernelGGL(update_f16_kernel<1>, grid, dim3(256), 0, s, (float *)tiles,
                         (const _Float16 *)p16, N, pw, k0, K, super_tile, G, G8, info);
    else if (store == STORE_F64 && mode == 0)
      hipLaunchKernelGGL(update_f64_kernel<0>, grid, dim3(256), 0, s, (double *)tiles, N, p0, pw,
                         k0, K, super_tile, G, G8, info);
    else if (store == STORE_F64)
      hipLaunchKernelGGL(update_f64_kernel<1>, grid, dim3(256), 0, s, (double *)tiles, N, p0, pw,
                         k0, K, super_tile, G, G8, info);
    else if (mode == 0)
      hipLaunchKernelGGL(update_f32_kernel<0>, grid, dim3(256), 0, s, (float *)tiles, N, p0, pw,
                         k0, K, super_tile, G, G8, info);
    else
      hipLaunchKernelGGL(update_f32_kernel<1>, grid, dim3(256), 0, s, (float *)tiles, N, p0, pw,
                         k0, K, super_tile, G, G8, info);
  } else {
    const dim3 grid((unsigned)((G + 3) / 4));  // four tiles (waves) per workgroup
    if (store == STORE_F64)
      hipLaunchKernelGGL(update64_kernel<double>, grid, dim3(256), 0, s, (double *)tiles, N, p0,
                         pw, k0, K, mode, super_tile, G, info);
    else
      hipLaunchKernelGGL(update64_kernel<float>, grid, dim3(256), 0, s, (float *)tiles, N, p0, pw,
                         k0, K, mode, super_tile, G, info);
  }
}

void launch_batch_update(const BatchDesc *d, int upd_grid, int super_tile, hipStream_t s) {
  hipLaunchKernelGGL(update_f32_kernel<3>, dim3((unsigned)(upd_grid / 8 * 8)), dim3(256), 0, s,
                     (float *)d, (int64_t)0, (int64_t)0, 1, (int64_t)0, (int64_t)0, super_tile,
                     (int64_t)0, (int64_t)0, (const int64_t *)nullptr);
}

}  // namespace chol
