// MFMA GEMM for gfx950 with fused epilogues.
//
// C-tile 128 x 128 per workgroup of 256 threads (four wave64s in a 2 x 2
// arrangement, 64 x 64 per wave).  K-slabs are double-buffered in LDS with
// each operand stored k-contiguous, so a lane reads several k values of its
// row with one 128-bit LDS load, and the next slab's global loads are in
// flight during the current slab's MFMAs (one barrier per slab):
//   float : v_mfma_f32_32x32x2f32 (2 x 2 blocks of 32 x 32 per wave), slabs
//           of 32 (slabs of 16 and three workgroups per CU for launches of
//           2-3 tiles per CU)
//   double: v_mfma_f64_16x16x4f64 (4 x 4 blocks of 16 x 16 per wave), slabs
//           of 16
// B is the first MFMA operand, so the accumulator holds the tile transposed
// and the epilogue's accesses to C are coalesced.
// Column-major operands; op(A) is M x K, op(B) is K x N; batches via strides.
//
// The epilogue functor receives every output element (i, j) exactly once and
// returns a double that is summed over the workgroup (the residual epilogue
// uses this for ||R||_F^2; the others return 0).  In "tri" mode only tiles
// on or below the diagonal are launched (symmetric results) and the functor
// is told to mirror the element to (j, i).
#pragma once

#include <string>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace msqrt {

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
  static constexpr int TM = 32, TN = 32, TK = 2, NACC = 16, MB = 2, NB = 2;
  typedef float acc_t __attribute__((ext_vector_type(16)));
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  // operand fragment coordinates of lane l
  __device__ static inline int frag_mn(int l) { return l % 32; }
  __device__ static inline int frag_k(int l) { return l / 32; }
  // accumulator element r of lane l
  __device__ static inline int c_row(int l, int r) { return 8 * (r / 4) + 4 * (l / 32) + (r % 4); }
  __device__ static inline int c_col(int l, int) { return l % 32; }
};

template <>
struct Mfma<double> {
  static constexpr int TM = 16, TN = 16, TK = 4, NACC = 4, MB = 4, NB = 4;
  typedef double acc_t __attribute__((ext_vector_type(4)));
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int frag_mn(int l) { return l % 16; }
  __device__ static inline int frag_k(int l) { return l / 16; }
  __device__ static inline int c_row(int l, int r) { return (l / 16) + 4 * r; }
  __device__ static inline int c_col(int l, int) { return l % 16; }
};

struct GemmShape {
  int M, N, K;
  int K_last;     // K of the last batch entry (split-K over a ragged range)
  int64_t lda, ldb, sA, sB;
  int tri;        // launch only tiles with tile_m >= tile_n
  int tiles_m, tiles_n, ntiles, per_xcd;
};

constexpr int GBM = 128, GBN = 128, GTHREADS = 256;
// tile of the wide kernels for large symmetric-output products, and the
// smallest order of a triangle that takes them
constexpr int WBM = 192;
constexpr int kWideMin = 1536;

// Epilogues that define kPrefetch = true also provide pre(b, i, j), a load
// issued for every element of a block before post(b, i, j, v, mir, pre)
// stores any of them.
template <class Epi, class = void>
struct EpiPrefetches : std::false_type {};
template <class Epi>
struct EpiPrefetches<Epi, std::void_t<decltype(Epi::kPrefetch)>>
    : std::integral_constant<bool, Epi::kPrefetch> {};

// Epilogues that define kStaged = true are written by the float kernels with
// 32 x 32 accumulator blocks through epi_block_staged.  They provide
//   out_t                          the type stored,
//   bool live(b)                   false: batch entry b is left untouched,
//   out_t* dst(b), int64_t ld()    the output of entry b,
//   double load(b, i, j)           what value() needs from memory at (i, j),
//   out_t value(b, i, j, v, x)     the element stored at (i, j), and at (j, i)
//                                  for a symmetric output (x = load(b, i, j)).
template <class Epi, class = void>
struct EpiStages : std::false_type {};
template <class Epi>
struct EpiStages<Epi, std::void_t<decltype(Epi::kStaged)>> : std::integral_constant<bool, Epi::kStaged> {};

// One 32 x 32 output block of a float MFMA kernel whose accumulator holds
// element (gi0 + l % 32, gj0 + c_row(l, r)) in lane l, register r.  Every
// load of the block is issued before any store.  The direct store is
// coalesced (32 consecutive rows per half-wave).  For a symmetric output the
// mirror (j, i) is written from the wave's own LDS block st (32 x 33 out_t),
// read in transposed order, so those stores are coalesced too instead of
// touching 32 rows per store instruction.
constexpr int kStageLd = 33;

template <class Epi, class Acc>
__device__ inline void epi_block_staged(const GemmShape& s, const Epi& epi, int b, int gi0, int gj0,
                                        const Acc& acc, typename Epi::out_t* st, int lane) {
  using O = typename Epi::out_t;
  using M = Mfma<float>;
  static_assert(M::TM == 32 && M::TN == 32 && M::NACC == 16, "32 x 32 accumulator blocks");
  if (s.tri && gi0 + 31 < gj0) return;  // block above the diagonal (wave-uniform)
  O* dst = epi.dst(b);
  const int64_t ld = epi.ld();
  const int gi = gi0 + lane % 32;
  double x0[M::NACC];
#pragma unroll
  for (int r = 0; r < M::NACC; ++r) {
    const int gj = gj0 + M::c_row(lane, r);
    const bool ok = gi < s.M && gj < s.N && !(s.tri && gi < gj);
    x0[r] = ok ? epi.load(b, gi, gj) : 0.0;
  }
#pragma unroll
  for (int r = 0; r < M::NACC; ++r) {
    const int gj = gj0 + M::c_row(lane, r);
    const bool ok = gi < s.M && gj < s.N && !(s.tri && gi < gj);
    const O x = ok ? epi.value(b, gi, gj, acc[r], x0[r]) : O(0);
    if (ok) dst[gi + (int64_t)gj * ld] = x;
    if (s.tri) st[(lane % 32) * kStageLd + M::c_row(lane, r)] = x;
  }
  if (!s.tri) return;
  // other lanes of the same wave read what was just written
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int li = 2 * q + lane / 32, lj = lane % 32;
    const int mi = gi0 + li, mj = gj0 + lj;
    if (mi < s.M && mj < s.N && mi > mj) dst[mj + (int64_t)mi * ld] = st[li * kStageLd + lj];
  }
  // the next block's writes to st follow these reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Maps the hardware workgroup id to a tile id so that each of the 8 XCDs
// (workgroups are dispatched round-robin over XCDs) works on a contiguous
// range of tiles, then the tile id to (tile_m, tile_n).
__device__ inline bool gemm_tile_coords(const GemmShape& s, int& tm, int& tn) {
  const int b = blockIdx.x;
  const int id = (b % 8) * s.per_xcd + b / 8;
  if (id >= s.ntiles) return false;
  if (s.tri) {
    // id -> (tm, tn), tm >= tn, row-major over the lower triangle of tiles.
    int r = (int)((sqrt(8.0 * id + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= id) ++r;
    while (r * (r + 1) / 2 > id) --r;
    tm = r;
    tn = id - r * (r + 1) / 2;
    return true;
  }
  // Grouped ordering: 8 tile-rows per group, walking columns within a group.
  const int GM = 8;
  const int per_group = GM * s.tiles_n;
  const int g = id / per_group;
  const int first = g * GM;
  const int gsz = min(s.tiles_m - first, GM);
  const int w = id % per_group;
  tm = first + w % gsz;
  tn = w / gsz;
  return true;
}


// ---------------------------------------------------------------------------
// Float kernel with a deeper pipeline: K-slabs of 32 double-buffered in LDS
// (the next slab's global loads are in flight during the current slab's
// MFMAs and land in the other buffer, one barrier per slab), each operand
// stored k-contiguous ([row][k], row stride 36 floats) so a lane reads four
// k values of its row with one 128-bit LDS load.  Within a slab, lane half h
// of a wave supplies k = 16 h + s at MFMA step s (A and B use the same
// assignment, so every k is summed once).

constexpr int FBK = 32, FLD = FBK + 4;
constexpr size_t kGemmF32Lds = (size_t)2 * 2 * GBM * FLD * sizeof(float);
static_assert(GBM == GBN, "square tiles");

// One operand slab (128 rows x 32 k) of op(X): element (r, k) is
// X[r + k ld] when rows are contiguous (RC), else X[k + r ld].
template <bool RC>
__device__ inline void f32_slab_load(const float* __restrict__ X, int64_t ld, int r0, int R, int k0,
                                     int K, int t, float (&v)[16]) {
  const int lane = t % kWave, wave = t / kWave;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int r, k;
    if (RC) {
      // 8 rows x 8 k per wave instruction: 32-byte row segments, 2-way LDS
      // bank use on the store
      const int id = wave * 16 + e;
      r = (id % 16) * 8 + lane % 8;
      k = (id / 16) * 8 + lane / 8;
    } else {
      const int idx = t + GTHREADS * e;
      k = idx % FBK;
      r = idx / FBK;
    }
    const int gr = r0 + r, gk = k0 + k;
    v[e] = (gr < R && gk < K) ? (RC ? X[gr + (int64_t)gk * ld] : X[gk + (int64_t)gr * ld]) : 0.f;
  }
}

template <bool RC>
__device__ inline void f32_slab_store(float* Xs, int t, const float (&v)[16]) {
  const int lane = t % kWave, wave = t / kWave;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    int r, k;
    if (RC) {
      const int id = wave * 16 + e;
      r = (id % 16) * 8 + lane % 8;
      k = (id / 16) * 8 + lane / 8;
    } else {
      const int idx = t + GTHREADS * e;
      k = idx % FBK;
      r = idx / FBK;
    }
    Xs[r * FLD + k] = v[e];
  }
}

template <bool TA, bool TB, class Epi>
__global__ __launch_bounds__(GTHREADS, 2) void gemm_f32_kernel(GemmShape s, const float* __restrict__ A,
                                                               const float* __restrict__ B, Epi epi,
                                                               double* __restrict__ partials) {
  using M = Mfma<float>;
  extern __shared__ __attribute__((aligned(16))) float gemm_lds[];
  __shared__ double red[GTHREADS / kWave];
  // [buffer][operand][row][k]
  auto slab = [&](int buf, int op) { return gemm_lds + (size_t)(buf * 2 + op) * GBM * FLD; };

  int tm, tn;
  if (!gemm_tile_coords(s, tm, tn)) return;
  const int batch = blockIdx.y;
  const int K = (batch == (int)gridDim.y - 1) ? s.K_last : s.K;
  A += (int64_t)batch * s.sA;
  B += (int64_t)batch * s.sB;
  const int m0 = tm * GBM, n0 = tn * GBN;
  const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const int wm = wave % 2, wn = wave / 2;
  // op(A) rows are contiguous unless A is transposed; op(B)^T rows (the
  // columns n of op(B)) are contiguous when B is transposed
  constexpr bool ARC = !TA, BRC = TB;

  typename M::acc_t acc[M::MB][M::NB];
#pragma unroll
  for (int i = 0; i < M::MB; ++i)
#pragma unroll
    for (int j = 0; j < M::NB; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[i][j][r] = 0.f;

  float ra[16], rb[16];
  if (K > 0) {
    f32_slab_load<ARC>(A, s.lda, m0, s.M, 0, K, t, ra);
    f32_slab_load<BRC>(B, s.ldb, n0, s.N, 0, K, t, rb);
    f32_slab_store<ARC>(slab(0, 0), t, ra);
    f32_slab_store<BRC>(slab(0, 1), t, rb);
  }
  __syncthreads();
  const int h = lane / 32, fr = lane % 32;
  for (int k0 = 0, buf = 0; k0 < K; k0 += FBK, buf ^= 1) {
    const bool more = k0 + FBK < K;
    if (more) {
      f32_slab_load<ARC>(A, s.lda, m0, s.M, k0 + FBK, K, t, ra);
      f32_slab_load<BRC>(B, s.ldb, n0, s.N, k0 + FBK, K, t, rb);
    }
    const float* As = slab(buf, 0);
    const float* Bs = slab(buf, 1);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kc = h * 16 + s4 * 4;
      float4 a4[M::MB], b4[M::NB];
#pragma unroll
      for (int i = 0; i < M::MB; ++i)
        a4[i] = *reinterpret_cast<const float4*>(As + (wm * 64 + i * 32 + fr) * FLD + kc);
#pragma unroll
      for (int j = 0; j < M::NB; ++j)
        b4[j] = *reinterpret_cast<const float4*>(Bs + (wn * 64 + j * 32 + fr) * FLD + kc);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < M::MB; ++i)
#pragma unroll
          for (int j = 0; j < M::NB; ++j) {
            const float av = c == 0 ? a4[i].x : c == 1 ? a4[i].y : c == 2 ? a4[i].z : a4[i].w;
            const float bv = c == 0 ? b4[j].x : c == 1 ? b4[j].y : c == 2 ? b4[j].z : b4[j].w;
            // B as the first operand: the accumulator holds the tile
            // transposed, lane l on row l % 32 of C, so the epilogue's loads
            // and stores of C are 128-byte coalesced
            acc[i][j] = M::mma(bv, av, acc[i][j]);
          }
    }
    if (more) {
      f32_slab_store<ARC>(slab(buf ^ 1, 0), t, ra);
      f32_slab_store<BRC>(slab(buf ^ 1, 1), t, rb);
    }
    __syncthreads();
  }

  double part = 0.0;
#pragma unroll
  for (int i = 0; i < M::MB; ++i)
#pragma unroll
    for (int j = 0; j < M::NB; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) {
        const int gi = m0 + wm * 64 + i * M::TM + M::c_col(lane, r);
        const int gj = n0 + wn * 64 + j * M::TN + M::c_row(lane, r);
        if (gi < s.M && gj < s.N) {
          if (s.tri && gi < gj) continue;
          part += epi(batch, gi, gj, acc[i][j][r], s.tri && gi != gj);
        }
      }
  if (Epi::kReduces) {
    part = block_sum(part, red);
    if (t == 0) {
      const int id = (blockIdx.x % 8) * s.per_xcd + blockIdx.x / 8;
      partials[(int64_t)batch * s.ntiles + id] = part;
    }
  }
}

// Double kernel of the same design: K-slabs of 16 double-buffered in LDS,
// k-contiguous rows (stride 18 doubles), v_mfma_f64_16x16x4f64 with lane
// quarter h supplying k = 4 h + s at step s, so a lane reads its four k
// values of a row with two 128-bit LDS loads; B is the first MFMA operand,
// so the epilogue's accesses to C are coalesced.
constexpr int DBK = 16, DLD = DBK + 2;
constexpr size_t kGemmF64Lds = (size_t)2 * 2 * GBM * DLD * sizeof(double);

template <bool RC>
__device__ inline void f64_slab_index(int t, int e, int& r, int& k) {
  const int lane = t % kWave, wave = t / kWave;
  if (RC) {
    const int id = wave * 8 + e;  // 32 blocks of 8 rows x 8 k
    r = (id % 16) * 8 + lane % 8;
    k = (id / 16) * 8 + lane / 8;
  } else {
    const int idx = t + GTHREADS * e;
    k = idx % DBK;
    r = idx / DBK;
  }
}

template <bool RC>
__device__ inline void f64_slab_load(const double* __restrict__ X, int64_t ld, int r0, int R, int k0,
                                     int K, int t, double (&v)[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int r, k;
    f64_slab_index<RC>(t, e, r, k);
    const int gr = r0 + r, gk = k0 + k;
    v[e] = (gr < R && gk < K) ? (RC ? X[gr + (int64_t)gk * ld] : X[gk + (int64_t)gr * ld]) : 0.0;
  }
}

template <bool RC>
__device__ inline void f64_slab_store(double* Xs, int t, const double (&v)[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int r, k;
    f64_slab_index<RC>(t, e, r, k);
    Xs[r * DLD + k] = v[e];
  }
}

template <bool TA, bool TB, class Epi>
__global__ __launch_bounds__(GTHREADS, 2) void gemm_f64_kernel(GemmShape s, const double* __restrict__ A,
                                                               const double* __restrict__ B, Epi epi,
                                                               double* __restrict__ partials) {
  using M = Mfma<double>;
  extern __shared__ __attribute__((aligned(16))) double gemm_lds64[];
  __shared__ double red[GTHREADS / kWave];
  auto slab = [&](int buf, int op) { return gemm_lds64 + (size_t)(buf * 2 + op) * GBM * DLD; };

  int tm, tn;
  if (!gemm_tile_coords(s, tm, tn)) return;
  const int batch = blockIdx.y;
  const int K = (batch == (int)gridDim.y - 1) ? s.K_last : s.K;
  A += (int64_t)batch * s.sA;
  B += (int64_t)batch * s.sB;
  const int m0 = tm * GBM, n0 = tn * GBN;
  const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const int wm = wave % 2, wn = wave / 2;
  constexpr bool ARC = !TA, BRC = TB;

  typename M::acc_t acc[M::MB][M::NB];
#pragma unroll
  for (int i = 0; i < M::MB; ++i)
#pragma unroll
    for (int j = 0; j < M::NB; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[i][j][r] = 0.0;

  double ra[8], rb[8];
  if (K > 0) {
    f64_slab_load<ARC>(A, s.lda, m0, s.M, 0, K, t, ra);
    f64_slab_load<BRC>(B, s.ldb, n0, s.N, 0, K, t, rb);
    f64_slab_store<ARC>(slab(0, 0), t, ra);
    f64_slab_store<BRC>(slab(0, 1), t, rb);
  }
  __syncthreads();
  const int h = lane / 16, fr = lane % 16;
  for (int k0 = 0, buf = 0; k0 < K; k0 += DBK, buf ^= 1) {
    const bool more = k0 + DBK < K;
    if (more) {
      f64_slab_load<ARC>(A, s.lda, m0, s.M, k0 + DBK, K, t, ra);
      f64_slab_load<BRC>(B, s.ldb, n0, s.N, k0 + DBK, K, t, rb);
    }
    const double* As = slab(buf, 0);
    const double* Bs = slab(buf, 1);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int kc = h * 4 + half * 2;
      double2 a2[M::MB], b2[M::NB];
#pragma unroll
      for (int i = 0; i < M::MB; ++i)
        a2[i] = *reinterpret_cast<const double2*>(As + (wm * 64 + i * 16 + fr) * DLD + kc);
#pragma unroll
      for (int j = 0; j < M::NB; ++j)
        b2[j] = *reinterpret_cast<const double2*>(Bs + (wn * 64 + j * 16 + fr) * DLD + kc);
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < M::MB; ++i)
#pragma unroll
          for (int j = 0; j < M::NB; ++j)
            acc[i][j] = M::mma(c == 0 ? b2[j].x : b2[j].y, c == 0 ? a2[i].x : a2[i].y, acc[i][j]);
    }
    if (more) {
      f64_slab_store<ARC>(slab(buf ^ 1, 0), t, ra);
      f64_slab_store<BRC>(slab(buf ^ 1, 1), t, rb);
    }
    __syncthreads();
  }

  double part = 0.0;
#pragma unroll
  for (int i = 0; i < M::MB; ++i)
#pragma unroll
    for (int j = 0; j < M::NB; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) {
        const int gi = m0 + wm * 64 + i * M::TM + M::c_col(lane, r);
        const int gj = n0 + wn * 64 + j * M::TN + M::c_row(lane, r);
        if (gi < s.M && gj < s.N) {
          if (s.tri && gi < gj) continue;
          part += epi(batch, gi, gj, acc[i][j][r], s.tri && gi != gj);
        }
      }
  if (Epi::kReduces) {
    part = block_sum(part, red);
    if (t == 0) {
      const int id = (blockIdx.x % 8) * s.per_xcd + blockIdx.x / 8;
      partials[(int64_t)batch * s.ntiles + id] = part;
    }
  }
}

// Double kernel with 192 x 192 tiles for large symmetric-output products
// (the float64 residual A - X X^T of the SPD route): a triangle of 128-tiles
// at n = 4096 has 528 tiles, two workgroups per CU hold 512 and the last 16
// run in a second, nearly empty round; 192-tiles give 253, one per CU.
// Eight waves in a 2 x 4 arrangement, 96 x 48 each (6 x 3 blocks of
// v_mfma_f64_16x16x4f64), K-slabs of 16.
constexpr int kW64Threads = 512;
constexpr size_t kGemmF64wLds = (size_t)2 * 2 * WBM * DLD * sizeof(double);

template <bool RC>
__device__ inline void f64w_slab_index(int t, int e, int& r, int& k) {
  const int lane = t % kWave, wave = t / kWave;
  if (RC) {
    const int id = wave * 6 + e;  // 48 blocks of 8 rows x 8 k
    r = (id % 24) * 8 + lane % 8;
    k = (id / 24) * 8 + lane / 8;
  } else {
    const int idx = t + kW64Threads * e;
    k = idx % DBK;
    r = idx / DBK;
  }
}

template <bool RC>
__device__ inline void f64w_slab_load(const double* __restrict__ X, int64_t ld, int r0, int R, int k0,
                                      int K, int t, double (&v)[6]) {
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    int r, k;
    f64w_slab_index<RC>(t, e, r, k);
    const int gr = r0 + r, gk = k0 + k;
    v[e] = (gr < R && gk < K) ? (RC ? X[gr + (int64_t)gk * ld] : X[gk + (int64_t)gr * ld]) : 0.0;
  }
}

template <bool RC>
__device__ inline void f64w_slab_store(double* Xs, int t, const double (&v)[6]) {
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    int r, k;
    f64w_slab_index<RC>(t, e, r, k);
    Xs[r * DLD + k] = v[e];
  }
}

template <bool TA, bool TB, class Epi>
__global__ __launch_bounds__(kW64Threads, 1) void gemm_f64w_kernel(GemmShape s, const double* __restrict__ A,
                                                                   const double* __restrict__ B, Epi epi,
                                                                   double* __restrict__ partials) {
  using M = Mfma<double>;
  constexpr int MBW = 6, NBW = 3;  // 16 x 16 blocks per wave: 6 down, 3 across
  extern __shared__ __attribute__((aligned(16))) double gemm_lds64w[];
  __shared__ double red[kW64Threads / kWave];
  auto slab = [&](int buf, int op) { return gemm_lds64w + (size_t)(buf * 2 + op) * WBM * DLD; };

  int tm, tn;
  if (!gemm_tile_coords(s, tm, tn)) return;
  const int batch = blockIdx.y;
  const int K = (batch == (int)gridDim.y - 1) ? s.K_last : s.K;
  A += (int64_t)batch * s.sA;
  B += (int64_t)batch * s.sB;
  const int m0 = tm * WBM, n0 = tn * WBM;
  const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const int wm = wave % 2, wn = wave / 2;  // rows wm * 96, columns wn * 48
  constexpr bool ARC = !TA, BRC = TB;

  typename M::acc_t acc[MBW][NBW];
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[i][j][r] = 0.0;

  double ra[6], rb[6];
  if (K > 0) {
    f64w_slab_load<ARC>(A, s.lda, m0, s.M, 0, K, t, ra);
    f64w_slab_load<BRC>(B, s.ldb, n0, s.N, 0, K, t, rb);
    f64w_slab_store<ARC>(slab(0, 0), t, ra);
    f64w_slab_store<BRC>(slab(0, 1), t, rb);
  }
  __syncthreads();
  const int h = lane / 16, fr = lane % 16;
  for (int k0 = 0, buf = 0; k0 < K; k0 += DBK, buf ^= 1) {
    const bool more = k0 + DBK < K;
    if (more) {
      f64w_slab_load<ARC>(A, s.lda, m0, s.M, k0 + DBK, K, t, ra);
      f64w_slab_load<BRC>(B, s.ldb, n0, s.N, k0 + DBK, K, t, rb);
    }
    const double* As = slab(buf, 0);
    const double* Bs = slab(buf, 1);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int kc = h * 4 + half * 2;
      double2 a2[MBW], b2[NBW];
#pragma unroll
      for (int i = 0; i < MBW; ++i)
        a2[i] = *reinterpret_cast<const double2*>(As + (wm * 96 + i * 16 + fr) * DLD + kc);
#pragma unroll
      for (int j = 0; j < NBW; ++j)
        b2[j] = *reinterpret_cast<const double2*>(Bs + (wn * 48 + j * 16 + fr) * DLD + kc);
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < MBW; ++i)
#pragma unroll
          for (int j = 0; j < NBW; ++j)
            acc[i][j] = M::mma(c == 0 ? b2[j].x : b2[j].y, c == 0 ? a2[i].x : a2[i].y, acc[i][j]);
    }
    if (more) {
      f64w_slab_store<ARC>(slab(buf ^ 1, 0), t, ra);
      f64w_slab_store<BRC>(slab(buf ^ 1, 1), t, rb);
    }
    __syncthreads();
  }

  double part = 0.0;
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) {
        const int gi = m0 + wm * 96 + i * M::TM + M::c_col(lane, r);
        const int gj = n0 + wn * 48 + j * M::TN + M::c_row(lane, r);
        if (gi < s.M && gj < s.N) {
          if (s.tri && gi < gj) continue;
          part += epi(batch, gi, gj, acc[i][j][r], s.tri && gi != gj);
        }
      }
  if (Epi::kReduces) {
    part = block_sum(part, red);
    if (t == 0) {
      const int id = (blockIdx.x % 8) * s.per_xcd + blockIdx.x / 8;
      partials[(int64_t)batch * s.ntiles + id] = part;
    }
  }
}

// Float kernel for launches slightly larger than two workgroups per CU
// (a triangle of 528 tiles at n = 4096 leaves 16 tiles for a second round):
// K-slabs of 16 double-buffered (40 KiB of LDS, at most 170 registers), so
// three workgroups share a CU and the whole launch runs in one round.
constexpr int HBK = 16, HLD = HBK + 4;
constexpr size_t kGemmF32k16Lds = (size_t)2 * 2 * GBM * HLD * sizeof(float);

template <bool RC>
__device__ inline void f32h_slab_load(const float* __restrict__ X, int64_t ld, int r0, int R, int k0,
                                      int K, int t, float (&v)[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int r, k;
    f64_slab_index<RC>(t, e, r, k);  // same 128 x 16 slab geometry
    const int gr = r0 + r, gk = k0 + k;
    v[e] = (gr < R && gk < K) ? (RC ? X[gr + (int64_t)gk * ld] : X[gk + (int64_t)gr * ld]) : 0.f;
  }
}

template <bool RC>
__device__ inline void f32h_slab_store(float* Xs, int t, const float (&v)[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int r, k;
    f64_slab_index<RC>(t, e, r, k);
    Xs[r * HLD + k] = v[e];
  }
}

template <bool TA, bool TB, class Epi>
__global__ __launch_bounds__(GTHREADS, 3) void gemm_f32k16_kernel(GemmShape s, const float* __restrict__ A,
                                                                  const float* __restrict__ B, Epi epi,
                                                                  double* __restrict__ partials) {
  using M = Mfma<float>;
  extern __shared__ __attribute__((aligned(16))) float gemm_lds16[];
  __shared__ double red[GTHREADS / kWave];
  auto slab = [&](int buf, int op) { return gemm_lds16 + (size_t)(buf * 2 + op) * GBM * HLD; };

  int tm, tn;
  if (!gemm_tile_coords(s, tm, tn)) return;
  const int batch = blockIdx.y;
  const int K = (batch == (int)gridDim.y - 1) ? s.K_last : s.K;
  A += (int64_t)batch * s.sA;
  B += (int64_t)batch * s.sB;
  const int m0 = tm * GBM, n0 = tn * GBN;
  const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const int wm = wave % 2, wn = wave / 2;
  constexpr bool ARC = !TA, BRC = TB;

  typename M::acc_t acc[M::MB][M::NB];
#pragma unroll
  for (int i = 0; i < M::MB; ++i)
#pragma unroll
    for (int j = 0; j < M::NB; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[i][j][r] = 0.f;

  float ra[8], rb[8];
  if (K > 0) {
    f32h_slab_load<ARC>(A, s.lda, m0, s.M, 0, K, t, ra);
    f32h_slab_load<BRC>(B, s.ldb, n0, s.N, 0, K, t, rb);
    f32h_slab_store<ARC>(slab(0, 0), t, ra);
    f32h_slab_store<BRC>(slab(0, 1), t, rb);
  }
  __syncthreads();
  // lane half h supplies k = 8 h + s at step s
  const int h = lane / 32, fr = lane % 32;
  for (int k0 = 0, buf = 0; k0 < K; k0 += HBK, buf ^= 1) {
    const bool more = k0 + HBK < K;
    if (more) {
      f32h_slab_load<ARC>(A, s.lda, m0, s.M, k0 + HBK, K, t, ra);
      f32h_slab_load<BRC>(B, s.ldb, n0, s.N, k0 + HBK, K, t, rb);
    }
    const float* As = slab(buf, 0);
    const float* Bs = slab(buf, 1);
#pragma unroll
    for (int s4 = 0; s4 < 2; ++s4) {
      const int kc = h * 8 + s4 * 4;
      float4 a4[M::MB], b4[M::NB];
#pragma unroll
      for (int i = 0; i < M::MB; ++i)
        a4[i] = *reinterpret_cast<const float4*>(As + (wm * 64 + i * 32 + fr) * HLD + kc);
#pragma unroll
      for (int j = 0; j < M::NB; ++j)
        b4[j] = *reinterpret_cast<const float4*>(Bs + (wn * 64 + j * 32 + fr) * HLD + kc);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < M::MB; ++i)
#pragma unroll
          for (int j = 0; j < M::NB; ++j) {
            const float av = c == 0 ? a4[i].x : c == 1 ? a4[i].y : c == 2 ? a4[i].z : a4[i].w;
            const float bv = c == 0 ? b4[j].x : c == 1 ? b4[j].y : c == 2 ? b4[j].z : b4[j].w;
            acc[i][j] = M::mma(bv, av, acc[i][j]);
          }
    }
    if (more) {
      f32h_slab_store<ARC>(slab(buf ^ 1, 0), t, ra);
      f32h_slab_store<BRC>(slab(buf ^ 1, 1), t, rb);
    }
    __syncthreads();
  }

  double part = 0.0;
#pragma unroll
  for (int i = 0; i < M::MB; ++i)
#pragma unroll
    for (int j = 0; j < M::NB; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) {
        const int gi = m0 + wm * 64 + i * M::TM + M::c_col(lane, r);
        const int gj = n0 + wn * 64 + j * M::TN + M::c_row(lane, r);
        if (gi < s.M && gj < s.N) {
          if (s.tri && gi < gj) continue;
          part += epi(batch, gi, gj, acc[i][j][r], s.tri && gi != gj);
        }
      }
  if (Epi::kReduces) {
    part = block_sum(part, red);
    if (t == 0) {
      const int id = (blockIdx.x % 8) * s.per_xcd + blockIdx.x / 8;
      partials[(int64_t)batch * s.ntiles + id] = part;
    }
  }
}

// ---------------------------------------------------------------------------
// Float kernel with 192 x 192 tiles: one workgroup of four wave64s per CU,
// each wave a 96 x 96 block (3 x 3 MFMA 32 x 32 blocks, 144 accumulator
// registers), K-slabs of 32 double-buffered in LDS as in the 128 kernel
// (110 KiB).  It serves the large symmetric-output products: at n = 4096 the
// lower triangle has 253 tiles of 192 (one per CU) against 528 of 128
// (2.06 per CU, so some CUs run a third tile while the rest idle); measured
// 0.78 ms against 1.01 ms for the n^3 flops of one such product.
//
// The same kernel with 256 x 256 tiles (each wave 128 x 128: 4 x 4 blocks,
// 256 accumulator registers, which the MFMA instructions take from the
// accumulation register file; 144 KiB of slabs) serves large full products
// (single products with K >= 2048) whose 256-tiles fill one round on the CUs
// where the 128 kernel needs two:
// at n = 4096 the 256 tiles of 256 against 1024 of 128 (1.27 against 1.36 ms
// per product).

template <int WB>
constexpr size_t f32w_lds() { return (size_t)2 * 2 * WB * FLD * sizeof(float); }
constexpr size_t kGemmF32wLds = f32w_lds<WBM>();
constexpr int WBX = 256;

template <bool RC, int WB>
__device__ inline void f32w_slab_index(int t, int e, int& r, int& k) {
  constexpr int SL = WB * FBK / GTHREADS;  // slab elements per thread
  const int lane = t % kWave, wave = t / kWave;
  if (RC) {
    // WB / 2 blocks of 8 rows x 8 k, SL per wave
    const int id = wave * SL + e;
    r = (id % (WB / 8)) * 8 + lane % 8;
    k = (id / (WB / 8)) * 8 + lane / 8;
  } else {
    const int idx = t + GTHREADS * e;
    k = idx % FBK;
    r = idx / FBK;
  }
}

template <bool RC, int WB>
__device__ inline void f32w_slab_load(const float* __restrict__ X, int64_t ld, int r0, int R, int k0,
                                      int K, int t, float (&v)[WB * FBK / GTHREADS]) {
#pragma unroll
  for (int e = 0; e < WB * FBK / GTHREADS; ++e) {
    int r, k;
    f32w_slab_index<RC, WB>(t, e, r, k);
    const int gr = r0 + r, gk = k0 + k;
    v[e] = (gr < R && gk < K) ? (RC ? X[gr + (int64_t)gk * ld] : X[gk + (int64_t)gr * ld]) : 0.f;
  }
}

template <bool RC, int WB>
__device__ inline void f32w_slab_store(float* Xs, int t, const float (&v)[WB * FBK / GTHREADS]) {
#pragma unroll
  for (int e = 0; e < WB * FBK / GTHREADS; ++e) {
    int r, k;
    f32w_slab_index<RC, WB>(t, e, r, k);
    Xs[r * FLD + k] = v[e];
  }
}

template <bool TA, bool TB, class Epi, int WB = WBM>
__global__ __launch_bounds__(GTHREADS, 1) void gemm_f32w_kernel(GemmShape s, const float* __restrict__ A,
                                                                const float* __restrict__ B, Epi epi,
                                                                double* __restrict__ partials) {
  using M = Mfma<float>;
  constexpr int NBW = WB / 64;      // 32 x 32 blocks per wave side
  constexpr int HW = WB / 2;        // wave block side
  constexpr int SL = WB * FBK / GTHREADS;
  static_assert(WB % 64 == 0 && SL * GTHREADS == WB * FBK, "tile size");
  extern __shared__ __attribute__((aligned(16))) float gemm_ldsw[];
  __shared__ double red[GTHREADS / kWave];
  auto slab = [&](int buf, int op) { return gemm_ldsw + (size_t)(buf * 2 + op) * WB * FLD; };

  int tm, tn;
  if (!gemm_tile_coords(s, tm, tn)) return;
  const int batch = blockIdx.y;
  const int K = (batch == (int)gridDim.y - 1) ? s.K_last : s.K;
  A += (int64_t)batch * s.sA;
  B += (int64_t)batch * s.sB;
  const int m0 = tm * WB, n0 = tn * WB;
  const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const int wm = wave % 2, wn = wave / 2;
  constexpr bool ARC = !TA, BRC = TB;

  typename M::acc_t acc[NBW][NBW];
#pragma unroll
  for (int i = 0; i < NBW; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[i][j][r] = 0.f;

  float ra[SL], rb[SL];
  if (K > 0) {
    f32w_slab_load<ARC, WB>(A, s.lda, m0, s.M, 0, K, t, ra);
    f32w_slab_load<BRC, WB>(B, s.ldb, n0, s.N, 0, K, t, rb);
    f32w_slab_store<ARC, WB>(slab(0, 0), t, ra);
    f32w_slab_store<BRC, WB>(slab(0, 1), t, rb);
  }
  __syncthreads();
  const int h = lane / 32, fr = lane % 32;
  for (int k0 = 0, buf = 0; k0 < K; k0 += FBK, buf ^= 1) {
    const bool more = k0 + FBK < K;
    if (more) {
      f32w_slab_load<ARC, WB>(A, s.lda, m0, s.M, k0 + FBK, K, t, ra);
      f32w_slab_load<BRC, WB>(B, s.ldb, n0, s.N, k0 + FBK, K, t, rb);
    }
    const float* As = slab(buf, 0);
    const float* Bs = slab(buf, 1);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kc = h * 16 + s4 * 4;
      float4 a4[NBW], b4[NBW];
#pragma unroll
      for (int i = 0; i < NBW; ++i)
        a4[i] = *reinterpret_cast<const float4*>(As + (wm * HW + i * 32 + fr) * FLD + kc);
#pragma unroll
      for (int j = 0; j < NBW; ++j)
        b4[j] = *reinterpret_cast<const float4*>(Bs + (wn * HW + j * 32 + fr) * FLD + kc);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < NBW; ++i)
#pragma unroll
          for (int j = 0; j < NBW; ++j) {
            const float av = c == 0 ? a4[i].x : c == 1 ? a4[i].y : c == 2 ? a4[i].z : a4[i].w;
            const float bv = c == 0 ? b4[j].x : c == 1 ? b4[j].y : c == 2 ? b4[j].z : b4[j].w;
            acc[i][j] = M::mma(bv, av, acc[i][j]);
          }
    }
    if (more) {
      f32w_slab_store<ARC, WB>(slab(buf ^ 1, 0), t, ra);
      f32w_slab_store<BRC, WB>(slab(buf ^ 1, 1), t, rb);
    }
    __syncthreads();
  }

  if constexpr (EpiStages<Epi>::value) {
    static_assert(!Epi::kReduces, "staged epilogues return no sums");
    static_assert((size_t)(GTHREADS / kWave) * 32 * kStageLd * sizeof(typename Epi::out_t) <= f32w_lds<WB>(),
                  "staging blocks fit the slab buffers");
    // the slab buffers are free: the last slab ended with a barrier
    if (!epi.live(batch)) return;
    typename Epi::out_t* st = reinterpret_cast<typename Epi::out_t*>(gemm_ldsw) + wave * 32 * kStageLd;
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int j = 0; j < NBW; ++j)
        epi_block_staged(s, epi, batch, m0 + wm * HW + i * M::TM, n0 + wn * HW + j * M::TN, acc[i][j], st, lane);
    return;
  }
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < NBW; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
      if constexpr (EpiPrefetches<Epi>::value) {
        // every load of the block first, then the stores
        double x0[M::NACC];
#pragma unroll
        for (int r = 0; r < M::NACC; ++r) {
          const int gi = m0 + wm * HW + i * M::TM + M::c_col(lane, r);
          const int gj = n0 + wn * HW + j * M::TN + M::c_row(lane, r);
          const bool ok = gi < s.M && gj < s.N && !(s.tri && gi < gj);
          x0[r] = ok ? epi.pre(batch, gi, gj) : 0.0;
        }
#pragma unroll
        for (int r = 0; r < M::NACC; ++r) {
          const int gi = m0 + wm * HW + i * M::TM + M::c_col(lane, r);
          const int gj = n0 + wn * HW + j * M::TN + M::c_row(lane, r);
          if (gi < s.M && gj < s.N && !(s.tri && gi < gj))
            epi.post(batch, gi, gj, acc[i][j][r], s.tri && gi != gj, x0[r]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < M::NACC; ++r) {
          const int gi = m0 + wm * HW + i * M::TM + M::c_col(lane, r);
          const int gj = n0 + wn * HW + j * M::TN + M::c_row(lane, r);
          if (gi < s.M && gj < s.N) {
            if (s.tri && gi < gj) continue;
            part += epi(batch, gi, gj, acc[i][j][r], s.tri && gi != gj);
          }
        }
      }
    }
  if (Epi::kReduces) {
    part = block_sum(part, red);
    if (t == 0) {
      const int id = (blockIdx.x % 8) * s.per_xcd + blockIdx.x / 8;
      partials[(int64_t)batch * s.ntiles + id] = part;
    }
  }
}

inline int gemm_cu_count() {
  static int ncu = 0;
  if (!ncu) {
    int dev = 0;
    MSQRT_HIP(hipGetDevice(&dev));
    MSQRT_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu <= 0) ncu = 1;
  }
  return ncu;
}

// Raises the dynamic LDS limit of kernel k once (kernels of equal signature
// share a function type, so they are told apart by address).
template <class Kern>
inline void gemm_lds_attr(Kern k, size_t bytes) {
  static std::vector<const void*> done;
  const void* f = (const void*)k;
  if (std::find(done.begin(), done.end(), f) != done.end()) return;
  MSQRT_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done.push_back(f);
}

// ---------------------------------------------------------------------------
// BF16-split variant for float operands: every element x is split into
// h = bf16(x) and l = bf16(x - h) (round to nearest even) while it is staged
// into LDS, and the product is accumulated in float as
//   A B ~ Ah Bh + Ah Bl + Al Bh
// with v_mfma_f32_32x32x16_bf16 (unit roundoff about 2^-16 instead of 2^-24,
// at the bf16 matrix rate).  Same 128 x 128 tiling as the float kernel, K-slabs of 32;
// LDS holds the hi and lo parts k-contiguous so that every lane reads its 8
// consecutive k values with one 16-byte load.

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int SBK = 32;              // K-slab of the split kernel
constexpr int SLD = SBK + 8;         // padded LDS row (bf16 elements)

template <bool TA, bool TB, class Epi>
__global__ __launch_bounds__(GTHREADS, 2) void gemm_split_kernel(GemmShape s,
                                                                 const float* __restrict__ A,
                                                                 const float* __restrict__ B,
                                                                 Epi epi,
                                                                 double* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[GBM][SLD], Al[GBM][SLD];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[GBN][SLD], Bl[GBN][SLD];
  __shared__ double red[GTHREADS / kWave];

  int tm, tn;
  if (!gemm_tile_coords(s, tm, tn)) return;
  const int batch = blockIdx.y;
  const int K = (batch == (int)gridDim.y - 1) ? s.K_last : s.K;
  A += (int64_t)batch * s.sA;
  B += (int64_t)batch * s.sB;
  const int m0 = tm * GBM, n0 = tn * GBN;
  const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
  const int wm = wave % 2, wn = wave / 2;

  // Each thread stages 16 consecutive k of one row of A (m) and of one
  // column of B (n): (row, k-half) = contiguous-m mapping (t % 128, t / 128)
  // when m is the unit-stride index, else (t / 2, t % 2).
  float ra[16], rb[16];
  const int am = TA ? t / 2 : t % GBM, ak = TA ? 16 * (t % 2) : 16 * (t / GBM);
  const int bn = TB ? t % GBN : t / 2, bk = TB ? 16 * (t / GBN) : 16 * (t % 2);
  // An operand whose k index is the unit-stride one is read 16 bytes at a
  // time (two lanes cover a 128-byte line of one row) when its leading
  // dimension and base keep those loads aligned.
  const bool vecA = TA && s.lda % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
  const bool vecB = !TB && s.ldb % 4 == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  auto load = [&](int k0) {
    if (TA && vecA) {
      const int gm = m0 + am;
#pragma unroll
      for (int i4 = 0; i4 < 4; ++i4) {
        const int gk = k0 + ak + 4 * i4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gm < s.M) {
          if (gk + 3 < K) {
            v = *reinterpret_cast<const float4*>(&A[gk + (int64_t)gm * s.lda]);
          } else {
            if (gk < K) v.x = A[gk + (int64_t)gm * s.lda];
            if (gk + 1 < K) v.y = A[gk + 1 + (int64_t)gm * s.lda];
            if (gk + 2 < K) v.z = A[gk + 2 + (int64_t)gm * s.lda];
          }
        }
        ra[4 * i4] = v.x;
        ra[4 * i4 + 1] = v.y;
        ra[4 * i4 + 2] = v.z;
        ra[4 * i4 + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int gm = m0 + am, gk = k0 + ak + i;
        float v = 0.f;
        if (gm < s.M && gk < K) v = TA ? A[gk + (int64_t)gm * s.lda] : A[gm + (int64_t)gk * s.lda];
        ra[i] = v;
      }
    }
    if (!TB && vecB) {
      const int gn = n0 + bn;
#pragma unroll
      for (int i4 = 0; i4 < 4; ++i4) {
        const int gk = k0 + bk + 4 * i4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gn < s.N) {
          if (gk + 3 < K) {
            v = *reinterpret_cast<const float4*>(&B[gk + (int64_t)gn * s.ldb]);
          } else {
            if (gk < K) v.x = B[gk + (int64_t)gn * s.ldb];
            if (gk + 1 < K) v.y = B[gk + 1 + (int64_t)gn * s.ldb];
            if (gk + 2 < K) v.z = B[gk + 2 + (int64_t)gn * s.ldb];
          }
        }
        rb[4 * i4] = v.x;
        rb[4 * i4 + 1] = v.y;
        rb[4 * i4 + 2] = v.z;
        rb[4 * i4 + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int gn = n0 + bn, gk = k0 + bk + i;
        float v = 0.f;
        if (gn < s.N && gk < K) v = TB ? B[gn + (int64_t)gk * s.ldb] : B[gk + (int64_t)gn * s.ldb];
        rb[i] = v;
      }
    }
  };
  auto split_store = [&](const float* r, __bf16 (*hi)[SLD], __bf16 (*lo)[SLD], int row, int k) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      bf16x8_t h, l;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float x = r[8 * half + i];
        const __bf16 xh = (__bf16)x;
        h[i] = xh;
        l[i] = (__bf16)(x - (float)xh);
      }
      *reinterpret_cast<bf16x8_t*>(&hi[row][k + 8 * half]) = h;
      *reinterpret_cast<bf16x8_t*>(&lo[row][k + 8 * half]) = l;
    }
  };

  f32x16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += SBK) {
    __syncthreads();
    split_store(ra, Ah, Al, am, ak);
    split_store(rb, Bh, Bl, bn, bk);
    __syncthreads();
    if (k0 + SBK < K) load(k0 + SBK);
#pragma unroll
    for (int kk = 0; kk < SBK; kk += 16) {
      const int fk = kk + 8 * (lane / 32), fr = lane % 32;
      bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ah[i] = *reinterpret_cast<const bf16x8_t*>(&Ah[wm * 64 + 32 * i + fr][fk]);
        al[i] = *reinterpret_cast<const bf16x8_t*>(&Al[wm * 64 + 32 * i + fr][fk]);
        bh[i] = *reinterpret_cast<const bf16x8_t*>(&Bh[wn * 64 + 32 * i + fr][fk]);
        bl[i] = *reinterpret_cast<const bf16x8_t*>(&Bl[wn * 64 + 32 * i + fr][fk]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
  }

  double part = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int gi = m0 + wm * 64 + i * 32 + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        const int gj = n0 + wn * 64 + j * 32 + lane % 32;
        if (gi < s.M && gj < s.N) {
          if (s.tri && gi < gj) continue;
          part += epi(batch, gi, gj, acc[i][j][r], s.tri && gi != gj);
        }
      }
  if (Epi::kReduces) {
    part = block_sum(part, red);
    if (t == 0) {
      const int id = (blockIdx.x % 8) * s.per_xcd + blockIdx.x / 8;
      partials[(int64_t)batch * s.ntiles + id] = part;
    }
  }
}

// ---------------------------------------------------------------------------
// Epilogues

template <typename T>
struct EpiStore {
  static constexpr const char* kName = "store";
  static constexpr bool kReduces = false;
  T* C;
  int64_t ldc, sC;
  T alpha, beta;
  __device__ double operator()(int b, int i, int j, T v, bool mir) const {
    T* c = C + (int64_t)b * sC;
    T r = alpha * v;
    if (beta != T(0)) r += beta * c[i + (int64_t)j * ldc];
    c[i + (int64_t)j * ldc] = r;
    if (mir) c[j + (int64_t)i * ldc] = r;
    return 0.0;
  }
  static constexpr bool kStaged = true;
  typedef T out_t;
  __device__ bool live(int) const { return true; }
  __device__ T* dst(int b) const { return C + (int64_t)b * sC; }
  __device__ int64_t ld() const { return ldc; }
  __device__ double load(int b, int i, int j) const {
    return beta != T(0) ? (double)C[(int64_t)b * sC + i + (int64_t)j * ldc] : 0.0;
  }
  __device__ T value(int, int, int, T v, double c) const {
    T r = alpha * v;
    if (beta != T(0)) r += beta * (T)c;
    return r;
  }
};

// R = ascale * A - acc in float64; writes R_l = fl32(R) and returns R^2
// (twice for mirrored off-diagonal elements).
struct EpiResidual {
  static constexpr const char* kName = "residual";
  static constexpr bool kReduces = true;
  const double* A;
  int64_t lda, sA;
  const double* ascale;  // per batch entry: 4^-k
  float* R;
  int64_t ldr, sR;
  __device__ double operator()(int b, int i, int j, double v, bool mir) const {
    const double r = (ascale ? ascale[b] : 1.0) * A[(int64_t)b * sA + i + (int64_t)j * lda] - v;
    const float rl = (float)r;
    float* rb = R + (int64_t)b * sR;
    rb[i + (int64_t)j * ldr] = rl;
    if (mir) rb[j + (int64_t)i * ldr] = rl;
    return mir ? 2.0 * r * r : r * r;
  }
};

// Same residual in float64 but keeping R in float64 (fixed-FP64 path).
struct EpiResidual64 {
  static constexpr const char* kName = "residual";
  static constexpr bool kReduces = true;
  const double* A;
  int64_t lda, sA;
  const double* ascale;
  double* R;
  int64_t ldr, sR;
  __device__ double operator()(int b, int i, int j, double v, bool mir) const {
    const double r = (ascale ? ascale[b] : 1.0) * A[(int64_t)b * sA + i + (int64_t)j * lda] - v;
    double* rb = R + (int64_t)b * sR;
    rb[i + (int64_t)j * ldr] = r;
    if (mir) rb[j + (int64_t)i * ldr] = r;
    return mir ? 2.0 * r * r : r * r;
  }
};

// SPD correction solve fused into the Q^T (R Q) product (Alg. 3):
// y_ij = acc_ij / (s_i + s_j), in the factor precision T.
template <typename T>
struct EpiDiagSylv {
  static constexpr const char* kName = "diagsylv";
  static constexpr bool kReduces = false;
  const T* s;
  int64_t sS;
  T* Y;
  int64_t ldy, sY;
  __device__ double operator()(int b, int i, int j, T v, bool mir) const {
    const T* sb = s + (int64_t)b * sS;
    const T y = v / (sb[i] + sb[j]);
    T* yb = Y + (int64_t)b * sY;
    yb[i + (int64_t)j * ldy] = y;
    if (mir) yb[j + (int64_t)i * ldy] = y;
    return 0.0;
  }
  static constexpr bool kStaged = true;
  typedef T out_t;
  __device__ bool live(int) const { return true; }
  __device__ T* dst(int b) const { return Y + (int64_t)b * sY; }
  __device__ int64_t ld() const { return ldy; }
  // s_i + s_j, summed in T (exact in double)
  __device__ double load(int b, int i, int j) const {
    const T* sb = s + (int64_t)b * sS;
    return (double)(sb[i] + sb[j]);
  }
  __device__ T value(int, int, int, T v, double d) const { return v / (T)d; }
};

// Working-precision update X += fl64(acc) fused into the last product of
// Q Y Q^T (Alg. 2/3, last line of the loop).  A mirrored (symmetric) X is
// exactly symmetric before the update, so the mirror element receives the
// updated value itself: a store, without the load of the transposed element
// (which lies in another row for every lane).
template <typename T>
struct EpiUpdate {
  static constexpr const char* kName = "update";
  static constexpr bool kReduces = false;
  double* X;
  int64_t ldx, sX;
  const int* active;  // per batch entry; NULL = all active
  __device__ double operator()(int b, int i, int j, T v, bool mir) const {
    if (active && !active[b]) return 0.0;
    double* xb = X + (int64_t)b * sX;
    const double x = xb[i + (int64_t)j * ldx] + (double)v;
    xb[i + (int64_t)j * ldx] = x;
    if (mir) xb[j + (int64_t)i * ldx] = x;
    return 0.0;
  }
  // Split form for kernels that load a block's X values before any store
  // (the loads of one block are then in flight together).
  static constexpr bool kPrefetch = true;
  __device__ double pre(int b, int i, int j) const {
    if (active && !active[b]) return 0.0;
    return X[(int64_t)b * sX + i + (int64_t)j * ldx];
  }
  __device__ void post(int b, int i, int j, T v, bool mir, double x0) const {
    if (active && !active[b]) return;
    double* xb = X + (int64_t)b * sX;
    const double x = x0 + (double)v;
    xb[i + (int64_t)j * ldx] = x;
    if (mir) xb[j + (int64_t)i * ldx] = x;
  }
  static constexpr bool kStaged = true;
  typedef double out_t;
  __device__ bool live(int b) const { return !active || active[b]; }
  __device__ double* dst(int b) const { return X + (int64_t)b * sX; }
  __device__ int64_t ld() const { return ldx; }
  __device__ double load(int b, int i, int j) const { return X[(int64_t)b * sX + i + (int64_t)j * ldx]; }
  __device__ double value(int, int, int, T v, double x) const { return x + (double)v; }
};


// X = fl64(acc) (initial iterate X_0 = Q S Q^T).
template <typename T>
struct EpiSetF64 {
  static constexpr const char* kName = "set_x0";
  static constexpr bool kReduces = false;
  double* X;
  int64_t ldx, sX;
  __device__ double operator()(int b, int i, int j, T v, bool mir) const {
    double* xb = X + (int64_t)b * sX;
    const double d = (double)v;
    xb[i + (int64_t)j * ldx] = d;
    if (mir) xb[j + (int64_t)i * ldx] = d;
    return 0.0;
  }
  static constexpr bool kStaged = true;
  typedef double out_t;
  __device__ bool live(int) const { return true; }
  __device__ double* dst(int b) const { return X + (int64_t)b * sX; }
  __device__ int64_t ld() const { return ldx; }
  __device__ double load(int, int, int) const { return 0.0; }
  __device__ double value(int, int, int, T v, double) const { return (double)v; }
};

// Host-side shape setup shared by the launchers.
inline GemmShape make_shape(int M, int N, int K, int64_t lda, int64_t ldb, int64_t sA, int64_t sB,
                            bool tri, int tile = GBM) {
  GemmShape s;
  s.M = M; s.N = N; s.K = K; s.K_last = K; s.lda = lda; s.ldb = ldb; s.sA = sA; s.sB = sB;
  s.tri = tri ? 1 : 0;
  s.tiles_m = (int)ceil_div(M, tile);
  s.tiles_n = (int)ceil_div(N, tile);
  s.ntiles = tri ? s.tiles_m * (s.tiles_m + 1) / 2 : s.tiles_m * s.tiles_n;
  s.per_xcd = (int)ceil_div(s.ntiles, 8);
  return s;
}

// split = true selects the BF16-split kernel (float operands only).
// Returns the number of tiles per batch entry of the launch (the count of
// per-tile partial sums a reducing epilogue wrote), which depends on the
// kernel chosen.
template <typename T, class Epi>
int launch_gemm(hipStream_t st, bool ta, bool tb, const GemmShape& s, const T* A, const T* B,
                const Epi& epi, double* partials, int batch, bool split = false) {
  if (s.M <= 0 || s.N <= 0 || batch <= 0) return 0;
  dim3 grid(8 * s.per_xcd, batch), block(GTHREADS);
  const int tok = prof_begin(st);
  if (split) {
    if constexpr (std::is_same<T, float>::value) {
      if (!ta && !tb) hipLaunchKernelGGL((gemm_split_kernel<false, false, Epi>), grid, block, 0, st, s, A, B, epi, partials);
      else if (ta && !tb) hipLaunchKernelGGL((gemm_split_kernel<true, false, Epi>), grid, block, 0, st, s, A, B, epi, partials);
      else if (!ta && tb) hipLaunchKernelGGL((gemm_split_kernel<false, true, Epi>), grid, block, 0, st, s, A, B, epi, partials);
      else hipLaunchKernelGGL((gemm_split_kernel<true, true, Epi>), grid, block, 0, st, s, A, B, epi, partials);
      MSQRT_LAUNCH_CHECK();
      if (tok >= 0) {
        const double outs = s.tri ? 0.5 * (double)s.N * (s.N + 1) : (double)s.M * s.N;
        const double kk = (double)s.K * (batch - 1) + s.K_last;
        const std::string cls = std::string("gemm_bf16x3:") + Epi::kName;
        prof_end(tok, st, cls.c_str(), 2.0 * outs * kk, 0.0);
      }
      return s.ntiles;
    }
  }
  if constexpr (std::is_same<T, float>::value) {
    const int64_t ncu = gemm_cu_count();
    if (s.tri && s.M >= kWideMin && s.K >= 256 && (int64_t)s.ntiles * batch > 2 * ncu) {
      // large triangles that 128-tiles would spread over more than two
      // workgroups per CU: 192 x 192 tiles, one workgroup per CU.  (Full
      // products keep the 128 kernel: at n = 4096 its 1024 tiles fill every
      // CU with two co-resident workgroups, measured 1.31 ms against 1.58 ms.)
      GemmShape w = make_shape(s.M, s.N, s.K, s.lda, s.ldb, s.sA, s.sB, s.tri != 0, WBM);
      w.K_last = s.K_last;
      dim3 gw(8 * w.per_xcd, batch);
      auto gow = [&](auto kern) {
        gemm_lds_attr(kern, kGemmF32wLds);
        hipLaunchKernelGGL(kern, gw, block, kGemmF32wLds, st, w, A, B, epi, partials);
      };
      if (!ta && !tb) gow(gemm_f32w_kernel<false, false, Epi>);
      else if (ta && !tb) gow(gemm_f32w_kernel<true, false, Epi>);
      else if (!ta && tb) gow(gemm_f32w_kernel<false, true, Epi>);
      else gow(gemm_f32w_kernel<true, true, Epi>);
      MSQRT_LAUNCH_CHECK();
      if (tok >= 0) {
        const double outs = w.tri ? 0.5 * (double)w.N * (w.N + 1) : (double)w.M * w.N;
        const double kk = (double)w.K * (batch - 1) + w.K_last;
        const std::string cls = std::string("gemm_f32:") + Epi::kName;
        prof_end(tok, st, cls.c_str(), 2.0 * outs * kk, 0.0);
      }
      return w.ntiles;
    }
    // single full products with a long K that 128-tiles would spread over
    // more than two workgroups per CU while 256-tiles fill one round on at
    // least 90% of the CUs: 256 x 256 tiles, one workgroup per CU (at
    // n = 4096 measured 7% faster than the 128 kernel).  Batches of short
    // products (64 x 512^3) measured 40% slower on it than on the 128 kernel,
    // so they keep that one.
    const int64_t t256 = ceil_div(s.M, WBX) * ceil_div(s.N, WBX);
    if (batch == 1 && !s.tri && s.K >= 2048 && (int64_t)s.ntiles > 2 * ncu && t256 <= ncu &&
        10 * t256 >= 9 * ncu) {
      GemmShape w = make_shape(s.M, s.N, s.K, s.lda, s.ldb, s.sA, s.sB, false, WBX);
      w.K_last = s.K_last;
      dim3 gw(8 * w.per_xcd, batch);
      auto gox = [&](auto kern) {
        gemm_lds_attr(kern, f32w_lds<WBX>());
        hipLaunchKernelGGL(kern, gw, block, f32w_lds<WBX>(), st, w, A, B, epi, partials);
      };
      if (!ta && !tb) gox(gemm_f32w_kernel<false, false, Epi, WBX>);
      else if (ta && !tb) gox(gemm_f32w_kernel<true, false, Epi, WBX>);
      else if (!ta && tb) gox(gemm_f32w_kernel<false, true, Epi, WBX>);
      else gox(gemm_f32w_kernel<true, true, Epi, WBX>);
      MSQRT_LAUNCH_CHECK();
      if (tok >= 0) {
        const double kk = (double)w.K * (batch - 1) + w.K_last;
        const std::string cls = std::string("gemm_f32:") + Epi::kName;
        prof_end(tok, st, cls.c_str(), 2.0 * (double)w.M * w.N * kk, 0.0);
      }
      return w.ntiles;
    }
    // more tiles than two workgroups per CU hold but no more than three:
    // the 16-deep variant runs them in one round
    const int64_t units = (int64_t)s.ntiles * batch;
    const bool three = units > 2 * ncu && units <= 3 * ncu;
    auto go = [&](auto kern, size_t lds) {
      gemm_lds_attr(kern, lds);
      hipLaunchKernelGGL(kern, grid, block, lds, st, s, A, B, epi, partials);
    };
    if (three) {
      if (!ta && !tb) go(gemm_f32k16_kernel<false, false, Epi>, kGemmF32k16Lds);
      else if (ta && !tb) go(gemm_f32k16_kernel<true, false, Epi>, kGemmF32k16Lds);
      else if (!ta && tb) go(gemm_f32k16_kernel<false, true, Epi>, kGemmF32k16Lds);
      else go(gemm_f32k16_kernel<true, true, Epi>, kGemmF32k16Lds);
    } else {
      if (!ta && !tb) go(gemm_f32_kernel<false, false, Epi>, kGemmF32Lds);
      else if (ta && !tb) go(gemm_f32_kernel<true, false, Epi>, kGemmF32Lds);
      else if (!ta && tb) go(gemm_f32_kernel<false, true, Epi>, kGemmF32Lds);
      else go(gemm_f32_kernel<true, true, Epi>, kGemmF32Lds);
    }
  } else {
    const int64_t ncu = gemm_cu_count();
    if (s.tri && s.M >= kWideMin && s.K >= 256 && (int64_t)s.ntiles * batch > 2 * ncu) {
      GemmShape w = make_shape(s.M, s.N, s.K, s.lda, s.ldb, s.sA, s.sB, true, WBM);
      w.K_last = s.K_last;
      dim3 gw(8 * w.per_xcd, batch);
      auto gow = [&](auto kern) {
        gemm_lds_attr(kern, kGemmF64wLds);
        hipLaunchKernelGGL(kern, gw, dim3(kW64Threads), kGemmF64wLds, st, w, A, B, epi, partials);
      };
      if (!ta && !tb) gow(gemm_f64w_kernel<false, false, Epi>);
      else if (ta && !tb) gow(gemm_f64w_kernel<true, false, Epi>);
      else if (!ta && tb) gow(gemm_f64w_kernel<false, true, Epi>);
      else gow(gemm_f64w_kernel<true, true, Epi>);
      MSQRT_LAUNCH_CHECK();
      if (tok >= 0) {
        const double outs = 0.5 * (double)w.N * (w.N + 1);
        const double kk = (double)w.K * (batch - 1) + w.K_last;
        const std::string cls = std::string("gemm_f64:") + Epi::kName;
        prof_end(tok, st, cls.c_str(), 2.0 * outs * kk, 0.0);
      }
      return w.ntiles;
    }
    auto go = [&](auto kern) {
      gemm_lds_attr(kern, kGemmF64Lds);
      hipLaunchKernelGGL(kern, grid, block, kGemmF64Lds, st, s, A, B, epi, partials);
    };
    if (!ta && !tb) go(gemm_f64_kernel<false, false, Epi>);
    else if (ta && !tb) go(gemm_f64_kernel<true, false, Epi>);
    else if (!ta && tb) go(gemm_f64_kernel<false, true, Epi>);
    else go(gemm_f64_kernel<true, true, Epi>);
  }
  MSQRT_LAUNCH_CHECK();
  if (tok >= 0) {
    // algorithmic work: 2 M N K per entry, or the lower triangle only for
    // symmetric outputs
    const double outs = s.tri ? 0.5 * (double)s.N * (s.N + 1) : (double)s.M * s.N;
    const double kk = (double)s.K * (batch - 1) + s.K_last;
    // class "gemm_f32:<epilogue>" / "gemm_f64:<epilogue>"
    const std::string cls = std::string(sizeof(T) == 4 ? "gemm_f32:" : "gemm_f64:") + Epi::kName;
    prof_end(tok, st, cls.c_str(), 2.0 * outs * kk, 0.0);
  }
  return s.ntiles;
}

}  // namespace msqrt
