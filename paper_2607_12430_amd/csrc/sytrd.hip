// Householder tridiagonalisation of a symmetric matrix (first step of the
// spectral decomposition used by Alg. 3), blocked by panels of nb columns.
//
// Panel: one cooperative launch of G = TR (TR + 1) / 2 workgroups, one per
// lower-triangular tile of the trailing matrix (at most 192 x 192, up to 253
// workgroups), that walks the panel's columns with ONE grid barrier per
// column.  For column j with updated sub-column u (rows j+1..n-1) the
// reflector is v = (u - beta e1) c, c = 1/(alpha - beta).  Because every
// quantity the panel needs from v is linear in v, each workgroup forms its
// tile's share of the trailing product with the *unnormalised* u (A22 u and,
// off the diagonal, A22^T u), plus partial sums of ||u||^2, u^T A22 u,
// u^T A22 e1, V^T u and W^T u, before the barrier.  After the barrier every
// workgroup finishes the reflector scalars, y = A22 v - V (W^T v) - W (V^T v)
// and w = tau y - (tau/2)(tau y^T v) v for the rows it needs, and prepares
// the next column's u -- so the classic two reductions per column (norm,
// then product) cost a single synchronisation.
//
// After a panel, A22 -= [V W] [W V]^T.  The float kernel holds its tile in
// registers for the whole panel and applies the previous panel's update to
// it at launch start; it keeps only the lower triangle current (a diagonal
// tile reads its upper half from the mirror).  The double kernel streams its
// tile at every column and leaves the update to an MFMA GEMM with symmetric
// output (both triangles written).
#include <vector>

#include "gemm.hpp"
#include "kernels.hpp"
#include "profile.hpp"
#include "tridiag.hpp"

namespace msqrt {

namespace {

constexpr int kThreads = 1024;
constexpr int kMaxTs = 192;  // max tile size handled by one workgroup
constexpr int kTRMax = 22;   // max tiles per dimension: 253 workgroups, one per CU
constexpr int kGMax = kTRMax * (kTRMax + 1) / 2;
constexpr int kNbMax = 32;
// Row work of a column is spread over three thread ranges that run side by
// side: rows of I on [0, kMaxTs), pivot rows on [kPivT, kPivT + kNbMax), rows
// of K on [kKT, kKT + kMaxTs).
constexpr int kPivT = 256;
constexpr int kKT = 512;
static_assert(kMaxTs <= kPivT && kPivT + kNbMax <= kKT && kKT + kMaxTs <= 1024, "thread ranges");

// Values exchanged between workgroups inside a launch (partial products and
// sums) are written and read with agent-scope atomic stores and loads, which
// are coherent across the XCDs' L2 caches, so the barrier needs no device-wide
// fence: such a fence writes back and invalidates the whole L2 of every XCD
// on every column, and the tiles cached there would be fetched again.
template <typename T>
__device__ inline void cstore(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline T cload(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront sum by DPP: butterflies inside every row of 16 lanes (two quad
// permutations, the half-row mirror, the row mirror) leave each lane with
// its row's sum; the four row sums are then read with readlane.  Every lane
// gets the total (in a fixed order, so results are reproducible).  All 64
// lanes must be active: every call site in this file is reached by whole
// wavefronts.
template <int CTRL>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline float dpp_v(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ inline double dpp_v(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline float lane_of(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double lane_of(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over each row of 16 lanes, left in every lane of the row.
template <typename V>
__device__ inline V rsum16(V v) {
  v += dpp_v<0xB1>(v);
  v += dpp_v<0x4E>(v);
  v += dpp_v<0x141>(v);
  v += dpp_v<0x140>(v);
  return v;
}
// Sum over each group of 8 lanes (half a row), left in every lane of it.
template <typename V>
__device__ inline V hsum8(V v) {
  v += dpp_v<0xB1>(v);
  v += dpp_v<0x4E>(v);
  v += dpp_v<0x141>(v);
  return v;
}
template <typename V>
__device__ inline V wsum(V v) {
  v += dpp_v<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_v<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_v<0x141>(v);  // row_half_mirror
  v += dpp_v<0x140>(v);  // row_mirror
  return (lane_of(v, 0) + lane_of(v, 16)) + (lane_of(v, 32) + lane_of(v, 48));
}

// Grid barrier state of one batch entry (unsigned words): the top counter,
// the sticky failure flag, the release word and 8 group counters, each on a
// 256-byte line of its own.
constexpr int kBarTop = 0, kBarFail = 1, kBarRel = 64, kBarSub = 128, kBarSubStride = 64;

// Counter values at the start of a launch.  All counters only grow within one
// reduction, so a barrier needs no reset: the host adds what every launch
// contributes.
struct BarrierBase {
  unsigned gen;     // release word: barriers completed
  unsigned top;     // top counter
  unsigned sub[8];  // group counters
};

// Two-level grid barrier, split into arrival and wait so that a workgroup
// can do work that needs no other workgroup's results while the barrier
// completes.  The G workgroups of a batch entry form 8 groups (workgroup
// index mod 8, which is the XCD a workgroup is dispatched to when the entry
// starts on a multiple of 8); a workgroup adds 1 to its group's counter, the
// group's last arrival (known from the value its add returns) adds 1 to the
// top counter, and the last arrival there writes the barrier's generation
// number to the release word, which the other workgroups poll.  Spreading the
// arrivals over 8 counters halves the cost of a barrier of 253 workgroups
// against one shared counter.  Every thread waits for its own coherent
// stores to complete before the workgroup arrives.  The counters are handled
// by the first lane of the last wave (kBarT), which has no row work, so the
// atomics' round trips hold up no thread that has.  A spin limit keeps a
// broken launch from hanging: it raises the sticky failure flag.
constexpr int kBarT = kThreads - kWave;

// Arrival; returns true in thread kBarT if this workgroup released barrier k.
__device__ inline bool grid_arrive(unsigned* bar, const BarrierBase& base, unsigned sub_base, int blk,
                                   int G, int k) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // A launch of one workgroup per batch entry synchronises with itself only:
  // the wait above and the workgroup barrier make its stores visible to its
  // own later loads.  (The trailing order only shrinks, so every later launch
  // of the reduction has G = 1 too and no counter is read again.)
  if (G == 1) return true;
  bool released = false;
  if (threadIdx.x == kBarT) {
    const unsigned g = (unsigned)blk & 7u;
    const unsigned gsz = (unsigned)G / 8u + (g < ((unsigned)G & 7u) ? 1u : 0u);
    const unsigned ng = G < 8 ? (unsigned)G : 8u;
    // with G <= 8 every group has one member, which is always its group's
    // last arrival: its counter is skipped (later launches of the reduction
    // have G <= 8 too, so the group counters are not read again)
    const unsigned old =
        G <= 8 ? sub_base + gsz * (unsigned)k - 1u
               : __hip_atomic_fetch_add(&bar[kBarSub + kBarSubStride * g], 1u, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1u == sub_base + gsz * (unsigned)k) {
      const unsigned o2 = __hip_atomic_fetch_add(&bar[kBarTop], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 + 1u == base.top + ng * (unsigned)k) {
        cstore(&bar[kBarRel], base.gen + (unsigned)k);
        released = true;
      }
    }
  }
  return released;
}

// Wait for barrier k (released: what grid_arrive returned).
__device__ inline void grid_wait(unsigned* bar, const BarrierBase& base, int k, bool released) {
  if (threadIdx.x == kBarT && !released) {
    const unsigned gen = base.gen + (unsigned)k;
    unsigned spins = 0;
    while (cload(&bar[kBarRel]) < gen) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0u) {
        if (cload(&bar[kBarFail]) != 0u) break;
        if (spins > (1u << 24)) {
          cstore(&bar[kBarFail], 1u);
          break;
        }
      }
    }
  }
  __syncthreads();
}

__device__ inline void grid_barrier(unsigned* bar, const BarrierBase& base, unsigned sub_base, int blk,
                                    int G, int k) {
  grid_wait(bar, base, k, grid_arrive(bar, base, sub_base, blk, G, k));
}

template <typename T>
struct PanelArgs {
  int n, p, nb;  // matrix size, first column of the panel, panel width
  int nbp;       // width of the previous panel whose trailing update this
                 // launch applies itself (float; 0: none, or applied by a GEMM)
  int TR;        // tiles per dimension; G = TR (TR + 1) / 2 workgroups (lower triangle)
  int r0, ts;    // tile grid origin (p + 1) and tile size (<= kMaxTs)
  T* A;          // n x n, ld n, full symmetric storage
  T* VW;         // n x 2 nb: [V W], rows >= p+1 written by the panel
  T* WV;         // n x 2 nb: [W V]
  T* d;
  T* e;
  T* tau;
  T* ypart;      // [2][TR][n]
  double* sp;    // [2][G][4]
  double* vp;    // [2][TR][2 kNbMax]
  unsigned* bar;
  BarrierBase bar_base;  // barrier counters when the launch starts
  // batch entry b = blockIdx.y: every pointer above advances by b times
  // its stride
  int64_t sA, sVW, sD, sYP, sSP, sVP, sBar;
};

// Tile product of one lower-triangular tile (I x K, I >= K) with the current
// u: zI = A(I, K) uK (all tiles) and zK = A(I, K)^T uI (off-diagonal tiles),
// masked to rows/columns >= jmin.  Wave w takes columns [16w, 16w+16) of the
// tile, lane l rows l, l+64, ...; all loads of a 16-column chunk are issued
// before any is used, so every wave of the workgroup has its whole share of
// the tile in flight at once.  Row partials stay in zi (NP passes of RPL rows
// per lane); column partials are reduced over the wave and added to zK.
template <typename T, int RPL, int NP>
__device__ inline void tile_product(const T* __restrict__ A, unsigned ld, int I0, int nI, int K0,
                                    int nK, int jmin, bool offdiag, const T* uI, const T* uK,
                                    T (&zi)[NP][RPL], T* zK, int tid) {
  constexpr int CW = sizeof(T) == 4 ? 12 : 6;            // columns per chunk
  constexpr int NCH = kMaxTs / (CW * (kThreads / kWave));  // chunks per wave
  static_assert(NCH * CW * (kThreads / kWave) == kMaxTs, "chunks must cover the tile");
  const int wave = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int ps = 0; ps < NP; ++ps)
#pragma unroll
    for (int q = 0; q < RPL; ++q) zi[ps][q] = T(0);
  for (int ch = 0; ch < NCH; ++ch) {
    const int cb = (ch * (kThreads / kWave) + wave) * CW;
    if (cb >= nK) break;
    // Columns below jmin or past the tile are skipped (wave-uniform test).
    const int cfirst = max(cb, jmin - K0);
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
      const int rb = ps * RPL * kWave;
      T v[CW][RPL];
      int rowoff[RPL];
      bool rowok[RPL];
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = rb + lane + q * kWave;
        rowok[q] = r < nI && (I0 + r) >= jmin;
        rowoff[q] = rowok[q] ? I0 + r : I0;
      }
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const int k = cb + c;
        const bool colok = k < nK && k >= cfirst;
        const T* colp = A + (unsigned)(K0 + (colok ? k : cb)) * ld;
#pragma unroll
        for (int q = 0; q < RPL; ++q) v[c][q] = (colok && rowok[q]) ? colp[rowoff[q]] : T(0);
      }
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const T uk = (cb + c < nK) ? uK[cb + c] : T(0);
        T zk = T(0);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          const int r = rb + lane + q * kWave;
          zi[ps][q] += v[c][q] * uk;
          if (offdiag) zk += v[c][q] * ((r < nI) ? uI[r] : T(0));
        }
        if (offdiag) {
          zk = wsum(zk);
          if (lane == 0 && cb + c < nK) zK[cb + c] = zk;
        }
      }
    }
  }
}

// Register-resident variant (float): wave w holds columns [CW w, CW w + CW)
// of the tile, lane l rows l, l+64, l+128 (CW RPL = 36 values), loaded once
// per launch.  The trailing matrix does not change inside a panel (its
// updates are applied lazily through V and W), and the rows and columns that
// the current column excludes are cancelled by the zero entries of u there,
// so the same registers serve every column of the panel.
template <typename T, int CW, int RPL>
__device__ inline void tile_load(const T* __restrict__ A, unsigned ld, int I0, int nI, int K0, int nK,
                                 bool diag, T (&v)[CW][RPL], int tid) {
  const int wave = tid / kWave, lane = tid % kWave;
  const int cb = wave * CW;
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const int k = cb + c;
    const bool colok = k < nK;
    const T* colp = A + (unsigned)(K0 + (colok ? k : 0)) * ld + I0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + q * kWave;
      // the upper part of a diagonal tile is read from its mirror in the
      // lower triangle (only the lower triangle is kept up to date)
      v[c][q] = (colok && r < nI) ? ((diag && r < k) ? A[K0 + k + (unsigned)(I0 + r) * ld] : colp[r]) : T(0);
    }
  }
}

template <typename T, int CW, int RPL>
__device__ inline void tile_mul(const T (&v)[CW][RPL], int nI, int nK, bool offdiag, const T* uI,
                                const T* uK, T (&zi)[RPL], T* zK, int tid) {
  const int wave = tid / kWave, lane = tid % kWave;
  const int cb = wave * CW;
  T ui[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = lane + q * kWave;
    zi[q] = T(0);
    ui[q] = (r < nI) ? uI[r] : T(0);
  }
  T zk[CW];
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const T uk = (cb + c < nK) ? uK[cb + c] : T(0);
    zk[c] = T(0);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      zi[q] += v[c][q] * uk;
      zk[c] += v[c][q] * ui[q];
    }
  }
  if (offdiag) {
    // Column sums over the 64 lanes, 12 columns at once: halving exchanges
    // between the wave's halves (columns c and c+6), then between the rows
    // of 16 lanes of each half (c and c+3), then sums inside each row.  Row
    // R of the wave ends with the sums of columns 3R .. 3R+2.
    static_assert(CW == 12 && sizeof(T) == 4, "the exchange pattern splits 12 float columns");
    T y[6], z[3];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(zk[c]), __float_as_uint(zk[c + 6]), false,
                                                       false);
      y[c] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(y[c]), __float_as_uint(y[c + 3]), false,
                                                       false);
      z[c] = rsum16(__uint_as_float(sw[0]) + __uint_as_float(sw[1]));
    }
    const int l16 = lane & 15, col = cb + 3 * (lane >> 4) + l16;
    if (l16 < 3 && col < nK) zK[col] = (l16 == 0) ? z[0] : (l16 == 1 ? z[1] : z[2]);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void sytrd_panel_kernel(PanelArgs<T> a) {
  constexpr int RPL = 3;
  const int n = a.n, nb = a.nb, TR = a.TR, G = TR * (TR + 1) / 2;
  // workgroup (x, y) = (tile, batch entry).  Both ids are scalar registers,
  // and so is everything derived from them below: the base pointers and the
  // tile origin never take vector registers.
  {
    const int64_t bz = blockIdx.y;
    a.A += bz * a.sA;
    a.VW += bz * a.sVW;
    a.WV += bz * a.sVW;
    a.d += bz * a.sD;
    a.e += bz * a.sD;
    a.tau += bz * a.sD;
    a.ypart += bz * a.sYP;
    a.sp += bz * a.sSP;
    a.vp += bz * a.sVP;
    a.bar += bz * a.sBar;
  }
  const int blk = blockIdx.x;
  // tile (bi, bj) of the lower triangle, row-major: bi (bi + 1) / 2 <= blk
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
  const int bj = blk - bi * (bi + 1) / 2;
  const bool diag = bi == bj, offdiag = !diag;
  // this workgroup's group counter base (selected without dynamic indexing)
  unsigned sub_base = 0;
#pragma unroll
  for (int g = 0; g < 8; ++g)
    if (g == (blk & 7)) sub_base = a.bar_base.sub[g];
  const int I0 = a.r0 + bi * a.ts, I1 = max(I0, min(n, I0 + a.ts));
  const int K0 = a.r0 + bj * a.ts, K1 = max(K0, min(n, K0 + a.ts));
  const int nI = I1 - I0, nK = K1 - K0;
  const int tid = threadIdx.x;
  // Offsets inside one batch entry fit 32 bits (n <= 4225, so n^2 < 2^31):
  // unsigned 32-bit offsets from the uniform base pointers let every global
  // access use one offset register instead of a 64-bit address.
  const unsigned ld = (unsigned)n;
  const int p = a.p;
  T* A = a.A;

  // Panel columns of this workgroup's rows: PVI[t][r] = V(I0 + r, t), etc.
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T* PVI = reinterpret_cast<T*>(smem_raw);
  T* PWI = PVI + nb * kMaxTs;
  T* PVK = PWI + nb * kMaxTs;
  T* PWK = PVK + nb * kMaxTs;
  __shared__ T uI[kMaxTs], uK[kMaxTs], zKs[kMaxTs];
  // zred (row partials of the tile product, before the barrier) and the
  // gathered partial sums (after it) share one buffer.
  constexpr int kZredBytes = (kThreads / kWave / 2) * kMaxTs * (int)sizeof(T);
  constexpr int kGathBytes = (3 * kGMax + kTRMax * 2 * kNbMax) * 8;
  __shared__ double scratch[(kZredBytes > kGathBytes ? kZredBytes : kGathBytes) / 8];
  T* zred = reinterpret_cast<T*>(scratch);
  double (*spl)[kGMax] = reinterpret_cast<double (*)[kGMax]>(scratch);
  double* vpl = scratch + 3 * kGMax;
  // Pivot rows r = p+1+q (q < nb) of V and W and their u for the current
  // column: every workgroup keeps its own copy, so no value written by another
  // workgroup in the current phase is ever read.
  __shared__ T PV[kNbMax][kNbMax + 1], PW[kNbMax][kNbMax + 1], PU[kNbMax];
  // V^T v and W^T v, rounded to T and held as double (they enter only
  // double sums)
  __shared__ double VTv[kNbMax], WTv[kNbMax];
  __shared__ double vts[2 * kNbMax];  // V^T u, W^T u summed over the row tiles
  __shared__ double red3[kThreads / kWave][3];
  __shared__ double sc[8];
  __shared__ T acI[kMaxTs], acK[kMaxTs], acP[kNbMax];  // A(:, j+1) on rows I, K, pivots
  __shared__ T yzI[kMaxTs], yzK[kMaxTs], yzP[kNbMax];  // (A22 u) on rows I, K, pivots

  // ---- prologue: u for the first column of the panel (and, for float, the
  // register copy of the tile)
  constexpr bool kResident = sizeof(T) == 4;
  constexpr int kRCW = kMaxTs / (kThreads / kWave);  // 12 columns per wave
  static_assert(!kResident || (kRCW * (kThreads / kWave) == kMaxTs && RPL * kWave == kMaxTs),
                "the register tile must cover the tile");
  T vt[kResident ? kRCW : 1][kResident ? RPL : 1];
  if constexpr (kResident) tile_load<T, kRCW, RPL>(A, ld, I0, nI, K0, nK, diag, vt, tid);
  // Trailing update of the previous panel, A(p:, p:) -= [V W] [W V]^T over its
  // 2 nbp columns (left in VW and WV), applied here instead of by a separate
  // GEMM: the register tile is updated and written back (the lower triangle
  // and the diagonal squares, with coherent stores), and column p, which no
  // tile covers, is corrected where it is read.  A grid barrier then makes the
  // written-back tiles visible; inside this launch they are read back with
  // coherent loads (a line of another XCD's L2 may hold the old values).
  const int nbp = kResident ? a.nbp : 0;
  __shared__ T vwp[2 * kNbMax], wvp[2 * kNbMax];  // VW(p, :), WV(p, :)
  __shared__ double app;                           // updated A(p, p)
  if (nbp > 0) {
    const int w2 = 2 * nbp;
    T* VWs = PVI;              // [t][r]: VW(I0 + r, t), w2 x kMaxTs
    T* WVs = PVI + w2 * kMaxTs;  // [t][k]: WV(K0 + k, t)
    {
      // every load of the staging issued before any store
      constexpr int kSt = 2 * kNbMax * kMaxTs / kThreads;
      static_assert(kSt * kThreads == 2 * kNbMax * kMaxTs, "staging split");
      T va[kSt], wa[kSt];
#pragma unroll
      for (int e = 0; e < kSt; ++e) {
        const int x = tid + e * kThreads, t = x / kMaxTs, r = x % kMaxTs;
        va[e] = (t < w2 && r < nI) ? a.VW[I0 + r + (unsigned)t * ld] : T(0);
        wa[e] = (t < w2 && r < nK) ? a.WV[K0 + r + (unsigned)t * ld] : T(0);
      }
#pragma unroll
      for (int e = 0; e < kSt; ++e) {
        const int x = tid + e * kThreads;
        if (x < w2 * kMaxTs) {
          VWs[x] = va[e];
          WVs[x] = wa[e];
        }
      }
    }
    if (tid < w2) {
      vwp[tid] = a.VW[p + (unsigned)tid * ld];
      wvp[tid] = a.WV[p + (unsigned)tid * ld];
    }
    __syncthreads();
    if constexpr (kResident) {
      // the products are summed apart and subtracted once, as a GEMM update
      // would round them
      const int wave = tid / kWave, lane = tid % kWave, cb = wave * kRCW;
      static_assert(kRCW % 4 == 0 && kMaxTs % 4 == 0, "float4 rows of WVs");
      T acc[kRCW][RPL];
#pragma unroll
      for (int c = 0; c < kRCW; ++c)
#pragma unroll
        for (int q = 0; q < RPL; ++q) acc[c][q] = T(0);
      for (int t = 0; t < w2; ++t) {
        T av[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) av[q] = VWs[t * kMaxTs + lane + q * kWave];
        const float4* b4 = reinterpret_cast<const float4*>(WVs + t * kMaxTs + cb);
#pragma unroll
        for (int c4 = 0; c4 < kRCW / 4; ++c4) {
          const float4 bq = b4[c4];
          const T bv[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int q = 0; q < RPL; ++q) acc[c4 * 4 + e][q] += av[q] * bv[e];
        }
      }
#pragma unroll
      for (int c = 0; c < kRCW; ++c)
#pragma unroll
        for (int q = 0; q < RPL; ++q) vt[c][q] -= acc[c][q];
#pragma unroll
      for (int c = 0; c < kRCW; ++c) {
        const int k = cb + c;
        if (k < nK) {
#pragma unroll
          for (int q = 0; q < RPL; ++q) {
            const int r = lane + q * kWave;
            if (r < nI) cstore(&A[I0 + r + (unsigned)(K0 + k) * ld], vt[c][q]);
          }
        }
      }
    }
    // column p on the rows of I and K (VW on the rows of K is WV with its
    // halves exchanged) and on the pivot rows; A(p, p)
    {
      const int j = p;
      if (tid < nI) {
        T cr = T(0);
        for (int t = 0; t < w2; ++t) cr += VWs[t * kMaxTs + tid] * wvp[t];
        uI[tid] = (I0 + tid >= j + 1) ? A[I0 + tid + (unsigned)j * ld] - cr : T(0);
      }
      if (tid >= kKT && tid - kKT < nK) {
        const int r = tid - kKT;
        T cr = T(0);
        for (int t = 0; t < w2; ++t) cr += WVs[((t + nbp) % w2) * kMaxTs + r] * wvp[t];
        uK[r] = (K0 + r >= j + 1) ? A[K0 + r + (unsigned)j * ld] - cr : T(0);
      }
      if (tid >= kPivT && tid < kPivT + kNbMax) {
        const int q = tid - kPivT, r = p + 1 + q;
        T u = T(0);
        if (q < nb && r < n) {
          T vr[2 * kNbMax];  // the row's coefficients, all loads issued together
#pragma unroll
          for (int t = 0; t < 2 * kNbMax; ++t) vr[t] = (t < w2) ? a.VW[r + (unsigned)t * ld] : T(0);
          T cr = T(0);
#pragma unroll
          for (int t = 0; t < 2 * kNbMax; ++t) cr += vr[t] * ((t < w2) ? wvp[t] : T(0));
          u = A[r + (unsigned)j * ld] - cr;
        }
        if (q < nb) PU[q] = u;
      }
      if (tid == 0) {
        double s = (double)A[p + (unsigned)p * ld];
        T corr = T(0);
        for (int t = 0; t < w2; ++t) corr += vwp[t] * wvp[t];
        app = s - (double)corr;
      }
    }
    grid_barrier(a.bar, a.bar_base, sub_base, blk, G, 1);
  } else {
    const int j = p;
    for (int r = tid; r < nI; r += kThreads) uI[r] = (I0 + r >= j + 1) ? A[I0 + r + (unsigned)j * ld] : T(0);
    for (int r = tid; r < nK; r += kThreads) uK[r] = (K0 + r >= j + 1) ? A[K0 + r + (unsigned)j * ld] : T(0);
    for (int q = tid; q < nb; q += kThreads) PU[q] = (p + 1 + q < n) ? A[p + 1 + q + (unsigned)j * ld] : T(0);
    if (tid == 0) app = (double)A[p + (unsigned)p * ld];
  }
  __syncthreads();
  const int kb0 = nbp > 0 ? 1 : 0;  // barriers before the first column's

  for (int jj = 0; jj < nb; ++jj) {
    const int j = p + jj;
    const int buf = jj & 1;
    // ---- column j+1 of A (a1 for the product, base of the next u), issued
    // together with the tile loads
    T acv_i = T(0), acv_k = T(0), acv_p = T(0);
    auto rd = [&](unsigned idx) -> T { return nbp > 0 ? cload(&A[idx]) : A[idx]; };
    if (tid < nI) acv_i = rd(I0 + tid + (unsigned)(j + 1) * ld);
    if (tid < nK) acv_k = rd(K0 + tid + (unsigned)(j + 1) * ld);
    if (tid < nb && p + 1 + tid < n) acv_p = rd(p + 1 + tid + (unsigned)(j + 1) * ld);
    // A(j, j) for d_j (never written inside the panel after the prologue)
    const double ajj = (tid == 0) ? (jj == 0 ? app : (double)rd(j + (unsigned)j * ld)) : 0.0;
    // ---- tile product; the 16 waves' row partials are folded onto 8 slots;
    // every column sum of zKs is written once, by the wave owning the column
    {
      constexpr int NP = kMaxTs / (RPL * kWave);
      static_assert(NP * RPL * kWave == kMaxTs, "row passes must cover the tile");
      T zi[NP][RPL];
      if constexpr (kResident) {
        static_assert(!kResident || NP == 1, "one row pass");
        tile_mul<T, kRCW, RPL>(vt, nI, nK, offdiag, uI, uK, zi[0], zKs, tid);
      } else {
        tile_product<T, RPL, NP>(A, ld, I0, nI, K0, nK, j + 1, offdiag, uI, uK, zi, zKs, tid);
      }
      const int wave = tid / kWave, lane = tid % kWave;
      if (wave < 8) {
#pragma unroll
        for (int ps = 0; ps < NP; ++ps)
#pragma unroll
          for (int q = 0; q < RPL; ++q) zred[wave * kMaxTs + ps * RPL * kWave + lane + q * kWave] = zi[ps][q];
      }
      __syncthreads();
      if (wave >= 8) {
#pragma unroll
        for (int ps = 0; ps < NP; ++ps)
#pragma unroll
          for (int q = 0; q < RPL; ++q) zred[(wave - 8) * kMaxTs + ps * RPL * kWave + lane + q * kWave] += zi[ps][q];
      }
      if (tid < nI) acI[tid] = acv_i;
      if (tid < nK) acK[tid] = acv_k;
      if (tid < nb) acP[tid] = acv_p;
      __syncthreads();
    }
    // zI = sum over the 8 slots; publish partial products and u^T A u
    double s_uAu = 0.0;
    for (int r = tid; r < nI; r += kThreads) {
      T z = T(0);
#pragma unroll
      for (int w = 0; w < 8; ++w) z += zred[w * kMaxTs + r];
      cstore(&a.ypart[((unsigned)buf * TR + bj) * n + I0 + r], z);
      s_uAu += (double)uI[r] * (double)z;
    }
    if (offdiag && tid >= kKT && tid - kKT < nK)
      cstore(&a.ypart[((unsigned)buf * TR + bi) * n + K0 + (tid - kKT)], zKs[tid - kKT]);
    // ---- row-owner partials (diagonal tiles): ||u(2:)||^2, u^T a1, V^T u, W^T u
    double s_sig = 0.0, s_ua1 = 0.0;
    if (diag) {
      for (int r = tid; r < nI; r += kThreads) {
        const int i = I0 + r;
        const double u = (double)uI[r];
        if (i >= j + 2) s_sig += u * u;
        if (i >= j + 1) s_ua1 += u * (double)acI[r];
      }
      // one row of 16 lanes per column of [V W] (2 kNbMax rows of 16 lanes =
      // the workgroup), each lane summing every 16th row of the tile
      static_assert(2 * kNbMax * 16 == kThreads, "one 16-lane row per panel column");
      const int c = tid >> 4, l16 = tid & 15;
      double s = 0.0;
      if (c < 2 * jj) {
        const T* col = c < jj ? (PVI + c * kMaxTs) : (PWI + (c - jj) * kMaxTs);
#pragma unroll
        for (int i = 0; i < kMaxTs / 16; ++i) {
          const int r = l16 + 16 * i;
          if (r < nI) s += (double)col[r] * (double)uI[r];
        }
      }
      s = rsum16(s);
      if (l16 == 0 && c < 2 * jj) cstore(&a.vp[((unsigned)buf * TR + bi) * (2 * kNbMax) + c], s);
    }
    // one reduction of the three scalars (wave sums, then one thread), and
    // the pivot-row correction of d_j summed by the first wave
    {
      const double w0 = wsum(s_uAu), w1 = diag ? wsum(s_sig) : 0.0, w2 = diag ? wsum(s_ua1) : 0.0;
      const int wv_ = tid / kWave, ln_ = tid % kWave;
      if (ln_ == 0) {
        red3[wv_][0] = w0;
        red3[wv_][1] = w1;
        red3[wv_][2] = w2;
      }
      double pd = 0.0;
      if (tid < kWave) {
        if (tid < jj) pd = (double)PV[jj - 1][tid] * (double)PW[jj - 1][tid];
        pd = wsum(pd);
      }
      __syncthreads();
      static_assert(kThreads / kWave == 16, "one lane of the first row per wave");
      if (tid < 16) {
        double t0 = rsum16(red3[tid][0]);
        const double t1 = rsum16(red3[tid][1]), t2 = rsum16(red3[tid][2]);
        if (offdiag) t0 *= 2.0;
        if (tid == 0) {
          double* spb = a.sp + ((unsigned)buf * G + blk) * 4;
          cstore(&spb[0], t0);
          cstore(&spb[1], t1);
          cstore(&spb[2], t2);
          // alpha = u_{j+1} (pivot row q = jj) and d_j = updated A(j, j), read
          // before the barrier: owners overwrite column j right after it.
          sc[0] = ajj - 2.0 * pd;
          sc[3] = (double)PU[jj];
        }
      }
    }

    const bool released = grid_arrive(a.bar, a.bar_base, sub_base, blk, G, kb0 + jj + 1);
    // While the barrier completes: this thread's row share of the next
    // column's correction, up_i = sum_{t < jj} V(i,t) W(jn,t) + W(i,t) V(jn,t)
    // for jn = j+1 (row jn's coefficients are pivot row jj).  It reads only
    // panel coefficients of earlier columns; the t = jj term is added once
    // this column's pivot row is finished.
    const int qp = jj + tid - kPivT;  // pivot row of this thread
    const bool pivt = tid >= kPivT && tid < kPivT + kNbMax && qp < nb;
    T upr = T(0);
    {
      auto upsum = [&](auto Vt, auto Wt) {
        T us = T(0);
        for (int t = 0; t < jj; ++t) us += Vt(t) * PW[jj][t] + Wt(t) * PV[jj][t];
        return us;
      };
      if (pivt && p + 1 + qp < n) upr = upsum([&](int t) { return PV[qp][t]; }, [&](int t) { return PW[qp][t]; });
      if (tid < nI && I0 + tid >= j + 1)
        upr = upsum([&](int t) { return PVI[t * kMaxTs + tid]; }, [&](int t) { return PWI[t * kMaxTs + tid]; });
      if (offdiag && tid >= kKT && tid - kKT < nK && K0 + tid - kKT >= j + 1) {
        const int r = tid - kKT;
        upr = upsum([&](int t) { return PVK[t * kMaxTs + r]; }, [&](int t) { return PWK[t * kMaxTs + r]; });
      }
    }
    grid_wait(a.bar, a.bar_base, kb0 + jj + 1, released);

    // ---- gather the partial sums of all workgroups into LDS in parallel
    // (one load per thread), then reduce them there.
    // All loads of the gather are issued before any result is stored, so
    // they share one round trip.
    static_assert(kGMax <= kThreads && kTRMax * 2 * kNbMax <= 2 * kThreads, "gather split");
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, gv0 = 0.0, gv1 = 0.0;
    const int nvp = TR * 2 * jj;
    if (tid < G) {
      const double* spb = a.sp + ((unsigned)buf * G + tid) * 4;
      g0 = cload(&spb[0]);
      g1 = cload(&spb[1]);
      g2 = cload(&spb[2]);
    }
    if (tid < nvp) gv0 = cload(&a.vp[((unsigned)buf * TR + tid / (2 * jj)) * (2 * kNbMax) + tid % (2 * jj)]);
    if (tid + kThreads < nvp) {
      const int x = tid + kThreads;
      gv1 = cload(&a.vp[((unsigned)buf * TR + x / (2 * jj)) * (2 * kNbMax) + x % (2 * jj)]);
    }
    // (A22 u)_i = sum of the TR partial products of row i, for the rows of I,
    // K and the pivot rows: all loads of a row issued together.
    {
      auto rowsum = [&](int i) -> T {
        T yv[kTRMax];
#pragma unroll
        for (int b = 0; b < kTRMax; ++b) yv[b] = (b < TR) ? cload(&a.ypart[((unsigned)buf * TR + b) * n + i]) : T(0);
        T z = T(0);
#pragma unroll
        for (int b = 0; b < kTRMax; ++b) z += yv[b];
        return z;
      };
      if (tid < nI) yzI[tid] = (I0 + tid >= j + 1) ? rowsum(I0 + tid) : T(0);
      if (offdiag && tid >= kKT && tid - kKT < nK) {
        const int r = tid - kKT;
        yzK[r] = (K0 + r >= j + 1) ? rowsum(K0 + r) : T(0);
      }
      if (tid >= kThreads - kNbMax) {
        const int q = tid - (kThreads - kNbMax);
        const int r = p + 1 + q;
        yzP[q] = (q < nb && r >= j + 1 && r < n) ? rowsum(r) : T(0);
      }
    }
    if (tid < G) {
      spl[0][tid] = g0;
      spl[1][tid] = g1;
      spl[2][tid] = g2;
    }
    if (tid < nvp) vpl[tid] = gv0;
    if (tid + kThreads < nvp) vpl[tid + kThreads] = gv1;
    __syncthreads();
    // Wave 0 reduces the scalars and forms the reflector while waves 8-15 sum
    // the row tiles' V^T u and W^T u (8 lanes per panel column).
    if (tid < kWave) {
      double uAu = 0.0, sig = 0.0, ua1 = 0.0;
      for (int b = tid; b < G; b += kWave) uAu += spl[0][b];
      for (int t = tid; t < TR; t += kWave) {
        const int b = t * (t + 1) / 2 + t;  // diagonal tile (t, t)
        sig += spl[1][b];
        ua1 += spl[2][b];
      }
      uAu = wsum(uAu);
      sig = wsum(sig);
      ua1 = wsum(ua1);
      if (tid == 0) {
        const double alpha = sc[3];
        double beta, tau, c;
        if (sig == 0.0) {
          beta = alpha; tau = 0.0; c = 0.0;
        } else {
          beta = -copysign(sqrt(alpha * alpha + sig), alpha);
          tau = (beta - alpha) / beta;
          c = 1.0 / (alpha - beta);
        }
        if (blk == 0) {
          a.d[j] = (T)sc[0];
          a.e[j] = (T)beta;
          a.tau[j] = (T)tau;
        }
        sc[0] = uAu; sc[1] = sig; sc[2] = ua1;
        sc[4] = beta; sc[5] = tau; sc[6] = c;
      }
    } else if (tid >= kThreads / 2) {
      static_assert(kThreads / 2 >= 2 * kNbMax * 8, "8 lanes per panel column");
      const int x = tid - kThreads / 2, c2 = x >> 3, l8 = x & 7;
      double sv = 0.0;
      if (c2 < 2 * jj)
        for (int b = l8; b < TR; b += 8) sv += vpl[b * 2 * jj + c2];
      sv = hsum8(sv);
      if (l8 == 0 && c2 < 2 * jj) vts[c2] = sv;
    }
    __syncthreads();
    // V^T v and W^T v (length jj; V(j+1, :), W(j+1, :) are pivot row jj) and
    // w0^T v, in wave 0
    if (tid < kWave) {
      const double beta = sc[4], tau = sc[5], c = sc[6];
      double vw = 0.0;
      if (tid < jj) {
        const T vt = (T)(c * (vts[tid] - beta * (double)PV[jj][tid]));
        const T wt = (T)(c * (vts[jj + tid] - beta * (double)PW[jj][tid]));
        VTv[tid] = (double)vt;
        WTv[tid] = (double)wt;
        vw = (double)vt * (double)wt;
      }
      vw = wsum(vw);
      if (tid == 0) {
        const double a11 = (double)acP[jj];
        const double vAv = c * c * (sc[0] - 2.0 * beta * sc[2] + beta * beta * a11);
        sc[7] = tau * (vAv - 2.0 * vw);  // w0^T v
      }
    }
    __syncthreads();
    const double beta = sc[4], tau = sc[5], c = sc[6];
    const double wv = sc[7];
    const bool zero_refl = (sc[1] == 0.0);

    // y_i, v_i, w_i of the current column for a row i >= j+1, given u_i,
    // (A22 u)_i, a1_i = A(i, j+1) and the row's panel coefficients.
    auto finish = [&](int i, T ui, T yzi, T a1i, auto Vt, auto Wt, T& vi, T& wi) {
      double ys = 0.0;
      for (int t = 0; t < jj; ++t) {
        const T vt = Vt(t), wt = Wt(t);
        ys += (double)vt * WTv[t] + (double)wt * VTv[t];
      }
      if (zero_refl) {
        vi = (i == j + 1) ? T(1) : T(0);
        wi = T(0);
        return;
      }
      const double y = c * ((double)yzi - beta * (double)a1i) - ys;
      const double v = (i == j + 1) ? 1.0 : c * (double)ui;
      vi = (T)v;
      wi = (T)(tau * y - 0.5 * tau * wv * v);
    };

    // Each thread finishes at most one row: a pivot row (every workgroup:
    // rows p+1+q >= j+1, i.e. q >= jj), a row of I or a row of K.  The
    // diagonal tile's workgroup owns its rows and publishes V, W and the
    // explicit reflector column A(:, j).
    T vr = T(0), wr = T(0);
    if (pivt) {
      const int r = p + 1 + qp;
      if (r < n)
        finish(r, PU[qp], yzP[qp], acP[qp], [&](int t) { return PV[qp][t]; }, [&](int t) { return PW[qp][t]; }, vr, wr);
      PV[qp][jj] = vr;
      PW[qp][jj] = wr;
    }
    if (tid < nI) {
      const int r = tid, i = I0 + r;
      if (i >= j + 1)
        finish(i, uI[r], yzI[r], acI[r], [&](int t) { return PVI[t * kMaxTs + r]; }, [&](int t) { return PWI[t * kMaxTs + r]; },
               vr, wr);
      PVI[jj * kMaxTs + r] = vr;
      PWI[jj * kMaxTs + r] = wr;
      if (diag) {
        a.VW[i + (unsigned)jj * ld] = vr;
        a.VW[i + (unsigned)(nb + jj) * ld] = wr;
        a.WV[i + (unsigned)jj * ld] = wr;
        a.WV[i + (unsigned)(nb + jj) * ld] = vr;
        A[i + (unsigned)j * ld] = vr;
      }
    }
    if (offdiag && tid >= kKT && tid - kKT < nK) {
      const int r = tid - kKT, i = K0 + r;
      if (i >= j + 1)
        finish(i, uK[r], yzK[r], acK[r], [&](int t) { return PVK[t * kMaxTs + r]; }, [&](int t) { return PWK[t * kMaxTs + r]; },
               vr, wr);
      PVK[jj * kMaxTs + r] = vr;
      PWK[jj * kMaxTs + r] = wr;
    }
    __syncthreads();
    if (jj + 1 == nb) break;
    // ---- next column jn = j+1: u_i = A(i, jn) - up_i - (V(i,jj) W(jn,jj) + W(i,jj) V(jn,jj))
    const int jn = j + 1;
    const T pwj = PW[jj][jj], pvj = PV[jj][jj];
    if (tid < nI) {
      const int r = tid;
      uI[r] = (I0 + r >= jn + 1) ? acI[r] - upr - (vr * pwj + wr * pvj) : T(0);
      if (diag && r < nK) uK[r] = uI[r];  // same rows
    }
    if (offdiag && tid >= kKT && tid - kKT < nK) {
      const int r = tid - kKT;
      uK[r] = (K0 + r >= jn + 1) ? acK[r] - upr - (vr * pwj + wr * pvj) : T(0);
    }
    if (pivt && qp >= jj + 1) PU[qp] = (p + 1 + qp < n) ? acP[qp] - upr - (vr * pwj + wr * pvj) : T(0);
    __syncthreads();
  }
}

// Last diagonal entry (one block per batch entry), with the last panel's
// trailing update over w2 columns of VW and WV when no GEMM applied it.
template <typename T>
__global__ void copy_last_diag(const T* A, int n, T* d, int64_t sA, int64_t sD, const T* VW,
                               const T* WV, int64_t sVW, int w2) {
  const int64_t b = blockIdx.x;
  if (threadIdx.x == 0) {
    T v = A[b * sA + (n - 1) + (int64_t)(n - 1) * n];
    T corr = T(0);
    for (int t = 0; t < w2; ++t)
      corr += VW[b * sVW + (n - 1) + (int64_t)t * n] * WV[b * sVW + (n - 1) + (int64_t)t * n];
    d[b * sD + n - 1] = v - corr;
  }
}

}  // namespace

int sytrd_max_n() { return kTRMax * kMaxTs + 1; }
static_assert((int64_t)(kTRMax * kMaxTs + 1) * (kTRMax * kMaxTs + 1) < (int64_t(1) << 31),
              "the panel kernel's 32-bit offsets cover an n x n matrix");

template <typename T>
void sytrd_batched(hipStream_t st, int n, int batch, T* A, int64_t sA, T* d, T* e, T* tau,
                   int64_t sD, SytrdWork& w) {
  if (n <= 0 || batch <= 0) return;
  if (n == 1) {
    hipLaunchKernelGGL(copy_last_diag<T>, dim3(batch), 64, 0, st, (const T*)A, n, d, sA, sD,
                       (const T*)nullptr, (const T*)nullptr, (int64_t)0, 0);
    MSQRT_LAUNCH_CHECK();
    return;
  }
  if (n > sytrd_max_n())
    throw Error{MSQRT_ERR_UNSUPPORTED, "tridiagonal reduction supports n <= 4225 in this build"};
  // Panel width: the LDS cache holds 4 * nb * kMaxTs values (at most 128 KiB).
  const int lds_budget = sizeof(T) == 4 ? 128 * 1024 : 96 * 1024;
  const int nb = std::min(kNbMax, (int)(lds_budget / (4 * kMaxTs * (int)sizeof(T))));
  const size_t dyn_lds = (size_t)4 * nb * kMaxTs * sizeof(T);
  static bool attr_set[2] = {false, false};
  static int resident[2] = {0, 0};  // co-resident workgroups of the panel kernel
  if (!attr_set[sizeof(T) == 8]) {
    MSQRT_HIP(hipFuncSetAttribute((const void*)sytrd_panel_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds));
    int per_cu = 0, ncu = 0, dev = 0;
    MSQRT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, (const void*)sytrd_panel_kernel<T>, kThreads, dyn_lds));
    MSQRT_HIP(hipGetDevice(&dev));
    MSQRT_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    resident[sizeof(T) == 8] = std::max(1, per_cu) * std::max(1, ncu);
    attr_set[sizeof(T) == 8] = true;
  }
  const int64_t sVW = (int64_t)n * 2 * kNbMax, sYP = (int64_t)2 * kTRMax * n,
                sSP = (int64_t)2 * kGMax * 4, sVP = (int64_t)2 * kTRMax * 2 * kNbMax, sBar = 32 * 40;
  T* VW = w.VW.ensure<T>(sVW * batch);
  T* WV = w.WV.ensure<T>(sVW * batch);
  T* ypart = w.ypart.ensure<T>(sYP * batch);
  double* sp = w.sp.ensure<double>(sSP * batch);
  double* vp = w.vp.ensure<double>(sVP * batch);
  unsigned* bar = w.bar.ensure<unsigned>(sBar * batch);
  MSQRT_HIP(hipMemsetAsync(bar, 0, sizeof(unsigned) * (size_t)(sBar * batch), st));
  w.nbar = batch;
  BarrierBase bar_base{};
  // float panels apply the previous panel's trailing update themselves
  constexpr bool kFused = sizeof(T) == 4;
  int nbp = 0;
  for (int p = 0; p < n - 1; p += nb) {
    const int nbe = std::min(nb, n - 1 - p);
    const int m = n - 1 - p;  // rows/cols of the tile region [p+1, n)
    const int TR = (int)std::min<int64_t>(kTRMax, std::max<int64_t>(1, ceil_div(m, kMaxTs)));
    const int ts = (int)ceil_div(m, TR);
    const int G = TR * (TR + 1) / 2;
    // as many batch entries per cooperative launch as fit co-resident
    const int chunk = std::max(1, resident[sizeof(T) == 8] / G);
    const int tok = prof_begin(st);
    for (int b0 = 0; b0 < batch; b0 += chunk) {
      const int nbt = std::min(chunk, batch - b0);
      PanelArgs<T> pa{n,          p,          nbe,        kFused ? nbp : 0, TR,      p + 1,         ts,
                      A + b0 * sA, VW + b0 * sVW, WV + b0 * sVW, d + b0 * sD, e + b0 * sD,
                      tau + b0 * sD, ypart + b0 * sYP, sp + b0 * sSP, vp + b0 * sVP,
                      bar + b0 * sBar, bar_base, sA, sVW, sD, sYP, sSP, sVP, sBar};
      void* args[] = {&pa};
      MSQRT_HIP(hipLaunchCooperativeKernel((const void*)sytrd_panel_kernel<T>, dim3(G, nbt),
                                           dim3(kThreads), args, dyn_lds, st));
    }
    const unsigned nbar = (unsigned)nbe + ((kFused && nbp > 0) ? 1u : 0u);  // barriers of the launch
    bar_base.gen += nbar;
    bar_base.top += (unsigned)std::min(G, 8) * nbar;
    for (int g = 0; g < 8; ++g) bar_base.sub[g] += (unsigned)(G / 8 + (g < G % 8 ? 1 : 0)) * nbar;
    if (tok >= 0) {
      // algorithmic traffic: one read of the symmetric trailing matrix (lower
      // triangle) per column for its product with the reflector, and, when
      // the launch applies the previous panel's update, one read and one
      // write of that triangle
      double bytes = 0.0, flops = 4.0 * 0.5 * (double)m * m * nbe;
      for (int jj = 0; jj < nbe; ++jj) {
        const double mj = (double)(n - 1 - (p + jj));
        bytes += 0.5 * mj * (mj + 1.0) * sizeof(T);
      }
      if (kFused && p > 0) {
        bytes += 2.0 * 0.5 * (double)m * (m + 1.0) * sizeof(T);
        flops += 2.0 * 0.5 * (double)m * (m + 1.0) * (2.0 * nbp);
      }
      prof_end(tok, st, sizeof(T) == 4 ? "sytrd_panel_f32" : "sytrd_panel_f64", flops * batch,
               bytes * batch);
    }
    nbp = nbe;
    // Trailing update A(q:n, q:n) -= [V W] [W V]^T, q = p + nbe, all entries
    // (float: applied by the next panel, or below for the last entry).
    const int q = p + nbe;
    if (!kFused && q < n) {
      const int mt = n - q;
      if (std::is_same<T, float>::value)
        gemm_store_f32(st, false, true, mt, mt, 2 * nbe, (const float*)(VW + q), n, sVW,
                       (const float*)(WV + q), n, sVW, (float*)(A + q + (int64_t)q * n), n, sA,
                       -1.f, 1.f, batch, true);
      else
        gemm_store_f64(st, false, true, mt, mt, 2 * nbe, (const double*)(VW + q), n, sVW,
                       (const double*)(WV + q), n, sVW, (double*)(A + q + (int64_t)q * n), n, sA,
                       -1.0, 1.0, batch, true);
    }
  }
  hipLaunchKernelGGL(copy_last_diag<T>, dim3(batch), 64, 0, st, (const T*)A, n, d, sA, sD,
                     (const T*)VW, (const T*)WV, sVW, kFused ? 2 * nbp : 0);
  MSQRT_LAUNCH_CHECK();
}

template <typename T>
void sytrd(hipStream_t st, int n, T* A, T* d, T* e, T* tau, SytrdWork& w) {
  sytrd_batched<T>(st, n, 1, A, (int64_t)n * n, d, e, tau, 0, w);
}

bool sytrd_failed(SytrdWork& w) {
  if (!w.bar.p || w.nbar <= 0) return false;
  std::vector<unsigned> flags((size_t)32 * 40 * w.nbar);
  MSQRT_HIP(hipMemcpy(flags.data(), w.bar.p, sizeof(unsigned) * flags.size(), hipMemcpyDeviceToHost));
  for (int b = 0; b < w.nbar; ++b)
    if (flags[(size_t)b * 32 * 40 + kBarFail]) return true;
  return false;
}

template void sytrd<float>(hipStream_t, int, float*, float*, float*, float*, SytrdWork&);
template void sytrd<double>(hipStream_t, int, double*, double*, double*, double*, SytrdWork&);
template void sytrd_batched<float>(hipStream_t, int, int, float*, int64_t, float*, float*, float*,
                                   int64_t, SytrdWork&);
template void sytrd_batched<double>(hipStream_t, int, int, double*, int64_t, double*, double*,
                                    double*, int64_t, SytrdWork&);

}  // namespace msqrt
