// Blocked triangular square root and triangular Sylvester solver on 32 x 32
// tiles, as one persistent kernel with tile-level dataflow.
//
// Triangular root (Sec. 2, blocked form of Eq. (subst)): for tiles I <= J of
// the upper triangular T,
//   diagonal tiles:  S_II = T_II^{1/2} by the recurrence
//                    s_ii = t_ii^{1/2},  s_ij = (t_ij - sum_{i<k<j} s_ik s_kj) / (s_ii + s_jj);
//   off-diagonal:    S_II S_IJ + S_IJ S_JJ = T_IJ - sum_{I<K<J} S_IK S_KJ.
// Triangular Sylvester S Y + Y S2 = C (the correction equation of Alg. 2 and
// the solver of Alg. 1): for every tile
//   S_II Y_IJ + Y_IJ S2_JJ = C_IJ - sum_{K>I} S_IK Y_KJ - sum_{K<J} Y_IK S2_KJ,
// which is the order in which Alg. 1's recursion produces the blocks (rows
// bottom-up, columns left to right).  Each tile's small Sylvester equation is
// solved by substitution along its anti-diagonals.
//
// Every workgroup takes one tile from an atomic ticket in wavefront order, so
// every tile a workgroup waits for was taken by a workgroup that is already
// running: the dataflow cannot deadlock, whatever the dispatch order.  Finished tiles
// are exchanged with agent-scope atomic accesses and published with a
// per-tile flag after the stores have completed; waits are bounded and a
// timed-out wait sets a sticky error flag.
#include <algorithm>

#include "gemm.hpp"
#include "kernels.hpp"
#include "schur.hpp"

namespace msqrt {

namespace {

constexpr int kTb = 32;
constexpr int kTThreads = 256;
static_assert(kTThreads == 4 * kWave, "one wave per real product of a complex tile product");
constexpr unsigned kSpinLimit = 1u << 22;

struct TileArgs {
  int mode;  // 0 = square root, 1 = Sylvester
  int m, p, mt, pt, ntiles;
  int64_t lda, ldb, ldx;
  int* flags;
  int* ticket;
  int* err;  // [0] wait timed out, [1] eigenvalue on R<=0
};

template <typename T>
__device__ inline cx<T> tload(const T* P, int64_t ld, int64_t i, int64_t j) {
  return {P[i + j * ld], P[i + j * ld + ld / 2]};
}
// Tiles produced by other workgroups are exchanged through agent-scope
// atomic loads and stores, which are coherent across the XCDs' L2 caches
// without writing back or invalidating the caches (the fences that would
// otherwise be needed flush the whole L2 on every publish and wait).
template <typename T>
__device__ inline cx<T> tload_c(const T* P, int64_t ld, int64_t i, int64_t j) {
  T* q = const_cast<T*>(P) + i + j * ld;
  return {__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
          __hip_atomic_load(q + ld / 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}
template <typename T>
__device__ inline void tstore_c(T* P, int64_t ld, int64_t i, int64_t j, cx<T> v) {
  T* q = P + i + j * ld;
  __hip_atomic_store(q, v.r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + ld / 2, v.i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront order of the tiles.
__device__ inline void tile_of(const TileArgs& a, int tk, int& I, int& J) {
  if (a.mode == 0) {
    int d = 0, base = 0;
    while (base + (a.mt - d) <= tk) { base += a.mt - d; ++d; }
    I = tk - base;
    J = I + d;
    return;
  }
  int base = 0;
  for (int d = 0;; ++d) {
    const int ilo = max(0, a.mt - 1 - d), ihi = min(a.mt - 1, a.mt - 1 - d + a.pt - 1);
    const int cnt = ihi - ilo + 1;
    if (cnt > 0 && tk < base + cnt) {
      I = ihi - (tk - base);
      J = d - (a.mt - 1 - I);
      return;
    }
    if (cnt > 0) base += cnt;
  }
}

__device__ inline void wait_tile(const TileArgs& a, int I, int J) {
  // Wave 0 spins as a whole (every lane loads the same flag; the values are
  // made uniform with readfirstlane), so no single-lane branch sits inside
  // the barrier-carrying loops of the caller.
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
  if (wave == 0) {
    int* f = &a.flags[I * a.pt + J];
    for (unsigned spins = 0;; ++spins) {
      if (__builtin_amdgcn_readfirstlane(
              __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
        break;
      if (__builtin_amdgcn_readfirstlane(
              __hip_atomic_load(&a.err[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
        break;
      if (spins > kSpinLimit) {
        __hip_atomic_store(&a.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

// Loads a tile (rows r0.., cols c0.., extent mr x mc, zero padded) to LDS;
// coherent = the tile was produced by another workgroup of this launch.
template <typename T>
__device__ inline void load_tile(cx<T> (*dst)[kTb + 1], const T* P, int64_t ld, int r0, int c0,
                                 int mr, int mc, bool coherent) {
  for (int x = threadIdx.x; x < kTb * kTb; x += blockDim.x) {
    const int i = x % kTb, j = x / kTb;
    cx<T> v = {T(0), T(0)};
    if (i < mr && j < mc) v = coherent ? tload_c(P, ld, r0 + i, c0 + j) : tload(P, ld, r0 + i, c0 + j);
    dst[j][i] = v;
  }
}

// The four real products of one complex 32 x 32 x 32 tile product C = A B
// on MFMA, one per wave: P0 = Ar Br, P1 = Ai Bi, P2 = Ar Bi, P3 = Ai Br
// (so Cr = P0 - P1, Ci = P2 + P3), stored to P[w][col][row].  A and B are
// the LDS tiles As[k][i] = A(i, k), Bs[j][k] = B(k, j).
template <typename T>
__device__ inline void tile_product_mfma(const cx<T> (*As)[kTb + 1], const cx<T> (*Bs)[kTb + 1],
                                         T (*P)[kTb][kTb + 1], int wave, int lane) {
  // P may overlay As and Bs: every wave reads its operands before any stores
  using M = Mfma<T>;
  constexpr int NT = kTb / M::TM;  // MFMA tiles per dimension
  const bool aim = wave == 1 || wave == 3, bim = wave == 1 || wave == 2;
  typename M::acc_t acc[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[i][j][r] = T(0);
  const int fmn = M::frag_mn(lane);
#pragma unroll
  for (int k0 = 0; k0 < kTb; k0 += M::TK) {
    const int fk = k0 + M::frag_k(lane);
    T av[NT], bv[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const cx<T> v = As[fk][i * M::TM + fmn];
      av[i] = aim ? v.i : v.r;
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const cx<T> v = Bs[j * M::TN + fmn][fk];
      bv[j] = bim ? v.i : v.r;
    }
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = M::mma(av[i], bv[j], acc[i][j]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r)
        P[wave][j * M::TN + M::c_col(lane, r)][i * M::TM + M::c_row(lane, r)] = acc[i][j][r];
}

template <typename T>
__global__ __launch_bounds__(kTThreads) void tile_kernel(TileArgs a, const T* A, const T* B, T* X) {
  // A and B operand tiles ([col][row]) in one array: after the MFMA products
  // have read them, the same storage holds the four real products
  __shared__ cx<T> ABs[2][kTb][kTb + 1];
  cx<T> (*As)[kTb + 1] = ABs[0];
  cx<T> (*Bs)[kTb + 1] = ABs[1];
  T (*Pp)[kTb][kTb + 1] = reinterpret_cast<T (*)[kTb][kTb + 1]>(&ABs[0][0][0]);
  static_assert(sizeof(ABs) == 4 * kTb * (kTb + 1) * sizeof(T), "product overlay");
  __shared__ cx<T> Ys[kTb][kTb + 1];
  __shared__ int sh_tk;
  const int t = threadIdx.x;
  const int ti = t % kTb, tj0 = t / kTb;  // owned entries (ti, tj0 + 8 q)
  const int wave = __builtin_amdgcn_readfirstlane(t / kWave);
  {
    // One ticket per workgroup, taken by wave 0 as a whole: lane 0 adds 1,
    // the other lanes add 0, and lane 0's old value is broadcast.  The
    // ticket and everything derived from it (tile, loop bounds around the
    // barriers) are uniform, so the compiler emits only uniform branches
    // around barriers.
    if (wave == 0) {
      const int old = atomicAdd(a.ticket, t == 0 ? 1 : 0);
      sh_tk = __builtin_amdgcn_readfirstlane(old);
    }
    __syncthreads();
  }
  const int tk = __builtin_amdgcn_readfirstlane(sh_tk);
  if (tk >= a.ntiles) return;
  {
    int I, J;
    tile_of(a, tk, I, J);
    const int mi = min(kTb, a.m - kTb * I), mj = min(kTb, a.p - kTb * J);
    // right-hand side
    cx<T> acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = tj0 + 8 * q;
      acc[q] = (ti < mi && j < mj)
                   ? tload(a.mode == 0 ? A : X, a.mode == 0 ? a.lda : a.ldx, kTb * I + ti, kTb * J + j)
                   : cx<T>{T(0), T(0)};
    }
    auto subtract = [&]() {
      __syncthreads();
      tile_product_mfma<T>(As, Bs, Pp, wave, t % kWave);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = tj0 + 8 * q;
        acc[q].r -= Pp[0][j][ti] - Pp[1][j][ti];
        acc[q].i -= Pp[2][j][ti] + Pp[3][j][ti];
      }
      __syncthreads();
    };
    if (a.mode == 0 && I == J) {
      // diagonal tile: the recurrence of Eq. (subst) by superdiagonals
#pragma unroll
      for (int q = 0; q < 4; ++q) Ys[tj0 + 8 * q][ti] = acc[q];  // T_II into Ys
      __syncthreads();
      if (t < mi) {
        const cx<T> d = Ys[t][t];
        // on or within a few ulps of the closed negative real axis
        const T eps = sizeof(T) == 4 ? T(5.9604645e-08) : T(1.1102230246251565e-16);
        if (d.r <= T(0) && fabs(d.i) <= T(16) * eps * fabs(d.r)) atomicOr(&a.err[1], 1);
        As[t][t] = csqrt_principal(d);
      }
      __syncthreads();
      for (int d = 1; d < mi; ++d) {
        if (t < mi - d) {
          const int i = t, j = t + d;
          cx<T> s = Ys[j][i];
          for (int k = i + 1; k < j; ++k) s = csub(s, cmul(As[k][i], As[j][k]));
          As[j][i] = cdiv(s, cadd(As[i][i], As[j][j]));
        }
        __syncthreads();
      }
      for (int x = t; x < kTb * kTb; x += blockDim.x) {
        const int i = x % kTb, j = x / kTb;
        if (i < mi && j < mj) tstore_c(X, a.ldx, kTb * I + i, kTb * J + j, i <= j ? As[j][i] : cx<T>{T(0), T(0)});
      }
    } else {
      if (a.mode == 0) {
        // S_IK S_KJ is ready once tiles (I, K) and (K, J) are, i.e. at
        // superdiagonal max(K - I, J - K): take K from the middle outwards
        const int klo = I + 1, khi = J - 1, cnt = khi - klo + 1, mid = (I + J) / 2;
        for (int q = 0, done = 0; done < cnt; ++q) {
          const int K = mid + ((q & 1) ? (q + 1) / 2 : -(q / 2));
          if (K < klo || K > khi) continue;
          ++done;
          wait_tile(a, I, K);
          wait_tile(a, K, J);
          const int mk = min(kTb, a.m - kTb * K);
          load_tile(As, X, a.ldx, kTb * I, kTb * K, mi, mk, true);
          load_tile(Bs, X, a.ldx, kTb * K, kTb * J, mk, mj, true);
          subtract();
        }
        wait_tile(a, I, I);
        wait_tile(a, J, J);
        load_tile(As, X, a.ldx, kTb * I, kTb * I, mi, mi, true);
        load_tile(Bs, X, a.ldx, kTb * J, kTb * J, mj, mj, true);
      } else {
        // the column terms S_IK Y_KJ (K > I, ready at wavefront
        // mt-1-K+J) and the row terms Y_IK S2_KJ (K < J, ready at mt-1-I+K)
        // are taken merged in order of readiness, so that only the last two
        // products remain once the final dependencies arrive
        int kc = a.mt - 1, kr = 0;
        while (kc > I || kr < J) {
          const int dc = kc > I ? a.mt - 1 - kc + J : 1 << 30;
          const int dr = kr < J ? a.mt - 1 - I + kr : 1 << 30;
          if (dc <= dr) {
            const int K = kc--;
            wait_tile(a, K, J);
            const int mk = min(kTb, a.m - kTb * K);
            load_tile(As, A, a.lda, kTb * I, kTb * K, mi, mk, false);
            load_tile(Bs, X, a.ldx, kTb * K, kTb * J, mk, mj, true);
          } else {
            const int K = kr++;
            wait_tile(a, I, K);
            const int mk = min(kTb, a.p - kTb * K);
            load_tile(As, X, a.ldx, kTb * I, kTb * K, mi, mk, true);
            load_tile(Bs, B, a.ldb, kTb * K, kTb * J, mk, mj, false);
          }
          subtract();
        }
        load_tile(As, A, a.lda, kTb * I, kTb * I, mi, mi, false);
        load_tile(Bs, B, a.ldb, kTb * J, kTb * J, mj, mj, false);
      }
      __syncthreads();
      // S_II Y + Y S2_JJ = acc by anti-diagonals e = (mi - 1 - i) + j
      const int ne = mi + mj - 1;
      for (int e = 0; e < ne; ++e) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = tj0 + 8 * q;
          if (ti < mi && j < mj && (mi - 1 - ti) + j == e)
            Ys[j][ti] = cdiv(acc[q], cadd(As[ti][ti], Bs[j][j]));
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = tj0 + 8 * q;
          if (ti < mi && j < mj && (mi - 1 - ti) + j > e) {
            const int k = mi - 1 - e + j;  // (k, j) on wavefront e
            if (k > ti && k < mi) acc[q] = csub(acc[q], cmul(As[k][ti], Ys[j][k]));
            const int k2 = e - (mi - 1 - ti);  // (ti, k2) on wavefront e
            if (k2 >= 0 && k2 < j) acc[q] = csub(acc[q], cmul(Ys[k2][ti], Bs[j][k2]));
          }
        }
      }
      __syncthreads();
      for (int x = t; x < kTb * kTb; x += blockDim.x) {
        const int i = x % kTb, j = x / kTb;
        if (i < mi && j < mj) tstore_c(X, a.ldx, kTb * I + i, kTb * J + j, Ys[j][i]);
      }
    }
    // every wave waits for its coherent stores to complete before the tile
    // is published
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (wave == 0)
      __hip_atomic_store(&a.flags[I * a.pt + J], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T>
void launch_tiles(hipStream_t st, TileArgs a, const T* A, const T* B, T* X, TrsylvWork& w) {
  const int nflags = a.mt * a.pt;
  int* buf = w.flags.ensure<int>(nflags + 64);
  a.flags = buf;
  a.ticket = buf + nflags;
  const bool fresh = w.ticket.p == nullptr;
  a.err = w.ticket.ensure<int>(4);
  if (fresh) MSQRT_HIP(hipMemsetAsync(a.err, 0, sizeof(int) * 4, st));
  MSQRT_HIP(hipMemsetAsync(buf, 0, sizeof(int) * (nflags + 64), st));
  // one workgroup per tile; tiles are taken in ticket (wavefront) order, so a
  // workgroup only ever waits for tiles held by workgroups already running
  const int grid = a.ntiles;
  if (grid <= 0) return;
  hipLaunchKernelGGL(tile_kernel<T>, dim3(grid), dim3(kTThreads), 0, st, a, A, B, X);
  MSQRT_LAUNCH_CHECK();
}

}  // namespace

void trsylv_reset(hipStream_t st, TrsylvWork& w) {
  int* e = w.ticket.ensure<int>(4);
  MSQRT_HIP(hipMemsetAsync(e, 0, sizeof(int) * 4, st));
}

// err[0]: a wait timed out; err[1]: a diagonal entry on R<=0.
void trsylv_errors(hipStream_t st, TrsylvWork& w, int* timed_out, int* nonprincipal) {
  int h[4] = {0, 0, 0, 0};
  if (w.ticket.p) {
    MSQRT_HIP(hipMemcpyAsync(h, w.ticket.p, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
    MSQRT_HIP(hipStreamSynchronize(st));
  }
  if (timed_out) *timed_out = h[0];
  if (nonprincipal) *nonprincipal = h[1];
}

template <typename T>
void trsqrt(hipStream_t st, int n, const T* Tm, T* S, TrsylvWork& w, int* bad) {
  (void)bad;
  if (n <= 0) return;
  const int64_t ld = 2 * (int64_t)n;
  MSQRT_HIP(hipMemsetAsync(S, 0, sizeof(T) * ld * n, st));
  TileArgs a{};
  a.mode = 0;
  a.m = a.p = n;
  a.mt = a.pt = (int)ceil_div(n, kTb);
  a.ntiles = a.mt * (a.mt + 1) / 2;
  a.lda = ld;
  a.ldb = ld;
  a.ldx = ld;
  launch_tiles<T>(st, a, Tm, Tm, S, w);
}

template <typename T>
void trsyl(hipStream_t st, int m, int p, const T* S, int64_t lds, const T* S2, int64_t lds2, T* C,
           int64_t ldc, TrsylvWork& w) {
  if (m <= 0 || p <= 0) return;
  TileArgs a{};
  a.mode = 1;
  a.m = m;
  a.p = p;
  a.mt = (int)ceil_div(m, kTb);
  a.pt = (int)ceil_div(p, kTb);
  a.ntiles = a.mt * a.pt;
  a.lda = lds;
  a.ldb = lds2;
  a.ldx = ldc;
  launch_tiles<T>(st, a, S, S2, C, w);
}

template void trsqrt<float>(hipStream_t, int, const float*, float*, TrsylvWork&, int*);
template void trsqrt<double>(hipStream_t, int, const double*, double*, TrsylvWork&, int*);
template void trsyl<float>(hipStream_t, int, int, const float*, int64_t, const float*, int64_t,
                           float*, int64_t, TrsylvWork&);
template void trsyl<double>(hipStream_t, int, int, const double*, int64_t, const double*, int64_t,
                            double*, int64_t, TrsylvWork&);

}  // namespace msqrt
