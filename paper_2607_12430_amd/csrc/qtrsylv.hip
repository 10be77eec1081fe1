// Tile solvers of the real route: square root of a quasi-upper-triangular T
// and the Sylvester equation S Y + Y S2 = C with quasi-upper-triangular S and
// S2 (1x1 and 2x2 diagonal blocks, the real Schur form of the remark on real
// input in Sec. 2.2.1).  Same dataflow as the complex tile solver: one
// persistent launch, one workgroup per tile taken from an atomic ticket in
// wavefront order, finished tiles published with per-tile flags after their
// agent-scope stores have completed, bounded waits with a sticky error flag.
//
// Tiles have at most 32 rows; their boundaries come from the host
// (quasi_partition): nominally every 32 rows, one row earlier where a
// boundary would separate the two rows of a 2x2 diagonal block, so that no
// 2x2 block is ever cut.  Inside a tile the diagonal blocks are the units:
//   root:       U_ii = T_ii^{1/2} (scalar root, or for a 2x2 block the
//               Cayley-Hamilton form (B + d I) / t, d = det(B)^{1/2},
//               t = (tr B + 2 d)^{1/2}), then by block superdiagonals
//               U_ii U_ij + U_ij U_jj = T_ij - sum_{i<k<j} U_ik U_kj;
//   Sylvester:  by block anti-diagonals,
//               S_ii Y_ij + Y_ij S2_jj = C_ij - (finished blocks),
// each block equation (at most 4 unknowns) solved in its Kronecker form by
// elimination with partial pivoting.
#include <algorithm>

#include "gemm.hpp"
#include "kernels.hpp"
#include "schur.hpp"

namespace msqrt {

namespace {

constexpr int kQb = 32;
constexpr int kQThreads = 256;
static_assert(kQThreads == 4 * kWave, "four waves split the inner dimension of a tile product");
constexpr unsigned kQSpinLimit = 1u << 22;

struct QTileArgs {
  int mode;  // 0 = square root, 1 = Sylvester
  int m, p, mt, pt, ntiles;
  int64_t lda, ldb, ldx;
  const int* rb;  // row tile boundaries (mt + 1 entries)
  const int* cb;  // column tile boundaries (pt + 1 entries)
  int* flags;
  int* ticket;
  int* err;  // [0] wait timed out, [1] eigenvalue on or next to R<=0
};

template <typename T>
__device__ inline T qeps();
template <> __device__ inline float qeps<float>() { return 5.9604645e-08f; }
template <> __device__ inline double qeps<double>() { return 1.1102230246251565e-16; }

template <typename T>
__device__ inline T qload_c(const T* P, int64_t ld, int64_t i, int64_t j) {
  return __hip_atomic_load(const_cast<T*>(P) + i + j * ld, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void qstore_c(T* P, int64_t ld, int64_t i, int64_t j, T v) {
  __hip_atomic_store(P + i + j * ld, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void qtile_of(const QTileArgs& a, int tk, int& I, int& J) {
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

__device__ inline void qwait_tile(const QTileArgs& a, int I, int J) {
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
      if (spins > kQSpinLimit) {
        __hip_atomic_store(&a.err[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

// Tile (rows r0.., cols c0.., extent mr x mc, zero padded) to LDS dst[col][row].
template <typename T>
__device__ inline void qload_tile(T (*dst)[kQb + 1], const T* P, int64_t ld, int r0, int c0, int mr,
                                  int mc, bool coherent) {
  for (int x = threadIdx.x; x < kQb * kQb; x += blockDim.x) {
    const int i = x % kQb, j = x / kQb;
    T v = T(0);
    if (i < mr && j < mc)
      v = coherent ? qload_c(P, ld, r0 + i, c0 + j) : P[(r0 + i) + (int64_t)(c0 + j) * ld];
    dst[j][i] = v;
  }
}

// Partial products of C = A B (32 x 32 x 32) on MFMA: wave w sums the inner
// indices 8w .. 8w+7 into P[w][col][row] (C = P0 + P1 + P2 + P3).  P may
// overlay As and Bs: every wave reads its operands before the barrier.
template <typename T>
__device__ inline void qtile_product(const T (*As)[kQb + 1], const T (*Bs)[kQb + 1],
                                     T (*P)[kQb][kQb + 1], int wave, int lane) {
  using M = Mfma<T>;
  constexpr int NT = kQb / M::TM;
  constexpr int KW = kQb / 4;
  typename M::acc_t acc[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < M::NACC; ++r) acc[i][j][r] = T(0);
  const int fmn = M::frag_mn(lane);
#pragma unroll
  for (int k0 = 0; k0 < KW; k0 += M::TK) {
    const int fk = wave * KW + k0 + M::frag_k(lane);
    T av[NT], bv[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) av[i] = As[fk][i * M::TM + fmn];
#pragma unroll
    for (int j = 0; j < NT; ++j) bv[j] = Bs[j * M::TN + fmn][fk];
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

// A Y + Y B = C for a p x p block A and a q x q block B (p, q <= 2), all
// given as 2 x 2 arrays (entries beyond p or q ignored): the Kronecker form
// (I_q kron A + B^T kron I_p) vec Y = vec C, padded to order 4 with identity
// rows for the unused unknowns, by Gaussian elimination with partial
// pivoting (fully unrolled, so everything stays in registers).  Unknown
// r + 2 c holds Y(r, c).
template <typename T>
__device__ inline void small_sylvester(int p, int q, const T (&A)[2][2], const T (&B)[2][2],
                                       const T (&C)[4], T (&Y)[4]) {
  T M[4][5];
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const int r = row & 1, c = row >> 1;
    const bool live = r < p && c < q;
#pragma unroll
    for (int col = 0; col < 4; ++col) {
      const int k = col & 1, l = col >> 1;
      T v = T(0);
      if (live && k < p && l < q) {
        if (l == c) v += A[r][k];
        if (k == r) v += B[l][c];
      }
      if (!live) v = row == col ? T(1) : T(0);
      M[row][col] = v;
    }
    M[row][4] = live ? C[row] : T(0);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int piv = k;
    T best = fabs(M[k][k]);
#pragma unroll
    for (int i = k + 1; i < 4; ++i)
      if (fabs(M[i][k]) > best) { best = fabs(M[i][k]); piv = i; }
#pragma unroll
    for (int i = k + 1; i < 4; ++i)
      if (piv == i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) { const T tmp = M[k][j]; M[k][j] = M[i][j]; M[i][j] = tmp; }
      }
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const T f = M[i][k] / M[k][k];
#pragma unroll
      for (int j = k; j < 5; ++j) M[i][j] -= f * M[k][j];
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    T acc = M[i][4];
#pragma unroll
    for (int j = i + 1; j < 4; ++j) acc -= M[i][j] * Y[j];
    Y[i] = acc / M[i][i];
  }
}

// Diagonal block structure of the LDS tile X[col][row] of order mm: block
// starts in bs[0..nb], block index of every row in blk[].  A 2x2 block starts
// at i when X(i+1, i) != 0.  Thread 0 only; the caller synchronises.
template <typename T>
__device__ inline int tile_blocks(const T (*X)[kQb + 1], int mm, int* bs, int* blk) {
  int nb = 0;
  for (int i = 0; i < mm;) {
    bs[nb] = i;
    const int sz = (i + 1 < mm && X[i][i + 1] != T(0)) ? 2 : 1;
    for (int k = 0; k < sz; ++k) blk[i + k] = nb;
    ++nb;
    i += sz;
  }
  bs[nb] = mm;
  return nb;
}

template <typename T>
__global__ __launch_bounds__(kQThreads) void qtile_kernel(QTileArgs a, const T* A, const T* B, T* X) {
  __shared__ T ABs[4][kQb][kQb + 1];  // As = ABs[0], Bs = ABs[1]; products overlay all four
  T (*As)[kQb + 1] = ABs[0];
  T (*Bs)[kQb + 1] = ABs[1];
  __shared__ T Ys[kQb][kQb + 1];
  __shared__ T Cs[kQb][kQb + 1];
  __shared__ int rbs[kQb + 1], cbs[kQb + 1], rblk[kQb], cblk[kQb];
  __shared__ int sh_nrb, sh_ncb, sh_tk;
  const int t = threadIdx.x;
  const int ti = t % kQb, tj0 = t / kQb;  // owned entries (ti, tj0 + 8 q)
  const int wave = __builtin_amdgcn_readfirstlane(t / kWave);
  {
    if (wave == 0) {
      const int old = atomicAdd(a.ticket, t == 0 ? 1 : 0);
      sh_tk = __builtin_amdgcn_readfirstlane(old);
    }
    __syncthreads();
  }
  const int tk = __builtin_amdgcn_readfirstlane(sh_tk);
  if (tk >= a.ntiles) return;
  int I, J;
  qtile_of(a, tk, I, J);
  const int r0 = a.rb[I], mi = a.rb[I + 1] - r0;
  const int c0 = a.cb[J], mj = a.cb[J + 1] - c0;
  T acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = tj0 + 8 * q;
    acc[q] = (ti < mi && j < mj)
                 ? (a.mode == 0 ? A[(r0 + ti) + (int64_t)(c0 + j) * a.lda]
                                : X[(r0 + ti) + (int64_t)(c0 + j) * a.ldx])
                 : T(0);
  }
  auto subtract = [&]() {
    __syncthreads();
    qtile_product<T>(As, Bs, ABs, wave, t % kWave);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = tj0 + 8 * q;
      acc[q] -= (ABs[0][j][ti] + ABs[1][j][ti]) + (ABs[2][j][ti] + ABs[3][j][ti]);
    }
    __syncthreads();
  };
  if (a.mode == 0 && I == J) {
    // diagonal tile: T_II into Ys, root into As
#pragma unroll
    for (int q = 0; q < 4; ++q) Ys[tj0 + 8 * q][ti] = acc[q];
    for (int x = t; x < kQb * kQb; x += blockDim.x) As[x / kQb][x % kQb] = T(0);
    __syncthreads();
    if (t == 0) sh_nrb = tile_blocks<T>(Ys, mi, rbs, rblk);
    __syncthreads();
    const int nb = sh_nrb;
    if (t < nb) {
      const int i0 = rbs[t], sz = rbs[t + 1] - i0;
      const T eps = qeps<T>();
      if (sz == 1) {
        const T d = Ys[i0][i0];
        if (!(d > T(0))) atomicOr(&a.err[1], 1);
        As[i0][i0] = sqrt(fmax(d, T(0)));
      } else {
        const T b11 = Ys[i0][i0], b21 = Ys[i0][i0 + 1], b12 = Ys[i0 + 1][i0], b22 = Ys[i0 + 1][i0 + 1];
        const T det = b11 * b22 - b12 * b21;
        const T dd = sqrt(fmax(det, T(0)));
        const T t2 = b11 + b22 + T(2) * dd;
        // a complex pair on or within a few ulps of the negative real axis
        const T re = T(0.5) * (b11 + b22);
        const T im2 = det - re * re;
        if (!(det > T(0)) || !(t2 > T(0)) ||
            (re < T(0) && im2 <= T(256) * eps * eps * re * re))
          atomicOr(&a.err[1], 1);
        const T tt = sqrt(fmax(t2, T(0)));
        As[i0][i0] = (b11 + dd) / tt;
        As[i0][i0 + 1] = b21 / tt;
        As[i0 + 1][i0] = b12 / tt;
        As[i0 + 1][i0 + 1] = (b22 + dd) / tt;
      }
    }
    __syncthreads();
    for (int d = 1; d < nb; ++d) {
      if (t < nb - d) {
        const int bi = t, bj = t + d;
        const int i0 = rbs[bi], p = rbs[bi + 1] - i0, j0 = rbs[bj], q = rbs[bj + 1] - j0;
        const int klo = rbs[bi + 1];
        T Cv[4], Yv[4], Am[2][2], Bm[2][2];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = u & 1, c = u >> 1;
          T s = T(0);
          if (r < p && c < q) {
            s = Ys[j0 + c][i0 + r];
            for (int k = klo; k < j0; ++k) s -= As[k][i0 + r] * As[j0 + c][k];
          }
          Cv[u] = s;
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            Am[r][c] = (r < p && c < p) ? As[i0 + c][i0 + r] : T(0);
            Bm[r][c] = (r < q && c < q) ? As[j0 + c][j0 + r] : T(0);
          }
        small_sylvester<T>(p, q, Am, Bm, Cv, Yv);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = u & 1, c = u >> 1;
          if (r < p && c < q) As[j0 + c][i0 + r] = Yv[u];
        }
      }
      __syncthreads();
    }
    for (int x = t; x < kQb * kQb; x += blockDim.x) {
      const int i = x % kQb, j = x / kQb;
      if (i < mi && j < mj) qstore_c(X, a.ldx, r0 + i, c0 + j, As[j][i]);
    }
  } else {
    if (a.mode == 0) {
      // U_IK U_KJ is ready once tiles (I, K) and (K, J) are: K from the
      // middle outwards
      const int klo = I + 1, khi = J - 1, cnt = khi - klo + 1, mid = (I + J) / 2;
      for (int q = 0, done = 0; done < cnt; ++q) {
        const int K = mid + ((q & 1) ? (q + 1) / 2 : -(q / 2));
        if (K < klo || K > khi) continue;
        ++done;
        qwait_tile(a, I, K);
        qwait_tile(a, K, J);
        const int k0 = a.rb[K], mk = a.rb[K + 1] - k0;
        qload_tile(As, X, a.ldx, r0, k0, mi, mk, true);
        qload_tile(Bs, X, a.ldx, k0, c0, mk, mj, true);
        subtract();
      }
      qwait_tile(a, I, I);
      qwait_tile(a, J, J);
      qload_tile(As, X, a.ldx, r0, r0, mi, mi, true);
      qload_tile(Bs, X, a.ldx, c0, c0, mj, mj, true);
    } else {
      // column terms S_IK Y_KJ (K > I) and row terms Y_IK S2_KJ (K < J),
      // taken merged in order of readiness
      int kc = a.mt - 1, kr = 0;
      while (kc > I || kr < J) {
        const int dc = kc > I ? a.mt - 1 - kc + J : 1 << 30;
        const int dr = kr < J ? a.mt - 1 - I + kr : 1 << 30;
        if (dc <= dr) {
          const int K = kc--;
          qwait_tile(a, K, J);
          const int k0 = a.rb[K], mk = a.rb[K + 1] - k0;
          qload_tile(As, A, a.lda, r0, k0, mi, mk, false);
          qload_tile(Bs, X, a.ldx, k0, c0, mk, mj, true);
        } else {
          const int K = kr++;
          qwait_tile(a, I, K);
          const int k0 = a.cb[K], mk = a.cb[K + 1] - k0;
          qload_tile(As, X, a.ldx, r0, k0, mi, mk, true);
          qload_tile(Bs, B, a.ldb, k0, c0, mk, mj, false);
        }
        subtract();
      }
      qload_tile(As, A, a.lda, r0, r0, mi, mi, false);
      qload_tile(Bs, B, a.ldb, c0, c0, mj, mj, false);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Cs[tj0 + 8 * q][ti] = acc[q];
    __syncthreads();
    if (t == 0) sh_nrb = tile_blocks<T>(As, mi, rbs, rblk);
    if (t == kWave) sh_ncb = tile_blocks<T>(Bs, mj, cbs, cblk);
    __syncthreads();
    const int nrb = sh_nrb, ncb = sh_ncb;
    // S_II Y + Y S2_JJ = C by block anti-diagonals e = (nrb - 1 - ib) + jb
    const int ne = nrb + ncb - 1;
    for (int e = 0; e < ne; ++e) {
      const int jlo = max(0, e - (nrb - 1)), jhi = min(ncb - 1, e);
      if (t <= jhi - jlo) {
        const int jb = jlo + t, ib = nrb - 1 - e + jb;
        const int i0 = rbs[ib], p = rbs[ib + 1] - i0, j0 = cbs[jb], q = cbs[jb + 1] - j0;
        T Cv[4], Yv[4], Am[2][2], Bm[2][2];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = u & 1, c = u >> 1;
          Cv[u] = (r < p && c < q) ? Cs[j0 + c][i0 + r] : T(0);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            Am[r][c] = (r < p && c < p) ? As[i0 + c][i0 + r] : T(0);
            Bm[r][c] = (r < q && c < q) ? Bs[j0 + c][j0 + r] : T(0);
          }
        small_sylvester<T>(p, q, Am, Bm, Cv, Yv);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = u & 1, c = u >> 1;
          if (r < p && c < q) Ys[j0 + c][i0 + r] = Yv[u];
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = tj0 + 8 * q;
        if (ti < mi && j < mj) {
          const int ib = rblk[ti], jb = cblk[j];
          if ((nrb - 1 - ib) + jb > e) {
            T c = Cs[j][ti];
            const int kb = nrb - 1 - e + jb;  // block (kb, jb) finished on e
            if (kb > ib && kb < nrb)
              for (int k = rbs[kb]; k < rbs[kb + 1]; ++k) c -= As[k][ti] * Ys[j][k];
            const int lb = e - (nrb - 1 - ib);  // block (ib, lb) finished on e
            if (lb >= 0 && lb < jb)
              for (int l = cbs[lb]; l < cbs[lb + 1]; ++l) c -= Ys[l][ti] * Bs[j][l];
            Cs[j][ti] = c;
          }
        }
      }
      __syncthreads();
    }
    for (int x = t; x < kQb * kQb; x += blockDim.x) {
      const int i = x % kQb, j = x / kQb;
      if (i < mi && j < mj) qstore_c(X, a.ldx, r0 + i, c0 + j, Ys[j][i]);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (wave == 0)
    __hip_atomic_store(&a.flags[I * a.pt + J], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
void launch_qtiles(hipStream_t st, QTileArgs a, const T* A, const T* B, T* X, TrsylvWork& w) {
  const int nflags = a.mt * a.pt;
  int* buf = w.flags.ensure<int>(nflags + 64);
  a.flags = buf;
  a.ticket = buf + nflags;
  const bool fresh = w.ticket.p == nullptr;
  a.err = w.ticket.ensure<int>(4);
  if (fresh) MSQRT_HIP(hipMemsetAsync(a.err, 0, sizeof(int) * 4, st));
  MSQRT_HIP(hipMemsetAsync(buf, 0, sizeof(int) * (nflags + 64), st));
  if (a.ntiles <= 0) return;
  hipLaunchKernelGGL(qtile_kernel<T>, dim3(a.ntiles), dim3(kQThreads), 0, st, a, A, B, X);
  MSQRT_LAUNCH_CHECK();
}

}  // namespace

std::vector<int> quasi_partition(int n, const unsigned char* sub) {
  std::vector<int> b{0};
  while (b.back() < n) {
    int e = std::min(b.back() + kQb, n);
    if (e < n && sub[e - 1]) --e;  // t(e, e-1) != 0: keep rows e-1, e together
    b.push_back(e);
  }
  return b;
}

template <typename T>
void trsqrt_quasi(hipStream_t st, int n, const T* Tm, T* U, const int* part, int nt,
                  TrsylvWork& w) {
  if (n <= 0) return;
  MSQRT_HIP(hipMemsetAsync(U, 0, sizeof(T) * (size_t)n * n, st));
  QTileArgs a{};
  a.mode = 0;
  a.m = a.p = n;
  a.mt = a.pt = nt;
  a.ntiles = nt * (nt + 1) / 2;
  a.lda = a.ldb = a.ldx = n;
  a.rb = a.cb = part;
  launch_qtiles<T>(st, a, Tm, Tm, U, w);
}

template <typename T>
void trsyl_quasi(hipStream_t st, int m, int p, const T* S, int64_t lds, const int* rpart, int mt,
                 const T* S2, int64_t lds2, const int* cpart, int pt, T* C, int64_t ldc,
                 TrsylvWork& w) {
  if (m <= 0 || p <= 0) return;
  QTileArgs a{};
  a.mode = 1;
  a.m = m;
  a.p = p;
  a.mt = mt;
  a.pt = pt;
  a.ntiles = mt * pt;
  a.lda = lds;
  a.ldb = lds2;
  a.ldx = ldc;
  a.rb = rpart;
  a.cb = cpart;
  launch_qtiles<T>(st, a, S, S2, C, w);
}

template void trsqrt_quasi<float>(hipStream_t, int, const float*, float*, const int*, int,
                                  TrsylvWork&);
template void trsqrt_quasi<double>(hipStream_t, int, const double*, double*, const int*, int,
                                   TrsylvWork&);
template void trsyl_quasi<float>(hipStream_t, int, int, const float*, int64_t, const int*, int,
                                 const float*, int64_t, const int*, int, float*, int64_t,
                                 TrsylvWork&);
template void trsyl_quasi<double>(hipStream_t, int, int, const double*, int64_t, const int*, int,
                                  const double*, int64_t, const int*, int, double*, int64_t,
                                  TrsylvWork&);

}  // namespace msqrt
