// Two-stage tridiagonalisation of a symmetric matrix (the first step of the
// spectral decomposition used by Alg. 3) and the back-transformation of the
// tridiagonal eigenvectors through both stages.
//
// Stage 1 (dense -> band of half-bandwidth B).  Panel p holds columns
// p..p+w-1; the rows below the band start at r0 = p + B.  The panel block is
// factored P = A(r0:, p:p+w) = (I - V T V^T) [R; 0] by one workgroup that
// keeps it in registers (one reduction of all pending dot products per
// column), and with X = A22 V T and W = X - 1/2 V (T^T V^T X) the trailing
// matrix becomes A22 - V W^T - W V^T (MFMA GEMMs; the last one computes the
// lower tiles and mirrors them, so A stays in full symmetric storage).
//
// Stage 2 (band -> tridiagonal) by bulge chasing.  Sweep s clears column s.
// Its step k works on the rows R_k = [s+1+kB, s+1+(k+1)B): for k >= 1 the
// sweep's previous reflector is applied from the right to the block
// A(R_k, R_{k-1}) (creating the bulge), a new reflector maps the block's first
// column (for k = 0: column s itself) to beta e_1 and is applied from the left
// to the rest of the block and from both sides to A(R_k, R_k).  A step reads
// and writes rows R_k only, and in the sequential order the only later step
// of the previous sweep that touches them is its step k+1; so step k of sweep
// s may start once sweep s-1 has finished step k+1.  One wavefront chases one
// sweep; sweeps are handed out by an atomic ticket in increasing order, so a
// sweep waited for is always held by a running wavefront (no deadlock for any
// residency), and band blocks are exchanged with agent-scope atomic loads and
// stores (coherent across the XCDs' L2 caches without cache flushes).
//
// Band storage: AB[d + 2B c] = A(c + d, c), 0 <= d < 2B.  The off-diagonal
// block A(R_k, R_{k-1}) reaches distance 2B - 1, so the bulge fits.
//
// Back-transformation: Z <- Q1 Q2 Z.  Q2's reflectors of one sweep act on
// disjoint rows, so a workgroup applies a whole sweep to its columns of Z (held
// in LDS) at once, sweeps from the last to the first; Q1 is applied as blocked
// compact-WY products (the same code as the one-stage reduction, with the
// reflectors' unit entries B rows below the diagonal).
#include <algorithm>

#include "kernels.hpp"
#include "profile.hpp"
#include "tridiag.hpp"

namespace msqrt {

namespace {

constexpr int kPT = 1024;  // panel workgroup
constexpr int kRPT = 4;    // panel rows per thread: panels of up to 4096 rows

template <typename T>
__device__ inline void cstore(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline T cload(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Householder scalars for x = (alpha, x_2..): H^T x = beta e_1 with
// H = I - tau v v^T, v = (1, x_2.. * scal).  sig = ||x_2..||^2.
template <typename T>
__device__ inline void house_scalars(T alpha, T sig, T& beta, T& tau, T& scal) {
  if (sig == T(0)) {
    beta = alpha;
    tau = T(0);
    scal = T(0);
  } else {
    beta = -copysign(sqrt(alpha * alpha + sig), alpha);
    tau = (beta - alpha) / beta;
    scal = T(1) / (alpha - beta);
  }
}

// ---------------------------------------------------------------- stage 1

template <typename T, int B>
__global__ __launch_bounds__(kPT) void sb_panel_kernel(int n, int p, const T* __restrict__ A,
                                                       T* __restrict__ AB, T* __restrict__ V1,
                                                       T* __restrict__ tau1, T* __restrict__ VW,
                                                       T* __restrict__ WV, T* __restrict__ VT,
                                                       T* __restrict__ Tg) {
  constexpr int L2B = 2 * B, NW = kPT / kWave;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int w = min(B, n - p), r0 = p + B, m = n - r0;
  __shared__ T nrm[NW];
  __shared__ T red[NW][B];
  __shared__ T fin[B];
  __shared__ T Ts[B][B + 1];
  __shared__ T Rs[B][B + 1];
  __shared__ T Rd[B];
  __shared__ T sh_alpha;
  for (int x = tid; x < B * (B + 1); x += kPT) Ts[x / (B + 1)][x % (B + 1)] = T(0);
  // band entries of the diagonal block (final: earlier updates are complete)
  for (int x = tid; x < w * L2B; x += kPT) {
    const int j = x / L2B, dd = x % L2B, c = p + j, r = c + dd;
    if (r < r0 || r >= n) AB[dd + (int64_t)c * L2B] = (r < n) ? A[r + (int64_t)c * n] : T(0);
  }
  if (m <= 0) {
    for (int j = tid; j < w; j += kPT) tau1[p + j] = T(0);
    return;
  }
  T P[kRPT][B];
#pragma unroll
  for (int q = 0; q < kRPT; ++q) {
    const int i = tid + q * kPT;
#pragma unroll
    for (int j = 0; j < B; ++j) P[q][j] = (i < m && j < w) ? A[r0 + i + (int64_t)(p + j) * n] : T(0);
  }
  __syncthreads();
  const int kq = min(w, m);
  // The column loop has a fixed trip count so that it unrolls and every
  // P[q][j] is a register.
#pragma clang loop unroll(full)
  for (int j = 0; j < B; ++j) {
    if (j < kq) {
      // ---- ||P(j+1:, j)||^2 and alpha = P(j, j)
      T part = T(0);
#pragma unroll
      for (int q = 0; q < kRPT; ++q) {
        const int i = tid + q * kPT;
        if (i > j && i < m) part += P[q][j] * P[q][j];
      }
      if (tid == j) sh_alpha = P[0][j];
      part = wave_sum(part);
      if (lane == 0) nrm[wave] = part;
      __syncthreads();
      T sig = T(0);
#pragma unroll
      for (int x = 0; x < NW; ++x) sig += nrm[x];
      T beta, tau, scal;
      house_scalars(sh_alpha, sig, beta, tau, scal);
      T vq[kRPT];
#pragma unroll
      for (int q = 0; q < kRPT; ++q) {
        const int i = tid + q * kPT;
        vq[q] = (i == j) ? T(1) : ((i > j && i < m) ? P[q][j] * scal : T(0));
        if (i >= j) P[q][j] = vq[q];
      }
      if (tid == 0) Rd[j] = beta;
      // ---- one reduction for every dot product this column needs: slot s
      // is column c = s (s < j: Gram entry V(:, c)^T v for T) or c = s + 1
      // (s >= j: v^T P(:, c) for the update).  Wave partials go to LDS; one
      // thread per slot sums them.
#pragma unroll
      for (int s = 0; s < B - 1; ++s) {
        const int c = s < j ? s : s + 1;
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < kRPT; ++q) acc += vq[q] * P[q][c];
        acc = wave_sum(acc);
        if (lane == 0) red[wave][s] = acc;
      }
      __syncthreads();
      if (tid < B - 1) {
        T t = T(0);
#pragma unroll
        for (int x = 0; x < NW; ++x) t += red[x][tid];
        fin[tid] = t;
      }
      __syncthreads();
      // ---- update the remaining panel columns
#pragma unroll
      for (int s = j; s < B - 1; ++s) {
        const T f = tau * fin[s];
#pragma unroll
        for (int q = 0; q < kRPT; ++q) P[q][s + 1] -= f * vq[q];
      }
      // ---- column j of T: T(0:j, j) = -tau T(0:j, 0:j) (V(:, 0:j)^T v)
      if (tid < j) {
        T acc = T(0);
        for (int c = tid; c < j; ++c) acc += Ts[tid][c] * fin[c];
        Ts[tid][j] = -tau * acc;
      }
      if (tid == j) Ts[j][j] = tau;
    }
  }
  // R above the diagonal, from the rows' owners
  if (tid < min(B, m)) {
#pragma unroll
    for (int j = 0; j < B; ++j) Rs[tid][j] = P[0][j];
  }
  __syncthreads();
  // ---- band entries on and below row r0: R (upper trapezoidal), zeros below
  for (int x = tid; x < w * L2B; x += kPT) {
    const int j = x / L2B, dd = x % L2B, c = p + j, r = c + dd;
    if (r >= r0 && r < n) {
      const int i = r - r0;
      // i < j: R(i, j) (also past the last reflector when m < w); i == j
      // (then j < kq): beta_j; i > j: cleared.
      AB[dd + (int64_t)c * L2B] = i < j ? Rs[i][j] : (i == j ? Rd[j] : T(0));
    }
  }
  // ---- reflectors: explicit columns of V1, [V W] / [W V] operands, V T
#pragma unroll
  for (int q = 0; q < kRPT; ++q) {
    const int i = tid + q * kPT;
    if (i >= m) continue;
    const int64_t r = r0 + i;
    T vrow[B];
#pragma unroll
    for (int a = 0; a < B; ++a) vrow[a] = (a < kq && i >= a) ? (i == a ? T(1) : P[q][a]) : T(0);
#pragma unroll
    for (int a = 0; a < B; ++a) {
      if (a >= w) break;
      VW[r + (int64_t)a * n] = vrow[a];
      T acc = T(0);
#pragma unroll
      for (int b = 0; b <= a; ++b) acc += vrow[b] * Ts[b][a];
      VT[r + (int64_t)a * n] = acc;
    }
  }
  for (int x = tid; x < B * B; x += kPT) Tg[x] = Ts[x % B][x / B];
  for (int j = tid; j < w; j += kPT) tau1[p + j] = Ts[j][j];
}

// out(i, c) = sum over q of P_q(i, c) (P_q m x w, ld m, stride m w), in q order.
template <typename T>
__global__ void sum_cols(int m, int w, int splits, const T* __restrict__ P, T* __restrict__ out,
                         int64_t ldo) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (int64_t)m * w) return;
  const int i = (int)(x % m), c = (int)(x / m);
  T s = T(0);
  for (int q = 0; q < splits; ++q) s += P[(int64_t)q * m * w + x];
  out[i + c * ldo] = s;
}

// W = X - 1/2 V M with M = T^T Y, Y = sum of the split-K partials of V^T X.
// One thread per row; every workgroup forms M itself (fixed summation order).
// It also copies V into [W V] and into the explicit reflector columns of V1
// (rows on and below each unit entry; V1 is zero elsewhere).
template <typename T, int B>
__global__ __launch_bounds__(256) void sb_w_kernel(int n, int p, int r0, int m, int w,
                                                   int splits, const T* __restrict__ Yp,
                                                   const T* __restrict__ Tg,
                                                   const T* __restrict__ X, T* __restrict__ VW,
                                                   T* __restrict__ WV, T* __restrict__ V1) {
  __shared__ T Ys[B][B + 1], Ms[B][B + 1];
  const int tid = threadIdx.x;
  for (int x = tid; x < B * B; x += blockDim.x) {
    const int a = x % B, c = x / B;
    T s = T(0);
    if (a < w && c < w)
      for (int g = 0; g < splits; ++g) s += Yp[(int64_t)g * w * w + a + c * w];
    Ys[a][c] = s;
  }
  __syncthreads();
  for (int x = tid; x < B * B; x += blockDim.x) {
    const int a = x % B, c = x / B;
    T s = T(0);
    for (int b = 0; b <= a; ++b) s += Tg[b + a * B] * Ys[b][c];
    Ms[a][c] = s;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + tid;
  if (i >= m) return;
  const int64_t r = r0 + i;
  T v[B];
#pragma unroll
  for (int a = 0; a < B; ++a) v[a] = a < w ? VW[r + (int64_t)a * n] : T(0);
#pragma unroll
  for (int a = 0; a < B; ++a) {
    if (a >= w) break;
    WV[r + (int64_t)(w + a) * n] = v[a];
    if (i >= a) V1[r + (int64_t)(p + a) * n] = v[a];
  }
#pragma unroll
  for (int c = 0; c < B; ++c) {
    if (c >= w) break;
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < B; ++a) acc += v[a] * Ms[a][c];
    const T wv = X[r + (int64_t)c * n] - T(0.5) * acc;
    VW[r + (int64_t)(w + c) * n] = wv;
    WV[r + (int64_t)c * n] = wv;
  }
}

// ---------------------------------------------------------------- stage 2

// Wavefront layout of a B x B block: lane l holds row l % B and the NQ
// columns (l / B) * NQ + q.
template <typename T, int B>
__device__ inline T rowsum(T v) {  // over the lanes holding the same row
#pragma unroll
  for (int off = B; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
template <typename T, int B>
__device__ inline T colsum(T v) {  // over the B rows of a lane group
#pragma unroll
  for (int off = 1; off < B; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T, int B>
__global__ __launch_bounds__(kWave) void sb2st_kernel(int n, int nsw, int kmax, T* AB, T* V2,
                                                      T* tau2, int* prog, int* ctl) {
  constexpr int L2B = 2 * B, NQ = B * B / kWave;
  const int lane = threadIdx.x;
  const int ri = lane % B, jb = (lane / B) * NQ;
  for (;;) {
    int s = 0;
    if (lane == 0) s = atomicAdd(&ctl[0], 1);
    s = __builtin_amdgcn_readfirstlane(s);
    if (s >= nsw) break;
    const int K = (n - 1 - s + B - 1) / B;
    const int Kprev = s > 0 ? (n - s + B - 1) / B : 0;
    T v0c[NQ], t0 = T(0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) v0c[q] = T(0);
    for (int k = 0; k < K; ++k) {
      if (s > 0) {
        const int need = min(k + 2, Kprev);
        unsigned spins = 0;
        int bad = 0;
        for (;;) {
          const int pv = __builtin_amdgcn_readfirstlane(cload(&prog[s - 1]));
          if (pv >= need) break;
          if (__builtin_amdgcn_readfirstlane(cload(&ctl[1])) != 0) { bad = 1; break; }
          if (++spins > (1u << 22)) {
            if (lane == 0) cstore(&ctl[1], 1);
            bad = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (bad) return;
      }
      const int rho = s + 1 + k * B, L = min(B, n - rho);
      T bm[NQ], dm[NQ], x = T(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) bm[q] = T(0);
      if (k == 0) {
        x = (ri < L) ? cload(&AB[1 + ri + (int64_t)s * L2B]) : T(0);
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int j = jb + q;
          bm[q] = (ri < L) ? cload(&AB[(B + ri - j) + (int64_t)(rho - B + j) * L2B]) : T(0);
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int j = jb + q;
        dm[q] = (ri < L && j < L) ? cload(&AB[abs(ri - j) + (int64_t)(rho + min(ri, j)) * L2B])
                                  : T(0);
      }
      if (k > 0) {
        // bulge: B <- B H_prev
        T y = T(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) y += bm[q] * v0c[q];
        y = t0 * rowsum<T, B>(y);
#pragma unroll
        for (int q = 0; q < NQ; ++q) bm[q] -= y * v0c[q];
        x = __shfl(bm[0], ri, kWave);  // column 0 sits in the first lane group
      }
      const T alpha = __shfl(x, 0, kWave);
      const T sig = colsum<T, B>(ri >= 1 ? x * x : T(0));
      T beta, tau, scal;
      house_scalars(alpha, sig, beta, tau, scal);
      const T vr = (ri == 0) ? T(1) : x * scal;
      T vc[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) vc[q] = __shfl(vr, jb + q, kWave);
      if (k > 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const T t = colsum<T, B>(vr * bm[q]);
          bm[q] -= tau * t * vr;
        }
        if (jb == 0) bm[0] = (ri == 0) ? beta : T(0);
      }
      // D <- H D H
      T pr = T(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) pr += dm[q] * vc[q];
      pr = tau * rowsum<T, B>(pr);
      const T kc = T(0.5) * tau * colsum<T, B>(pr * vr);
      const T wr = pr - kc * vr;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T wcq = __shfl(wr, jb + q, kWave);
        dm[q] -= vr * wcq + wr * vc[q];
      }
      if (k == 0) {
        if (lane < L) cstore(&AB[1 + lane + (int64_t)s * L2B], lane == 0 ? beta : T(0));
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int j = jb + q;
          if (ri < L) cstore(&AB[(B + ri - j) + (int64_t)(rho - B + j) * L2B], bm[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int j = jb + q;
        if (ri < L && j <= ri) cstore(&AB[(ri - j) + (int64_t)(rho + j) * L2B], dm[q]);
      }
      const int64_t slot = (int64_t)s * kmax + k;
      if (lane < B) V2[slot * B + lane] = vr;
      if (lane == 0) tau2[slot] = tau;
      __builtin_amdgcn_s_waitcnt(0);
      if (lane == 0) cstore(&prog[s], k + 1);
#pragma unroll
      for (int q = 0; q < NQ; ++q) v0c[q] = vc[q];
      t0 = tau;
    }
  }
}

template <typename T, int B>
__global__ void band_diag_kernel(int n, const T* AB, T* d, T* e) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  d[c] = AB[(int64_t)c * 2 * B];
  if (c + 1 < n) e[c] = AB[1 + (int64_t)c * 2 * B];
}

// Z(:, c0:c0+nc) <- Q2 Z(:, c0:c0+nc), the columns held in LDS.  One sweep
// per round, its reflectors in parallel; the reflectors of the next sweep
// (contiguous in V2) are loaded into registers while the current sweep is
// applied and parked in the other LDS buffer.  LDS layouts are padded so that
// the reflectors of one round, B rows apart, fall on different banks: row r
// of Z at r nc + r / B, reflector k at k (B + 1).
template <typename T, int B>
__global__ __launch_bounds__(kPT) void apply_q2_kernel(int n, int nsw, int kmax, int nc,
                                                       const T* __restrict__ V2,
                                                       const T* __restrict__ tau2, T* Z) {
  constexpr int kPre = 8;  // reflector values prefetched per thread (kmax B <= kPre kPT)
  extern __shared__ unsigned char smem_raw[];
  T* zs = reinterpret_cast<T*>(smem_raw);
  const int zlen = n * nc + n / B + 1;
  const int vpad = kmax * (B + 1);
  T* vs = zs + zlen;           // [2][kmax (B + 1)]
  T* ts = vs + 2 * vpad;       // [2][kmax]
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * nc, ncl = min(nc, n - c0);
  const int vlen = kmax * B;
  auto zi = [&](int r, int c) { return r * nc + r / B + c; };
  for (int x = tid; x < n * ncl; x += kPT) {
    const int c = x / n, r = x % n;
    zs[zi(r, c)] = Z[r + (int64_t)(c0 + c) * n];
  }
  if (nsw > 0) {
    const int64_t base = (int64_t)(nsw - 1) * kmax;
    T* vb = vs + ((nsw - 1) & 1) * vpad;
    for (int x = tid; x < vlen; x += kPT) vb[(x / B) * (B + 1) + x % B] = V2[base * B + x];
    for (int x = tid; x < kmax; x += kPT) ts[((nsw - 1) & 1) * kmax + x] = tau2[base + x];
  }
  __syncthreads();
  for (int s = nsw - 1; s >= 0; --s) {
    T pv[kPre], pt = T(0);
    if (s > 0) {
      const int64_t base = (int64_t)(s - 1) * kmax;
#pragma unroll
      for (int e = 0; e < kPre; ++e) {
        const int x = tid + e * kPT;
        pv[e] = x < vlen ? V2[base * B + x] : T(0);
      }
      if (tid < kmax) pt = tau2[base + tid];
    }
    const T* v = vs + (s & 1) * vpad;
    const T* tt = ts + (s & 1) * kmax;
    const int K = (n - 1 - s + B - 1) / B;
    for (int x = tid; x < K * ncl; x += kPT) {
      const int k = x / ncl, c = x % ncl;
      const int rho = s + 1 + k * B, L = min(B, n - rho);
      const T tau = tt[k];
      if (tau == T(0)) continue;
      const T* vk = v + k * (B + 1);
      T dot = T(0);
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i < L) dot += vk[i] * zs[zi(rho + i, c)];
      dot *= tau;
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i < L) zs[zi(rho + i, c)] -= vk[i] * dot;
    }
    if (s > 0) {
      T* vn = vs + ((s - 1) & 1) * vpad;
#pragma unroll
      for (int e = 0; e < kPre; ++e) {
        const int x = tid + e * kPT;
        if (x < vlen) vn[(x / B) * (B + 1) + x % B] = pv[e];
      }
      if (tid < kmax) ts[((s - 1) & 1) * kmax + tid] = pt;
    }
    __syncthreads();
  }
  for (int x = tid; x < n * ncl; x += kPT) {
    const int c = x / n, r = x % n;
    Z[r + (int64_t)(c0 + c) * n] = zs[zi(r, c)];
  }
}

template <typename T>
void gemm_t(hipStream_t st, bool ta, bool tb, int M, int N, int K, const T* A, int64_t lda,
            const T* Bm, int64_t ldb, T* C, int64_t ldc, T alpha, T beta, bool tri) {
  if (std::is_same<T, float>::value)
    gemm_store_f32(st, ta, tb, M, N, K, (const float*)A, lda, 0, (const float*)Bm, ldb, 0,
                   (float*)C, ldc, 0, (float)alpha, (float)beta, 1, tri);
  else
    gemm_store_f64(st, ta, tb, M, N, K, (const double*)A, lda, 0, (const double*)Bm, ldb, 0,
                   (double*)C, ldc, 0, (double)alpha, (double)beta, 1, tri);
}

}  // namespace

int sy2tr_max_n() { return kPT * kRPT + 8; }

template <typename T>
void sy2tr(hipStream_t st, int n, T* A, T* d, T* e, Sy2trWork& w) {
  constexpr int B = BandWidth<T>::B;
  if (n <= 0) return;
  if (n - B > kPT * kRPT)
    throw Error{MSQRT_ERR_UNSUPPORTED, "two-stage tridiagonal reduction supports n <= 4096 + B"};
  T* AB = w.AB.ensure<T>((int64_t)2 * B * n);
  T* V1 = w.V1.ensure<T>((int64_t)n * n);
  T* tau1 = w.tau1.ensure<T>((int64_t)n + 8);
  T* VW = w.VW.ensure<T>((int64_t)n * 2 * B);
  T* WV = w.WV.ensure<T>((int64_t)n * 2 * B);
  T* VT = w.VT.ensure<T>((int64_t)n * B);
  T* X = w.X.ensure<T>((int64_t)n * B);
  constexpr int kSplitsMax = 32;
  T* Yp = w.Yp.ensure<T>((int64_t)kSplitsMax * B * B);
  T* Tg = w.Tg.ensure<T>((int64_t)B * B);
  constexpr int kXSplits = 16;
  T* Xp = w.Xp.ensure<T>((int64_t)kXSplits * n * B);
  MSQRT_HIP(hipMemsetAsync(V1, 0, sizeof(T) * (size_t)n * n, st));
  const int tok = prof_begin(st);
  for (int p = 0; p < n; p += B) {
    const int wd = std::min(B, n - p), r0 = p + B, m = n - r0;
    hipLaunchKernelGGL((sb_panel_kernel<T, B>), dim3(1), dim3(kPT), 0, st, n, p, (const T*)A, AB,
                       V1, tau1, VW, WV, VT, Tg);
    MSQRT_LAUNCH_CHECK();
    if (m <= 0) continue;
    T* A22 = A + r0 + (int64_t)r0 * n;
    // X = A22 (V T): split-K partials (the output is only wd columns wide,
    // so the K range is what gives the launch its parallelism), then a
    // fixed-order sum.
    {
      const int xs = (int)std::min<int64_t>(kXSplits, std::max<int64_t>(1, ceil_div(m, 256)));
      const int xchunk = (int)ceil_div(m, xs);
      const int xsp = (int)ceil_div(m, xchunk);
      const int xlast = m - (xsp - 1) * xchunk;
      gemm_store_splitk<T>(st, false, false, m, wd, xchunk, xlast, A22, n, (int64_t)xchunk * n,
                           VT + r0, n, xchunk, Xp, m, (int64_t)m * wd, xsp);
      const int cnt = m * wd;
      hipLaunchKernelGGL((sum_cols<T>), dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, m, wd,
                         xsp, (const T*)Xp, X + r0, n);
      MSQRT_LAUNCH_CHECK();
    }
    // Y = V^T X (split-K partials)
    int splits = (int)std::min<int64_t>(kSplitsMax, std::max<int64_t>(1, ceil_div(m, 128)));
    const int chunk = (int)ceil_div(m, splits);
    splits = (int)ceil_div(m, chunk);
    const int klast = m - (splits - 1) * chunk;
    gemm_store_splitk<T>(st, true, false, wd, wd, chunk, klast, VW + r0, n, chunk, X + r0, n,
                         chunk, Yp, wd, (int64_t)wd * wd, splits);
    hipLaunchKernelGGL((sb_w_kernel<T, B>), dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, n,
                       p, r0, m, wd, splits, (const T*)Yp, (const T*)Tg, (const T*)X, VW, WV, V1);
    MSQRT_LAUNCH_CHECK();
    // A22 -= [V W] [W V]^T
    gemm_t<T>(st, false, true, m, m, 2 * wd, VW + r0, n, WV + r0, n, A22, n, T(-1), T(1), true);
  }
  if (tok >= 0) {
    // algorithmic traffic: per panel one read of A22 for X, one read and
    // one write of it for the update
    double bytes = 0.0, flops = 0.0;
    for (int p = 0; p < n; p += B) {
      const double m = (double)(n - p - B);
      if (m > 0) {
        bytes += 3.0 * m * m * sizeof(T);
        flops += 2.0 * m * m * B + 4.0 * m * m * B;
      }
    }
    prof_end(tok, st, sizeof(T) == 4 ? "sy2sb_f32" : "sy2sb_f64", flops, bytes);
  }
  const int nsw = std::max(0, n - 2);
  const int kmax = (int)std::max<int64_t>(1, ceil_div(n - 1, B));
  if (nsw > 0) {
    T* V2 = w.V2.ensure<T>((int64_t)nsw * kmax * B);
    T* tau2 = w.tau2.ensure<T>((int64_t)nsw * kmax);
    int* ctl = w.ctl.ensure<int>((int64_t)nsw + 64);
    int* prog = ctl + 64;
    MSQRT_HIP(hipMemsetAsync(ctl, 0, sizeof(int) * ((size_t)nsw + 64), st));
    const int tok2 = prof_begin(st);
    const int G = std::min(nsw, 512);
    hipLaunchKernelGGL((sb2st_kernel<T, B>), dim3(G), dim3(kWave), 0, st, n, nsw, kmax, AB, V2,
                       tau2, prog, ctl);
    MSQRT_LAUNCH_CHECK();
    if (tok2 >= 0) {
      // algorithmic traffic: every step reads and writes two B x B blocks
      const double steps = 0.5 * (double)nsw * (n - 1) / B;
      prof_end(tok2, st, sizeof(T) == 4 ? "sb2st_f32" : "sb2st_f64", steps * 8.0 * B * B,
               steps * 4.0 * B * B * sizeof(T));
    }
  }
  w.n = n;
  w.nsw = nsw;
  w.kmax = kmax;
  hipLaunchKernelGGL((band_diag_kernel<T, B>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st,
                     n, (const T*)AB, d, e);
  MSQRT_LAUNCH_CHECK();
}

template <typename T>
void sy2tr_back(hipStream_t st, int n, T* Z, Sy2trWork& w, OrmtrWork& ow) {
  constexpr int B = BandWidth<T>::B;
  if (w.nsw > 0) {
    const int lds_max = 160 * 1024;
    const int64_t ring = ((int64_t)2 * w.kmax * (B + 1) + 2 * w.kmax) * sizeof(T);
    const int64_t zpad = ((int64_t)n / B + 1) * sizeof(T);
    const int nc =
        (int)std::min<int64_t>(16, (lds_max - ring - zpad) / ((int64_t)n * sizeof(T)));
    if (nc < 1 || (int64_t)w.kmax * B > 8 * kPT)
      throw Error{MSQRT_ERR_UNSUPPORTED, "back-transformation: n too large"};
    const size_t lds = (size_t)n * nc * sizeof(T) + (size_t)(ring + zpad);
    static bool attr_set[2] = {false, false};
    if (!attr_set[sizeof(T) == 8]) {
      MSQRT_HIP(hipFuncSetAttribute((const void*)apply_q2_kernel<T, B>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds_max));
      attr_set[sizeof(T) == 8] = true;
    }
    const int tok = prof_begin(st);
    hipLaunchKernelGGL((apply_q2_kernel<T, B>), dim3((unsigned)ceil_div(n, nc)), dim3(kPT), lds, st,
                       n, w.nsw, w.kmax, nc, (const T*)w.V2.p, (const T*)w.tau2.p, Z);
    MSQRT_LAUNCH_CHECK();
    if (tok >= 0) {
      const double refl = 0.5 * (double)w.nsw * (n - 1) / B;
      prof_end(tok, st, sizeof(T) == 4 ? "apply_q2_f32" : "apply_q2_f64", refl * 4.0 * B * n,
               2.0 * (double)n * n * sizeof(T));
    }
  }
  const int nref = n - B - 1;
  if (nref > 0) ormtr_blocks<T>(st, n, nref, B, (const T*)w.V1.p, (const T*)w.tau1.p, Z, ow);
}

bool sy2tr_failed(Sy2trWork& w) {
  if (!w.ctl.p || w.nsw <= 0) return false;
  int flag[2] = {0, 0};
  MSQRT_HIP(hipMemcpy(flag, w.ctl.p, sizeof(flag), hipMemcpyDeviceToHost));
  return flag[1] != 0;
}

template void sy2tr<float>(hipStream_t, int, float*, float*, float*, Sy2trWork&);
template void sy2tr<double>(hipStream_t, int, double*, double*, double*, Sy2trWork&);
template void sy2tr_back<float>(hipStream_t, int, float*, Sy2trWork&, OrmtrWork&);
template void sy2tr_back<double>(hipStream_t, int, double*, Sy2trWork&, OrmtrWork&);

}  // namespace msqrt
