// Real Schur form of a real upper Hessenberg matrix by the Francis
// double-shift QR algorithm: the real Schur decomposition A = Q T Q^T of the
// remark on real input in Sec. 2.2.1 (T quasi-upper-triangular, 1x1 blocks
// for real eigenvalues, 2x2 blocks for complex conjugate pairs), GPU-resident.
//
//  * Blocks of at most RWin<T>::W rows are finished inside one workgroup: the
//    block and the accumulated orthogonal U live in LDS and double-shift
//    steps (3-element Householder reflectors, shifts = eigenvalues of the
//    trailing 2x2, exceptional shifts after 10 steps without deflation) run
//    until every diagonal block has order 1 or 2.  A converged 2x2 block is
//    rotated to standard form: upper triangular when its eigenvalues are
//    real, equal diagonal entries and off-diagonal entries of opposite sign
//    when they are a complex pair (rsmall_kernel).
//  * Larger active blocks are swept with a chain of ns/2 double-shift bulges
//    whose shift pairs are the eigenvalues of the trailing ns x ns block
//    (complex pairs together, real eigenvalues paired in order).  The chain
//    is chased in windows: one workgroup applies every reflector that fits
//    the window to its LDS copy and accumulates U (rchase_kernel); the rest
//    of H and Z is updated with U in one launch (rapply_kernel).
//  * Between sweeps, subdiagonal entries below u (|h_kk| + |h_k+1,k+1|) or
//    below u ||H||_F are set to zero and the active block shrinks.
// H and Z are real n x n, column-major, ld n.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"
#include "schur.hpp"

namespace msqrt {

namespace {

template <typename T> struct RWin;
template <> struct RWin<float> { static constexpr int W = 128, NS = 24; };
template <> struct RWin<double> { static constexpr int W = 64, NS = 16; };

constexpr int kRQrThreads = 256;
constexpr int kRApplyThreads = 1024;
constexpr int kRChaseThreads = 1024;
constexpr int kMaxBulges = 16;
constexpr int kRExited = 1 << 30;
constexpr int kRSchedCap = 3072;

template <typename T>
__device__ inline T reps();
template <> __device__ inline float reps<float>() { return 5.9604645e-08f; }
template <> __device__ inline double reps<double>() { return 1.1102230246251565e-16; }
template <typename T>
__device__ inline T rtiny();
template <> __device__ inline float rtiny<float>() { return 1.1754944e-38f; }
template <> __device__ inline double rtiny<double>() { return 2.2250738585072014e-308; }

// Householder reflector P = I - tau v v^T, v = (1, w1, w2), with
// P (x0, x1, x2)^T = (beta, 0, 0)^T (x2 = 0 and w2 = 0 for a 2-element
// reflector).  The vector is scaled by its largest entry first, so neither a
// subnormal nor a huge bulge over- or underflows.
template <typename T>
__device__ inline void house3(T x0, T x1, T x2, T& tau, T& w1, T& w2, T& beta) {
  const T sc = fmax(fabs(x0), fmax(fabs(x1), fabs(x2)));
  if (sc == T(0) || (x1 == T(0) && x2 == T(0))) {
    tau = T(0);
    w1 = w2 = T(0);
    beta = x0;
    return;
  }
  const T a = x0 / sc, b = x1 / sc, c = x2 / sc;
  const T nrm = sqrt(a * a + b * b + c * c);
  const T bs = a >= T(0) ? -nrm : nrm;
  tau = (bs - a) / bs;
  const T den = a - bs;
  w1 = b / den;
  w2 = c / den;
  beta = bs * sc;
}

// y <- P y for the 3-vector (y0, y1, y2) (y2 unused when nr = 2, w2 = 0).
template <typename T>
__device__ inline void refl3(T tau, T w1, T w2, T& y0, T& y1, T& y2) {
  const T s = tau * (y0 + w1 * y1 + w2 * y2);
  y0 -= s;
  y1 -= s * w1;
  y2 -= s * w2;
}

// Rotation G = [[c, -s], [s, c]] that brings the 2x2 block [[a, b], [e, d]]
// one step towards standard form under G^T M G:
//   real eigenvalues (((a - d)/2)^2 + b e >= 0): the first column of G is an
//     eigenvector, so the rotated block is upper triangular;
//   complex pair: 2 theta solves (a - d) cos 2t + (b + e) sin 2t = 0, the
//     difference of the rotated diagonal entries, which then agree.
// Returns 0 when the block already is in standard form, 1 for the real case,
// 2 for the complex case.
template <typename T>
__device__ inline int std_rotation(T a, T b, T e, T d, T& c, T& s) {
  c = T(1);
  s = T(0);
  if (e == T(0)) return 0;
  const T sc = fmax(fmax(fabs(a - d), fabs(b)), fabs(e));
  const T p = T(0.5) * (a - d) / sc;
  const T disc = p * p + (b / sc) * (e / sc);
  if (disc >= T(0)) {
    const T r = sqrt(disc);
    const T lm = p + (p >= T(0) ? r : -r);  // (lambda - d) / sc
    const T es = e / sc;
    const T nrm = sqrt(lm * lm + es * es);
    c = lm / nrm;
    s = es / nrm;
    return 1;
  }
  if (a == d) return 0;  // equal diagonal and b e < 0
  const T u = (a - d) / sc, v = (b + e) / sc;
  const T r = sqrt(u * u + v * v);
  const T c2 = v / r, s2 = -u / r;
  if (c2 >= T(0)) {
    c = sqrt(T(0.5) * (T(1) + c2));
    s = s2 / (T(2) * c);
  } else {
    s = sqrt(T(0.5) * (T(1) - c2));
    if (s2 < T(0)) s = -s;
    c = s2 / (T(2) * s);
  }
  return 2;
}

// Standardises the converged 2x2 block at rows/columns (p, p + 1) of the LDS
// block h (order m, stride ldh) and accumulates the rotation in u (if any).
// Called by the whole workgroup; the rotation is computed redundantly by
// every thread from the same LDS values, so it is uniform.
template <typename T>
__device__ void standardize_2x2(T* h, int ldh, T* u, int m, int p) {
  for (int pass = 0; pass < 3; ++pass) {
    const T a = h[p + p * ldh], b = h[p + (p + 1) * ldh];
    const T e = h[p + 1 + p * ldh], d = h[p + 1 + (p + 1) * ldh];
    T c, s;
    const int kind = std_rotation(a, b, e, d, c, s);
    __syncthreads();
    if (kind == 0) return;
    // rows p, p+1 (columns p..m-1): G^T
    for (int j = p + threadIdx.x; j < m; j += blockDim.x) {
      const T x = h[p + j * ldh], y = h[p + 1 + j * ldh];
      h[p + j * ldh] = c * x + s * y;
      h[p + 1 + j * ldh] = -s * x + c * y;
    }
    __syncthreads();
    // columns p, p+1 (rows 0..p+1 of H, all rows of U): G
    const int nh = p + 2, nu = u ? m : 0;
    for (int x = threadIdx.x; x < nh + nu; x += blockDim.x) {
      T* M = x < nh ? h : u;
      const int i = x < nh ? x : x - nh;
      const T y0 = M[i + p * ldh], y1 = M[i + (p + 1) * ldh];
      M[i + p * ldh] = c * y0 + s * y1;
      M[i + (p + 1) * ldh] = -s * y0 + c * y1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (kind == 1) {
        h[p + 1 + p * ldh] = T(0);
      } else {
        const T avg = T(0.5) * (h[p + p * ldh] + h[p + 1 + (p + 1) * ldh]);
        h[p + p * ldh] = avg;
        h[p + 1 + (p + 1) * ldh] = avg;
      }
    }
    __syncthreads();
  }
}

// Double-shift QR on the LDS block h (order m) until every diagonal block
// has order 1 or 2 (2x2 blocks standardised).  A subdiagonal entry counts as
// negligible below dtol (|h_kk| + |h_k+1,k+1|): the unit roundoff for a Schur
// form, a looser value when only shifts are wanted.  Returns false when the
// iteration limit was hit.
template <typename T>
__device__ bool lds_francis(T* h, int ldh, T* u, int m, T hnorm, T dtol) {
  __shared__ int sh_l;
  const T ulp = dtol, small = fmax(rtiny<T>() * T(1e4), reps<T>() * hnorm);
  int hi = m - 1, its = 0, total = 0;
  const int itmax = 30 * max(10, m);
  const bool w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave) == 0;
  while (hi >= 1) {
    if (w0) sh_l = 0;
    __syncthreads();
    for (int k = hi - (int)threadIdx.x; k >= 1; k -= blockDim.x) {
      const T sub = fabs(h[k + (k - 1) * ldh]);
      const T tst = fabs(h[k - 1 + (k - 1) * ldh]) + fabs(h[k + k * ldh]);
      if (sub <= ulp * tst || sub <= small) atomicMax(&sh_l, k);
    }
    __syncthreads();
    const int l = __builtin_amdgcn_readfirstlane(sh_l);
    __syncthreads();
    if (l > 0 && w0) h[l + (l - 1) * ldh] = T(0);
    __syncthreads();
    if (l == hi) { hi -= 1; its = 0; continue; }
    if (l == hi - 1) {
      standardize_2x2<T>(h, ldh, u, m, hi - 1);
      hi -= 2;
      its = 0;
      continue;
    }
    if (++total > itmax) return false;
    ++its;
    // shift pair as its sum tr and product det
    T tr, det;
    if (its % 10 == 0) {
      // exceptional pair: real part moved off the trailing entry by a
      // multiple of the coupling, imaginary part half that multiple
      T e = fabs(h[hi + (hi - 1) * ldh]);
      if (hi - 2 >= l) e += fabs(h[hi - 1 + (hi - 2) * ldh]);
      const T re = h[hi + hi * ldh] + T(0.75) * e, im = T(0.5) * e;
      tr = T(2) * re;
      det = re * re + im * im;
    } else {
      const T a = h[hi - 1 + (hi - 1) * ldh], b = h[hi - 1 + hi * ldh];
      const T c = h[hi + (hi - 1) * ldh], d = h[hi + hi * ldh];
      tr = a + d;
      det = a * d - b * c;
    }
    // first column of (H - s1 I)(H - s2 I) = H^2 - tr H + det I at row l
    const T h00 = h[l + l * ldh], h10 = h[l + 1 + l * ldh], h01 = h[l + (l + 1) * ldh];
    const T h11 = h[l + 1 + (l + 1) * ldh], h21 = h[l + 2 + (l + 1) * ldh];
    const T v0 = h00 * h00 + h01 * h10 - tr * h00 + det;
    const T v1 = h10 * (h00 + h11 - tr);
    const T v2 = h10 * h21;
    __syncthreads();
    for (int k = l - 1; k <= hi - 2; ++k) {
      const int nr = min(3, hi - k);  // reflector on rows/columns k+1 .. k+nr
      T x0, x1, x2;
      if (k == l - 1) {
        x0 = v0; x1 = v1; x2 = v2;
      } else {
        x0 = h[k + 1 + k * ldh];
        x1 = h[k + 2 + k * ldh];
        x2 = nr == 3 ? h[k + 3 + k * ldh] : T(0);
      }
      T tau, w1, w2, beta;
      house3(x0, x1, x2, tau, w1, w2, beta);
      __syncthreads();
      const int r = k + 1;
      // rows r..r+nr-1 from column max(k, l) on; column k (k >= l) becomes
      // (beta, 0, 0) exactly
      for (int j = max(k, l) + (int)threadIdx.x; j < m; j += blockDim.x) {
        if (j == k) {
          h[r + j * ldh] = beta;
          h[r + 1 + j * ldh] = T(0);
          if (nr == 3) h[r + 2 + j * ldh] = T(0);
          continue;
        }
        T y0 = h[r + j * ldh], y1 = h[r + 1 + j * ldh], y2 = nr == 3 ? h[r + 2 + j * ldh] : T(0);
        refl3(tau, w1, w2, y0, y1, y2);
        h[r + j * ldh] = y0;
        h[r + 1 + j * ldh] = y1;
        if (nr == 3) h[r + 2 + j * ldh] = y2;
      }
      __syncthreads();
      // columns r..r+nr-1: rows 0..min(k + 4, hi) of H, all rows of U
      const int nh = min(k + 4, hi) + 1, nu = u ? m : 0;
      for (int x = threadIdx.x; x < nh + nu; x += blockDim.x) {
        T* M = x < nh ? h : u;
        const int i = x < nh ? x : x - nh;
        T y0 = M[i + r * ldh], y1 = M[i + (r + 1) * ldh], y2 = nr == 3 ? M[i + (r + 2) * ldh] : T(0);
        refl3(tau, w1, w2, y0, y1, y2);
        M[i + r * ldh] = y0;
        M[i + (r + 1) * ldh] = y1;
        if (nr == 3) M[i + (r + 2) * ldh] = y2;
      }
      __syncthreads();
    }
  }
  return true;
}

// Copies the m x m block at (r0, r0) of H (ld n) to the LDS window h
// (stride W + 1), entries below the band-th subdiagonal as zero; every
// thread issues its loads before its LDS stores.
template <typename T, int W, int NT>
__device__ inline void rwin_load(T* h, const T* H, int n, int r0, int m, int band) {
  constexpr int E = (W * W + NT - 1) / NT;
  T v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = threadIdx.x + NT * e;
    const int i = x % W, j = x / W;
    v[e] = T(0);
    if (x < W * W && i < m && j < m && i <= j + band) v[e] = H[(r0 + i) + (int64_t)(r0 + j) * n];
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = threadIdx.x + NT * e;
    const int i = x % W, j = x / W;
    if (x < W * W && i < m && j < m) h[i + j * (W + 1)] = v[e];
  }
}

template <typename T, int W, int NT>
__device__ inline void rwin_identity(T* u, int m) {
  for (int x = threadIdx.x; x < W * W; x += NT) {
    const int i = x % W, j = x / W;
    if (i < m && j < m) u[i + j * (W + 1)] = i == j ? T(1) : T(0);
  }
}

// Writes the window back (entries below the band-th subdiagonal as zero) and
// U (ld W) when Uo is given.
template <typename T, int W, int NT>
__device__ inline void rwin_store(const T* h, const T* u, T* H, int n, int r0, int m, int band,
                                  T* Uo) {
  for (int x = threadIdx.x; x < W * W; x += NT) {
    const int i = x % W, j = x / W;
    if (i >= m || j >= m) continue;
    H[(r0 + i) + (int64_t)(r0 + j) * n] = i <= j + band ? h[i + j * (W + 1)] : T(0);
    if (Uo) Uo[i + j * W] = u[i + j * (W + 1)];
  }
}

// Block [b0, b0 + m) of H: quasi-triangular form with U (mode 0), or the
// shift pairs of its eigenvalues (mode 1, H untouched): sp[2 q] = sum and
// sp[2 q + 1] = product of pair q, complex conjugate pairs first, then the
// real eigenvalues paired in order.
// NT threads: 256 for the blocks finished in LDS, one wave for the shift
// computation on the trailing ns x ns block (whose barriers then cost
// almost nothing).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void rsmall_kernel(int n, T* H, int b0, int m, int mode,
                                                    T* Uo, T* sp, int* status, T hnorm) {
  constexpr int W = RWin<T>::W;
  extern __shared__ unsigned char smem_raw[];
  T* h = reinterpret_cast<T*>(smem_raw);
  T* u = h + (W + 1) * W;
  const int ldh = W + 1;
  if constexpr (NT >= kRQrThreads) {
    rwin_load<T, W, NT>(h, H, n, b0, m, 1);
  } else {
    // small blocks (the shift computation): a plain loop over the m x m block
    for (int x = threadIdx.x; x < m * m; x += NT) {
      const int i = x % m, j = x / m;
      h[i + j * (W + 1)] = i <= j + 1 ? H[(b0 + i) + (int64_t)(b0 + j) * n] : T(0);
    }
  }
  if (mode == 0) rwin_identity<T, W, NT>(u, m);
  __syncthreads();
  // shifts need a few correct digits only: blocks of the trailing matrix are
  // split once their coupling is below 2^-10 of the adjacent diagonal
  const T dtol = mode == 0 ? reps<T>() : T(9.765625e-4);
  const bool ok = lds_francis<T>(h, ldh, mode == 0 ? u : nullptr, m, hnorm, dtol);
  __syncthreads();
  if (!ok && threadIdx.x == 0) atomicOr(status, 1);
  if (mode == 1) {
    if (threadIdx.x == 0) {
      int q = 0;
      // complex pairs
      for (int i = 0; i < m;) {
        if (i + 1 < m && h[i + 1 + i * ldh] != T(0)) {
          const T a = h[i + i * ldh], d = h[i + 1 + (i + 1) * ldh];
          const T b = h[i + (i + 1) * ldh], e = h[i + 1 + i * ldh];
          sp[2 * q] = a + d;
          sp[2 * q + 1] = a * d - b * e;
          ++q;
          i += 2;
        } else {
          ++i;
        }
      }
      // real eigenvalues, paired in order
      T pend = T(0);
      bool have = false;
      for (int i = 0; i < m;) {
        if (i + 1 < m && h[i + 1 + i * ldh] != T(0)) { i += 2; continue; }
        const T lam = h[i + i * ldh];
        if (have) {
          sp[2 * q] = pend + lam;
          sp[2 * q + 1] = pend * lam;
          ++q;
          have = false;
        } else {
          pend = lam;
          have = true;
        }
        ++i;
      }
    }
    return;
  }
  rwin_store<T, W, NT>(h, u, H, n, b0, m, 1, Uo);
}

// ---- the double-shift bulge chain schedule (host)
//
// A bulge at position k next applies a reflector on indices k+1..k+3 (the
// last one, at k = hi - 2, on hi - 1, hi), computed from column k; its row
// operation starts at column k and its column operation reaches row k + 4.
// In a round each bulge moves one step when the rows it touches stay inside
// the window and the bulge ahead of it (already moved this round) sits at
// position >= k + 4; a new bulge is introduced at lo (reflector on lo..lo+2
// from the shift pair) when the bulge ahead sits at >= lo + 3.  The
// reflectors of one round then act on disjoint index sets and none reads an
// entry another changes, so they commute: the kernel computes them all from
// the state before the round, applies all row operations, then all column
// operations.
struct RChain {
  int nb, nintro;
  int pos[kMaxBulges];
};

inline int rmove_code(int kind, int j, int kl) { return (kind << 24) | (j << 16) | kl; }

inline bool rchain_round(RChain& ch, int s, int wend, int lo, int hi, std::vector<int>& mv) {
  bool progress = false;
  for (int j = 0; j < ch.nintro; ++j) {
    const int k = ch.pos[j];
    if (k == kRExited || k < s) continue;
    const bool exit_move = (k == hi - 2);
    if (std::min(k + 4, hi) > wend) continue;
    if (j > 0 && ch.pos[j - 1] != kRExited && ch.pos[j - 1] < k + 4) continue;
    mv.push_back(rmove_code(exit_move ? 1 : 0, j, k - s));
    ch.pos[j] = exit_move ? kRExited : k + 1;
    progress = true;
  }
  if (ch.nintro < ch.nb && s <= lo && std::min(lo + 3, hi) <= wend &&
      (ch.nintro == 0 || ch.pos[ch.nintro - 1] == kRExited || ch.pos[ch.nintro - 1] >= lo + 3)) {
    mv.push_back(rmove_code(2, ch.nintro, lo - s));
    ch.pos[ch.nintro] = lo;
    ch.nintro++;
    progress = true;
  }
  return progress;
}

struct RSweep {
  std::vector<int> win, rnd, mv;
};

inline void build_rsweep(int lo, int hi, int nb, int W, RSweep& sw) {
  sw.win.clear();
  sw.rnd.clear();
  sw.mv.clear();
  RChain ch;
  ch.nb = nb;
  ch.nintro = 0;
  for (int j = 0; j < kMaxBulges; ++j) ch.pos[j] = -1;
  int s = lo;
  for (int guard = 0;; ++guard) {
    if (guard > 4 * (hi - lo + 2))
      throw Error{MSQRT_ERR_DEVICE, "real Schur QR: bulge schedule did not finish"};
    const int wl = std::min(W, hi - s + 1);
    const int r0 = (int)sw.rnd.size() / 2;
    for (;;) {
      const int m0 = (int)sw.mv.size();
      if (!rchain_round(ch, s, s + wl - 1, lo, hi, sw.mv)) break;
      sw.rnd.push_back(m0);
      sw.rnd.push_back((int)sw.mv.size() - m0);
    }
    sw.win.push_back(s);
    sw.win.push_back(wl);
    sw.win.push_back(r0);
    sw.win.push_back((int)sw.rnd.size() / 2 - r0);
    bool all_gone = ch.nintro == nb;
    int top = kRExited;
    for (int j = 0; j < ch.nintro; ++j)
      if (ch.pos[j] != kRExited) {
        all_gone = false;
        top = std::min(top, ch.pos[j]);
      }
    if (all_gone) break;
    const int next = ch.nintro < nb ? lo : top;
    if (next == s) throw Error{MSQRT_ERR_DEVICE, "real Schur QR: bulge chain does not fit the window"};
    s = next;
  }
}

// One window of a sweep: every round's reflectors applied in LDS, U
// accumulated.  The rounds (first move, count) and the move codes are copied
// to LDS first (at most kRSchedCap ints; the host splits longer schedules).
template <typename T>
__global__ __launch_bounds__(kRChaseThreads) void rchase_kernel(int n, T* H, int s, int wl,
                                                                int nrounds,
                                                                const int* __restrict__ rnd,
                                                                const int* __restrict__ mv,
                                                                int mv0, int nmv, const T* sp,
                                                                T* Uo) {
  constexpr int W = RWin<T>::W;
  constexpr int G = kRChaseThreads / kMaxBulges;  // lanes per move: every move at once
  constexpr int RI = (W + G - 1) / G;             // row-operation columns per lane
  constexpr int CI = (2 * W + G - 1) / G;         // column-operation rows per lane
  static_assert(G >= kWave, "a move's lanes form whole waves");
  extern __shared__ unsigned char smem_raw[];
  T* h = reinterpret_cast<T*>(smem_raw);
  T* u = h + (W + 1) * W;
  int* sched = reinterpret_cast<int*>(u + (W + 1) * W);
  const int ldh = W + 1;
  const int t = threadIdx.x;
  for (int x = t; x < 2 * nrounds; x += blockDim.x) sched[x] = rnd[x];
  for (int x = t; x < nmv; x += blockDim.x) sched[2 * nrounds + x] = mv[mv0 + x];
  rwin_load<T, W, kRChaseThreads>(h, H, n, s, wl, 3);
  rwin_identity<T, W, kRChaseThreads>(u, wl);
  __syncthreads();
  const int* smv = sched + 2 * nrounds;
  const int lane = t % G, grp = t / G;
  static_assert(G == kWave, "one wave per move: its lanes read the reflector's vector before any writes it");
  for (int ri = 0; ri < nrounds; ++ri) {
    const int moff = sched[2 * ri] - mv0, nm = sched[2 * ri + 1];
    // Wave q owns move q of the round.  Every lane forms the move's
    // reflector itself (the same values in every lane) from the state the
    // previous round left: no other move of this round writes the entries it
    // reads (a bulge's rows and columns are disjoint from its neighbours'),
    // so no barrier separates the reflectors from the row operations.
    T tau = T(0), w1 = T(0), w2 = T(0), beta = T(0);
    int r = 0, nr = 0, c0 = 0, z = -1, r1 = 0;
    if (grp < nm) {
      const int code = smv[moff + grp];
      const int kind = code >> 24, j = (code >> 16) & 0xff, kl = code & 0xffff;
      T x0, x1, x2;
      if (kind == 2) {
        // introduction at lo (local kl) from shift pair j
        const T tr = sp[2 * j], det = sp[2 * j + 1];
        const T h00 = h[kl + kl * ldh], h10 = h[kl + 1 + kl * ldh], h01 = h[kl + (kl + 1) * ldh];
        const T h11 = h[kl + 1 + (kl + 1) * ldh], h21 = h[kl + 2 + (kl + 1) * ldh];
        x0 = h00 * h00 + h01 * h10 - tr * h00 + det;
        x1 = h10 * (h00 + h11 - tr);
        x2 = h10 * h21;
        r = kl;
        nr = 3;
        c0 = kl;
        z = -1;
      } else {
        nr = kind == 1 ? 2 : 3;
        x0 = h[kl + 1 + kl * ldh];
        x1 = h[kl + 2 + kl * ldh];
        x2 = nr == 3 ? h[kl + 3 + kl * ldh] : T(0);
        r = kl + 1;
        c0 = kl;
        z = kl;
      }
      house3(x0, x1, x2, tau, w1, w2, beta);
      if (nr != 3) w2 = T(0);
      r1 = min(r + nr, wl - 1);  // last row of the column operation
      // row operations (rows r..r+nr-1 of every move; disjoint).  A lane's
      // RI column items are all loaded before any is written, so their LDS
      // latencies overlap.
      T y[RI][3];
#pragma unroll
      for (int e = 0; e < RI; ++e) {
        const int jj = c0 + lane + G * e;
        const bool live = jj < wl && jj != z;
        y[e][0] = live ? h[r + jj * ldh] : T(0);
        y[e][1] = live ? h[r + 1 + jj * ldh] : T(0);
        y[e][2] = (live && nr == 3) ? h[r + 2 + jj * ldh] : T(0);
      }
#pragma unroll
      for (int e = 0; e < RI; ++e) {
        const int jj = c0 + lane + G * e;
        if (jj >= wl) continue;
        if (jj == z) {
          h[r + jj * ldh] = beta;
          h[r + 1 + jj * ldh] = T(0);
          if (nr == 3) h[r + 2 + jj * ldh] = T(0);
          continue;
        }
        refl3(tau, w1, w2, y[e][0], y[e][1], y[e][2]);
        h[r + jj * ldh] = y[e][0];
        h[r + 1 + jj * ldh] = y[e][1];
        if (nr == 3) h[r + 2 + jj * ldh] = y[e][2];
      }
    }
    __syncthreads();
    // column operations of H (rows 0..r1) and U (all rows); disjoint columns
    if (grp < nm) {
      const int tot = (r1 + 1) + wl;
      T y[CI][3];
#pragma unroll
      for (int e = 0; e < CI; ++e) {
        const int x = lane + G * e;
        const bool live = x < tot;
        T* M = x <= r1 ? h : u;
        const int i = x <= r1 ? x : x - (r1 + 1);
        y[e][0] = live ? M[i + r * ldh] : T(0);
        y[e][1] = live ? M[i + (r + 1) * ldh] : T(0);
        y[e][2] = (live && nr == 3) ? M[i + (r + 2) * ldh] : T(0);
      }
#pragma unroll
      for (int e = 0; e < CI; ++e) {
        const int x = lane + G * e;
        if (x >= tot) continue;
        T* M = x <= r1 ? h : u;
        const int i = x <= r1 ? x : x - (r1 + 1);
        refl3(tau, w1, w2, y[e][0], y[e][1], y[e][2]);
        M[i + r * ldh] = y[e][0];
        M[i + (r + 1) * ldh] = y[e][1];
        if (nr == 3) M[i + (r + 2) * ldh] = y[e][2];
      }
    }
    __syncthreads();
  }
  rwin_store<T, W, kRChaseThreads>(h, u, H, n, s, wl, 3, Uo);
}

// Off-window update with U (order bl, ld W):
//   region R: H(b0:b0+bl, b0+bl:n) <- U^T H(...)   (column blocks of 32)
//   region A: H(0:b0, b0:b0+bl)    <- H(...) U      (row blocks of 32)
//   region Z: Z(0:n, b0:b0+bl)     <- Z(...) U      (row blocks of 32)
template <typename T>
__global__ __launch_bounds__(kRApplyThreads) void rapply_kernel(int n, T* H, T* Z, int b0, int bl,
                                                                const T* Uo, int gR, int gA) {
  constexpr int W = RWin<T>::W;
  constexpr int RS = kRApplyThreads / 32;
  constexpr int Q = (W + RS - 1) / RS;
  extern __shared__ unsigned char smem_raw[];
  T* u = reinterpret_cast<T*>(smem_raw);  // (W + 1) x W
  T* pnl = u + (W + 1) * W;               // 32 x W panel
  const int ldu = W + 1;
  const int t = threadIdx.x;
  {
    constexpr int E = (W * W + kRApplyThreads - 1) / kRApplyThreads;
    T v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kRApplyThreads * e;
      v[e] = x < W * W ? Uo[x] : T(0);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kRApplyThreads * e;
      if (x < W * W) u[x % W + (x / W) * ldu] = v[e];
    }
  }
  const int b = blockIdx.x;
  if (b < gR) {
    const int c0 = b0 + bl + 32 * b;
    const int nc = min(32, n - c0);
    {
      constexpr int E = (W * 32 + kRApplyThreads - 1) / kRApplyThreads;
      T v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = t + kRApplyThreads * e;
        const int i = x % W, j = x / W;
        v[e] = (i < bl && j < nc) ? H[(b0 + i) + (int64_t)(c0 + j) * n] : T(0);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = t + kRApplyThreads * e;
        if (x < W * 32) pnl[x % W + (x / W) * ldu] = v[e];
      }
    }
    __syncthreads();
    const int jj = t % 32, i0 = t / 32;
    T acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = T(0);
    for (int k = 0; k < bl; ++k) {
      const T hv = pnl[k + jj * ldu];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = i0 + RS * q;
        if (i < bl) acc[q] += u[k + i * ldu] * hv;
      }
    }
    if (jj < nc) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = i0 + RS * q;
        if (i < bl) H[(b0 + i) + (int64_t)(c0 + jj) * n] = acc[q];
      }
    }
    return;
  }
  T* M;
  int r0, nr;
  if (b < gR + gA) {
    M = H;
    r0 = 32 * (b - gR);
    nr = min(32, b0 - r0);
  } else {
    M = Z;
    r0 = 32 * (b - gR - gA);
    nr = min(32, n - r0);
  }
  const int ldp = 33;
  {
    constexpr int E = (W * 32 + kRApplyThreads - 1) / kRApplyThreads;
    T v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kRApplyThreads * e;
      const int i = x % 32, j = x / 32;
      v[e] = (i < nr && j < bl) ? M[(r0 + i) + (int64_t)(b0 + j) * n] : T(0);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kRApplyThreads * e;
      if (x < W * 32) pnl[x % 32 + (x / 32) * ldp] = v[e];
    }
  }
  __syncthreads();
  const int ii = t % 32, j0 = t / 32;
  T acc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = T(0);
  for (int k = 0; k < bl; ++k) {
    const T hv = pnl[ii + k * ldp];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = j0 + RS * q;
      if (j < bl) acc[q] += hv * u[k + j * ldu];
    }
  }
  if (ii < nr) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = j0 + RS * q;
      if (j < bl) M[(r0 + ii) + (int64_t)(b0 + j) * n] = acc[q];
    }
  }
}

// Zero negligible subdiagonal entries in (lo, hi] and report the largest such
// index (or lo) in out[0] (same test as the LDS iteration).
template <typename T>
__global__ __launch_bounds__(1024) void rdeflate_kernel(int n, T* H, int lo, int hi, int* out,
                                                       T hnorm) {
  __shared__ int best;
  if (threadIdx.x == 0) best = lo;
  __syncthreads();
  const T ulp = reps<T>(), small = fmax(rtiny<T>() * T(1e4), ulp * hnorm);
  for (int k = lo + 1 + threadIdx.x; k <= hi; k += blockDim.x) {
    const T a = fabs(H[k + (int64_t)(k - 1) * n]);
    const T tst = fabs(H[(k - 1) + (int64_t)(k - 1) * n]) + fabs(H[k + (int64_t)k * n]);
    if (a <= ulp * tst || a <= small) {
      H[k + (int64_t)(k - 1) * n] = T(0);
      atomicMax(&best, k);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) out[0] = best;
}

template <typename T>
size_t rwin_lds() {
  constexpr int W = RWin<T>::W;
  return sizeof(T) * (size_t)(W + 1) * W * 2;
}
template <typename T>
size_t rchase_lds() {
  return rwin_lds<T>() + sizeof(int) * kRSchedCap;
}
template <typename T>
size_t rapply_lds() {
  constexpr int W = RWin<T>::W;
  return sizeof(T) * ((size_t)(W + 1) * W + std::max<size_t>((size_t)(W + 1) * 32, 33 * (size_t)W));
}

template <typename T>
void launch_rapply(hipStream_t st, int n, T* H, T* Z, int b0, int bl, const T* U) {
  const int gR = (int)ceil_div(n - b0 - bl, 32);
  const int gA = (int)ceil_div(b0, 32);
  const int gZ = (int)ceil_div(n, 32);
  const int g = gR + gA + gZ;
  if (g == 0) return;
  hipLaunchKernelGGL(rapply_kernel<T>, dim3(g), dim3(kRApplyThreads), rapply_lds<T>(), st, n, H, Z,
                     b0, bl, U, gR, gA);
  MSQRT_LAUNCH_CHECK();
}

}  // namespace

template <typename T>
bool rhseqr(hipStream_t st, int n, T* H, T* Z, HseqrWork& w, T hnorm) {
  constexpr int W = RWin<T>::W, NS = RWin<T>::NS;
  static_assert(NS / 2 <= kMaxBulges && NS <= W, "shift count");
  static bool attr_set = false;
  if (!attr_set) {
    MSQRT_HIP(hipFuncSetAttribute((const void*)rsmall_kernel<T, kRQrThreads>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)rwin_lds<T>()));
    MSQRT_HIP(hipFuncSetAttribute((const void*)rsmall_kernel<T, kWave>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)rwin_lds<T>()));
    MSQRT_HIP(hipFuncSetAttribute((const void*)rchase_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)rchase_lds<T>()));
    MSQRT_HIP(hipFuncSetAttribute((const void*)rapply_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)rapply_lds<T>()));
    attr_set = true;
  }
  if (n <= 0) return true;
  RSweep sw;
  T* U = w.U.ensure<T>((int64_t)W * W);
  T* sp = w.shifts.ensure<T>(NS + 8);
  int* flag = w.flag.ensure<int>(4);
  MSQRT_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, st));
  const int nb = NS / 2;
  int hi = n - 1;
  int sweeps = 0, stuck = 0, last_hi = -1, last_lo = -1;
  const int max_sweeps = 30 * std::max(10, n / NS) + 100;
  while (hi >= 0) {
    int lo = 0;
    if (hi > 0) {
      hipLaunchKernelGGL(rdeflate_kernel<T>, dim3(1), dim3(1024), 0, st, n, H, 0, hi, flag + 1, hnorm);
      MSQRT_LAUNCH_CHECK();
      MSQRT_HIP(hipMemcpyAsync(&lo, flag + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      MSQRT_HIP(hipStreamSynchronize(st));
    }
    const int m = hi - lo + 1;
    if (m <= W) {
      if (m > 1) {
        if (m <= kWave)
          hipLaunchKernelGGL((rsmall_kernel<T, kWave>), dim3(1), dim3(kWave), rwin_lds<T>(), st, n,
                             H, lo, m, 0, U, sp, flag, hnorm);
        else
          hipLaunchKernelGGL((rsmall_kernel<T, kRQrThreads>), dim3(1), dim3(kRQrThreads),
                             rwin_lds<T>(), st, n, H, lo, m, 0, U, sp, flag, hnorm);
        MSQRT_LAUNCH_CHECK();
        launch_rapply<T>(st, n, H, Z, lo, m, U);
      }
      hi = lo - 1;
      continue;
    }
    if (++sweeps > max_sweeps) return false;
    if (hi == last_hi && lo == last_lo) ++stuck;
    else stuck = 0;
    if (stuck > 300) return false;
    last_hi = hi;
    last_lo = lo;
    hipLaunchKernelGGL((rsmall_kernel<T, kWave>), dim3(1), dim3(kWave), rwin_lds<T>(), st, n, H,
                       hi - NS + 1, NS, 1, U, sp, flag, hnorm);
    MSQRT_LAUNCH_CHECK();
    if (stuck > 0 && stuck % 6 == 0) {
      // exceptional sweep: complex pairs around the trailing entry, moved off
      // it by multiples of the coupling
      T sub = 0, dd = 0;
      MSQRT_HIP(hipMemcpyAsync(&sub, H + hi + (int64_t)(hi - 1) * n, sizeof(T),
                               hipMemcpyDeviceToHost, st));
      MSQRT_HIP(hipMemcpyAsync(&dd, H + hi + (int64_t)hi * n, sizeof(T), hipMemcpyDeviceToHost, st));
      MSQRT_HIP(hipStreamSynchronize(st));
      const T e = std::fabs(sub);
      std::vector<T> hs(NS);
      for (int q = 0; q < nb; ++q) {
        const T re = dd + (q % 2 ? -e : e) * T(0.75) * T(1 + q % 3);
        const T im = T(0.5) * e;
        hs[2 * q] = T(2) * re;
        hs[2 * q + 1] = re * re + im * im;
      }
      MSQRT_HIP(hipMemcpyAsync(sp, hs.data(), sizeof(T) * NS, hipMemcpyHostToDevice, st));
      MSQRT_HIP(hipStreamSynchronize(st));
    }
    build_rsweep(lo, hi, nb, W, sw);
    const int nr = (int)sw.rnd.size(), nm = (int)sw.mv.size();
    int* dsched = w.scratch.ensure<int>(nr + nm + 64);
    MSQRT_HIP(hipMemcpyAsync(dsched, sw.rnd.data(), sizeof(int) * nr, hipMemcpyHostToDevice, st));
    MSQRT_HIP(hipMemcpyAsync(dsched + nr, sw.mv.data(), sizeof(int) * nm, hipMemcpyHostToDevice, st));
    for (size_t wi = 0; wi < sw.win.size(); wi += 4) {
      const int s = sw.win[wi], wl = sw.win[wi + 1], r0 = sw.win[wi + 2], nrw = sw.win[wi + 3];
      for (int ra = 0; ra < nrw;) {
        int rb = ra, used = 0;
        while (rb < nrw) {
          const int cnt = sw.rnd[2 * (r0 + rb) + 1];
          if (used + 2 + cnt > kRSchedCap) break;
          used += 2 + cnt;
          ++rb;
        }
        if (rb == ra) throw Error{MSQRT_ERR_DEVICE, "real Schur QR: round larger than the LDS schedule"};
        const int mv0 = sw.rnd[2 * (r0 + ra)];
        const int mv1 = sw.rnd[2 * (r0 + rb - 1)] + sw.rnd[2 * (r0 + rb - 1) + 1];
        hipLaunchKernelGGL(rchase_kernel<T>, dim3(1), dim3(kRChaseThreads), rchase_lds<T>(), st, n, H,
                           s, wl, rb - ra, (const int*)(dsched + 2 * (r0 + ra)),
                           (const int*)(dsched + nr), mv0, mv1 - mv0, (const T*)sp, U);
        MSQRT_LAUNCH_CHECK();
        launch_rapply<T>(st, n, H, Z, s, wl, U);
        ra = rb;
      }
    }
    MSQRT_HIP(hipStreamSynchronize(st));
  }
  int hflag = 0;
  MSQRT_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipStreamSynchronize(st));
  return hflag == 0;
}

template bool rhseqr<float>(hipStream_t, int, float*, float*, HseqrWork&, float);
template bool rhseqr<double>(hipStream_t, int, double*, double*, HseqrWork&, double);

}  // namespace msqrt
