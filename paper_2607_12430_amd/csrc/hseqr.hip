// Complex Schur form of an upper Hessenberg matrix by the shifted QR
// algorithm (the Schur decomposition of Alg. 2), GPU-resident.
//
//  * Blocks of at most kWin<T> rows are finished inside one workgroup: the
//    block and the accumulated unitary U live in LDS and the single-shift
//    QR iteration (Wilkinson shifts, exceptional shifts after 10 iterations
//    without deflation) runs to completion (small_schur_kernel).
//  * Larger active blocks are swept with a chain of ns single-shift bulges
//    (shifts = eigenvalues of the trailing ns x ns block).  The chain is
//    chased down in windows: one workgroup applies every rotation that fits
//    in the window to the LDS copy of the window and accumulates U
//    (chase_kernel); the rest of H and Z is then updated with U in one
//    launch (apply_u_kernel): H(win, right) <- U^* H(win, right),
//    H(above, win) <- H(above, win) U, Z(:, win) <- Z(:, win) U.
//  * After every sweep subdiagonal entries below u (|h_kk| + |h_k+1,k+1|)
//    are set to zero and the active block shrinks from the bottom.
// Rotations: G = [c s; -conj(s) c] with real c, H <- G H G^*, U <- U G^*.
#include <algorithm>
#include <cstring>
#include <vector>

#include "kernels.hpp"
#include "schur.hpp"

namespace msqrt {

namespace {

template <typename T> struct Win;
template <> struct Win<float> { static constexpr int W = 96, NS = 24; };
template <> struct Win<double> { static constexpr int W = 64, NS = 16; };

constexpr int kQrThreads = 256;
// off-window updates: two waves per SIMD at one workgroup per CU
constexpr int kApplyThreads = 1024;
constexpr int kMaxNs = 32;
constexpr int kExited = 1 << 30;

template <typename T>
__device__ inline T eps_of();
template <> __device__ inline float eps_of<float>() { return 5.9604645e-08f; }
template <> __device__ inline double eps_of<double>() { return 1.1102230246251565e-16; }
template <typename T>
__device__ inline T tiny_of();
template <> __device__ inline float tiny_of<float>() { return 1.1754944e-38f; }
template <> __device__ inline double tiny_of<double>() { return 2.2250738585072014e-308; }

template <typename T>
__device__ inline T cabs1(cx<T> a) { return fabs(a.r) + fabs(a.i); }

// Rotation with G [f; g] = [r; 0].  c and s do not change when f and g are
// scaled together, so both are first divided by max(|f|_1, |g|_1): no
// reciprocal of a tiny |f| or norm is ever formed (a bulge that has decayed
// to subnormal size, as at the top of a block that is about to deflate,
// otherwise overflows 1/|f| in float32 and turns the whole window into NaN).
template <typename T>
__device__ inline void make_rot(cx<T> f, cx<T> g, T& c, cx<T>& s) {
  const T ag = cabs1(g);
  if (ag == T(0)) { c = T(1); s = {T(0), T(0)}; return; }
  const T sc = fmax(cabs1(f), ag);
  const cx<T> fs = {f.r / sc, f.i / sc}, gs = {g.r / sc, g.i / sc};
  const T af = hypot(fs.r, fs.i);
  const T agg = hypot(gs.r, gs.i);
  if (af == T(0)) { c = T(0); s = {gs.r / agg, -gs.i / agg}; return; }
  const T nrm = hypot(af, agg);
  c = af / nrm;
  // s = (f / |f|) conj(g) / nrm
  const cx<T> p = cmul(cx<T>{fs.r / af, fs.i / af}, cconj(gs));
  s = {p.r / nrm, p.i / nrm};
}

// [a; b] <- G [a; b]
template <typename T>
__device__ inline void rot_rows(T c, cx<T> s, cx<T>& a, cx<T>& b) {
  const cx<T> na = cadd(cscale(a, c), cmul(s, b));
  const cx<T> nb = csub(cscale(b, c), cmulc(s, a));
  a = na;
  b = nb;
}
// [a, b] <- [a, b] G^*
template <typename T>
__device__ inline void rot_cols(T c, cx<T> s, cx<T>& a, cx<T>& b) {
  const cx<T> na = cadd(cscale(a, c), cmul(b, cconj(s)));
  const cx<T> nb = csub(cscale(b, c), cmul(a, s));
  a = na;
  b = nb;
}

// One similarity rotation on indices (r, r+1) of the LDS matrix h (column-
// major, stride ldh) of order m and of U (same stride, order m when u != 0):
// rows r, r+1 for columns [c0, m), columns r, r+1 for rows [0, r1].
template <typename T>
__device__ void apply_rot(cx<T>* h, int ldh, cx<T>* u, int m, int r, int c0, int r1, T c,
                          cx<T> s) {
  const int t = threadIdx.x;
  const int nrow = m - c0;            // row-op columns (incl. the corner)
  const int ncol = r1 + 1;            // col-op rows (incl. the corner)
  const int nu = u ? m : 0;
  const int total = nrow + ncol + nu;
  for (int x = t; x < total; x += blockDim.x) {
    if (x < nrow) {
      const int j = c0 + x;
      if (j == r || j == r + 1) continue;
      rot_rows(c, s, h[r + j * ldh], h[r + 1 + j * ldh]);
    } else if (x < nrow + ncol) {
      const int i = x - nrow;
      if (i == r || i == r + 1) continue;
      rot_cols(c, s, h[i + r * ldh], h[i + (r + 1) * ldh]);
    } else {
      const int i = x - nrow - ncol;
      rot_cols(c, s, u[i + r * ldh], u[i + (r + 1) * ldh]);
    }
  }
  if (__builtin_amdgcn_readfirstlane(t / kWave) == 0) {
    // corner: rows then columns (G M G^*); wave 0 computes it redundantly
    // (identical values) so the branch is wave-uniform
    cx<T> a = h[r + r * ldh], b = h[r + (r + 1) * ldh];
    cx<T> cc = h[r + 1 + r * ldh], d = h[r + 1 + (r + 1) * ldh];
    rot_rows(c, s, a, cc);
    rot_rows(c, s, b, d);
    rot_cols(c, s, a, b);
    rot_cols(c, s, cc, d);
    h[r + r * ldh] = a;
    h[r + (r + 1) * ldh] = b;
    h[r + 1 + r * ldh] = cc;
    h[r + 1 + (r + 1) * ldh] = d;
  }
  __syncthreads();
}

template <typename T>
__device__ inline cx<T> csqrt_any(cx<T> z) { return csqrt_principal(z); }

// Eigenvalue of the 2 x 2 [[a, b], [c, d]] closer to d.
template <typename T>
__device__ inline cx<T> wilkinson(cx<T> a, cx<T> b, cx<T> c, cx<T> d) {
  const cx<T> p = cscale(csub(a, d), T(0.5));
  const cx<T> disc = csqrt_any(cadd(cmul(p, p), cmul(b, c)));
  const cx<T> mid = cscale(cadd(a, d), T(0.5));
  const cx<T> l1 = cadd(mid, disc), l2 = csub(mid, disc);
  return cabs1(csub(l1, d)) <= cabs1(csub(l2, d)) ? l1 : l2;
}

// Single-shift QR on the LDS matrix h (order m) until upper triangular.
// Returns false if the iteration limit was hit.
template <typename T>
__device__ bool lds_qr(cx<T>* h, int ldh, cx<T>* u, int m, T hnorm) {
  __shared__ int sh_l;
  const T ulp = eps_of<T>(), small = max(tiny_of<T>() * T(1e4), ulp * hnorm);
  int hi = m - 1, its = 0, total = 0;
  const int itmax = 30 * max(10, m);
  const bool w0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave) == 0;
  while (hi >= 1) {
    if (w0) sh_l = 0;
    __syncthreads();
    for (int k = hi - threadIdx.x; k >= 1; k -= blockDim.x) {
      const T sub = cabs1(h[k + (k - 1) * ldh]);
      const T tst = cabs1(h[k - 1 + (k - 1) * ldh]) + cabs1(h[k + k * ldh]);
      if (sub <= ulp * tst || sub <= small) atomicMax(&sh_l, k);
    }
    __syncthreads();
    // uniform by construction; readfirstlane lets the compiler see it, so the
    // barrier-carrying loops below are compiled as uniform control flow
    const int l = __builtin_amdgcn_readfirstlane(sh_l);
    __syncthreads();
    if (l > 0 && w0) h[l + (l - 1) * ldh] = {T(0), T(0)};
    if (l == hi) { hi -= 1; its = 0; __syncthreads(); continue; }
    if (++total > itmax) return false;
    ++its;
    cx<T> sigma;
    if (its % 10 == 0) {
      // exceptional shift
      const T e = T(0.75) * cabs1(h[hi + (hi - 1) * ldh]);
      sigma = cadd(h[hi + hi * ldh], cx<T>{e, T(0)});
    } else {
      sigma = wilkinson(h[hi - 1 + (hi - 1) * ldh], h[hi - 1 + hi * ldh], h[hi + (hi - 1) * ldh],
                        h[hi + hi * ldh]);
    }
    __syncthreads();
    for (int k = l; k < hi; ++k) {
      cx<T> f, g;
      if (k == l) {
        f = csub(h[l + l * ldh], sigma);
        g = h[l + 1 + l * ldh];
      } else {
        f = h[k + (k - 1) * ldh];
        g = h[k + 1 + (k - 1) * ldh];
      }
      T c;
      cx<T> s;
      make_rot(f, g, c, s);
      __syncthreads();
      const int c0 = k == l ? l : k - 1;
      apply_rot(h, ldh, u, m, k, c0, min(k + 2, hi), c, s);
      if (k > l && w0) h[k + 1 + (k - 1) * ldh] = {T(0), T(0)};
      __syncthreads();
    }
  }
  return true;
}

template <typename T>
__device__ inline cx<T> gload(const T* H, int64_t ld, int64_t i, int64_t j) {
  return {H[i + j * ld], H[i + j * ld + ld / 2]};
}
template <typename T>
__device__ inline void gstore(T* H, int64_t ld, int64_t i, int64_t j, cx<T> v) {
  H[i + j * ld] = v.r;
  H[i + j * ld + ld / 2] = v.i;
}

// Copies the m x m block at (r0, c0) of a stacked global matrix into the LDS
// window h (stride W + 1), entries below the band-th subdiagonal as zero.
// The index map uses the compile-time W and every thread issues all of its
// loads before the first LDS store, so the global latencies overlap.
template <typename T, int W, int NT>
__device__ inline void win_load(cx<T>* h, const T* H, int64_t ld, int r0, int c0, int m,
                                int band) {
  constexpr int E = (W * W + NT - 1) / NT;
  cx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = threadIdx.x + NT * e;
    const int i = x % W, j = x / W;
    v[e] = {T(0), T(0)};
    if (x < W * W && i < m && j < m && i <= j + band) v[e] = gload(H, ld, r0 + i, c0 + j);
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = threadIdx.x + NT * e;
    const int i = x % W, j = x / W;
    if (x < W * W && i < m && j < m) h[i + j * (W + 1)] = v[e];
  }
}

// U window as the identity (order m) in LDS.
template <typename T, int W, int NT>
__device__ inline void win_identity(cx<T>* u, int m) {
  for (int x = threadIdx.x; x < W * W; x += NT) {
    const int i = x % W, j = x / W;
    if (i < m && j < m) u[i + j * (W + 1)] = {i == j ? T(1) : T(0), T(0)};
  }
}

// Writes the LDS windows back: H block (lower part below the band-th
// subdiagonal as zero) and U (stacked, ld 2W).
template <typename T, int W, int NT>
__device__ inline void win_store(const cx<T>* h, const cx<T>* u, T* H, int64_t ld, int r0, int m,
                                 int band, T* Uo) {
  for (int x = threadIdx.x; x < W * W; x += NT) {
    const int i = x % W, j = x / W;
    if (i >= m || j >= m) continue;
    gstore(H, ld, r0 + i, r0 + j, i <= j + band ? h[i + j * (W + 1)] : cx<T>{T(0), T(0)});
    if (u) {
      Uo[i + (int64_t)j * 2 * W] = u[i + j * (W + 1)].r;
      Uo[i + (int64_t)j * 2 * W + W] = u[i + j * (W + 1)].i;
    }
  }
}

// Block [b0, b0 + m) of H: full Schur form with U (mode 0) or eigenvalues
// only into eig (mode 1, H untouched).
template <typename T>
__global__ __launch_bounds__(kQrThreads) void small_schur_kernel(int n, T* H, int b0, int m,
                                                                 int mode, T* Uo, cx<T>* eig,
                                                                 int* status, T hnorm) {
  constexpr int W = Win<T>::W;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* h = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* u = h + (W + 1) * W;
  const int ldh = W + 1;
  const int64_t ld = 2 * (int64_t)n;
  win_load<T, W, kQrThreads>(h, H, ld, b0, b0, m, 1);
  if (mode == 0) win_identity<T, W, kQrThreads>(u, m);
  __syncthreads();
  const bool ok = lds_qr<T>(h, ldh, mode == 0 ? u : nullptr, m, hnorm);
  __syncthreads();
  if (!ok && threadIdx.x == 0) atomicOr(status, 1);
  if (mode == 1) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) eig[i] = h[i + i * ldh];
    return;
  }
  win_store<T, W, kQrThreads>(h, u, H, ld, b0, m, 0, Uo);
}

// ---- the bulge chain schedule (host)
//
// The schedule depends only on (lo, hi, ns, window size), not on the data,
// so the host builds it for a whole sweep.  It proceeds in rounds: in every
// round each bulge moves one step if it stays inside the window and keeps
// two rows to the bulge below it (bottom bulge first), and a new bulge is
// introduced at lo when there is room.  The rotations of one round act on
// disjoint index pairs and none changes another's input column, so they
// commute: the kernel computes them together, applies all row rotations,
// then all column rotations.
struct Chain {
  int ns, nintro;
  int pos[kMaxNs];  // bulge entry at (pos + 2, pos); kExited when gone
};

// move code: kind (0 move, 1 exit move, 2 introduce) << 24 | shift << 16 | k - s
inline int move_code(int kind, int j, int kl) { return (kind << 24) | (j << 16) | kl; }

// One round inside the window [s, wend]; appends the moves to mv.
inline bool chain_round(Chain& ch, int s, int wend, int lo, int hi, std::vector<int>& mv) {
  bool progress = false;
  for (int j = 0; j < ch.nintro; ++j) {
    const int k = ch.pos[j];
    if (k == kExited || k < s) continue;
    const bool exit_move = (k + 2 == hi);
    if (exit_move ? (k + 2 > wend) : (k + 3 > wend)) continue;
    if (j > 0 && ch.pos[j - 1] != kExited && ch.pos[j - 1] < k + 3) continue;
    mv.push_back(move_code(exit_move ? 1 : 0, j, k - s));
    ch.pos[j] = exit_move ? kExited : k + 1;
    progress = true;
  }
  if (ch.nintro < ch.ns && s <= lo && lo + 2 <= wend &&
      (ch.nintro == 0 || ch.pos[ch.nintro - 1] == kExited || ch.pos[ch.nintro - 1] >= lo + 2)) {
    mv.push_back(move_code(2, ch.nintro, lo - s));
    ch.pos[ch.nintro] = lo;
    ch.nintro++;
    progress = true;
  }
  return progress;
}

// Whole-sweep schedule: per window (s, wl, first round, rounds), per round
// (first move, moves), and the move codes.
struct Sweep {
  std::vector<int> win, rnd, mv;
};

inline void build_sweep(int lo, int hi, int ns, int W, Sweep& sw) {
  sw.win.clear();
  sw.rnd.clear();
  sw.mv.clear();
  Chain ch;
  ch.ns = ns;
  ch.nintro = 0;
  for (int j = 0; j < kMaxNs; ++j) ch.pos[j] = -1;
  int s = lo;
  for (int guard = 0;; ++guard) {
    if (guard > 4 * (hi - lo + 2)) throw Error{MSQRT_ERR_DEVICE, "Schur QR: bulge schedule did not finish"};
    const int wl = std::min(W, hi - s + 1);
    const int r0 = (int)sw.rnd.size() / 2;
    for (;;) {
      const int m0 = (int)sw.mv.size();
      if (!chain_round(ch, s, s + wl - 1, lo, hi, sw.mv)) break;
      sw.rnd.push_back(m0);
      sw.rnd.push_back((int)sw.mv.size() - m0);
    }
    sw.win.push_back(s);
    sw.win.push_back(wl);
    sw.win.push_back(r0);
    sw.win.push_back((int)sw.rnd.size() / 2 - r0);
    bool all_gone = ch.nintro == ns;
    int top = kExited;
    for (int j = 0; j < ch.nintro; ++j)
      if (ch.pos[j] != kExited) {
        all_gone = false;
        top = std::min(top, ch.pos[j]);
      }
    if (all_gone) break;
    const int next = ch.nintro < ns ? lo : top;
    if (next == s) throw Error{MSQRT_ERR_DEVICE, "Schur QR: bulge chain does not fit the window"};
    s = next;
  }
}

// One window of a sweep: all rounds of rotations in LDS, U accumulated.
// The window's rounds (first move, count) and move codes are copied to LDS
// first (at most kSchedCap ints; the host splits longer schedules).
constexpr int kSchedCap = 3072;
constexpr int kChaseThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kChaseThreads) void chase_kernel(int n, T* H, int s, int wl, int nrounds,
                                                           const int* __restrict__ rnd,
                                                           const int* __restrict__ mv, int mv0,
                                                           int nmv, const cx<T>* shifts, T* Uo) {
  constexpr int W = Win<T>::W;
  constexpr int G = kChaseThreads / kMaxNs;  // lanes per move: every move at once
  constexpr int RI = (W + G - 1) / G;        // columns (rows) per lane
  static_assert(G * kMaxNs == kChaseThreads, "one lane group per move");
  extern __shared__ unsigned char smem_raw[];
  cx<T>* h = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* u = h + (W + 1) * W;
  int* sched = reinterpret_cast<int*>(u + (W + 1) * W);  // rounds, then moves
  __shared__ T rot_c[kMaxNs];
  __shared__ cx<T> rot_s[kMaxNs];
  __shared__ int rot_r[kMaxNs], rot_c0[kMaxNs], rot_r1[kMaxNs], rot_z[kMaxNs];
  const int ldh = W + 1;
  const int64_t ld = 2 * (int64_t)n;
  const int t = threadIdx.x;
  for (int x = t; x < 2 * nrounds; x += blockDim.x) sched[x] = rnd[x];
  for (int x = t; x < nmv; x += blockDim.x) sched[2 * nrounds + x] = mv[mv0 + x];
  win_load<T, W, kChaseThreads>(h, H, ld, s, s, wl, 2);
  win_identity<T, W, kChaseThreads>(u, wl);
  __syncthreads();
  const int* smv = sched + 2 * nrounds;
  const int lane_j = t % G, grp = t / G;
  for (int ri = 0; ri < nrounds; ++ri) {
    const int moff = sched[2 * ri] - mv0, nm = sched[2 * ri + 1];
    // rotations of this round (inputs from the state before the round)
    if (t < nm) {
      const int code = smv[moff + t];
      const int kind = code >> 24, j = (code >> 16) & 0xff, kl = code & 0xffff;
      cx<T> f, g;
      int r;
      if (kind == 2) {
        f = csub(h[kl + kl * ldh], shifts[j]);
        g = h[kl + 1 + kl * ldh];
        r = kl;
      } else {
        f = h[kl + 1 + kl * ldh];
        g = h[kl + 2 + kl * ldh];
        r = kl + 1;
      }
      T c;
      cx<T> sr;
      make_rot(f, g, c, sr);
      rot_c[t] = c;
      rot_s[t] = sr;
      rot_r[t] = r;
      rot_c0[t] = kl;
      rot_r1[t] = min(kind == 2 ? kl + 2 : kl + 3, wl - 1);
      rot_z[t] = kind == 2 ? -1 : kl;  // column whose bulge entry becomes 0
    }
    __syncthreads();
    // all row rotations (rows r, r+1 of every move; disjoint): lane group
    // grp owns move grp, and a lane's RI columns are loaded before any is
    // written, so their LDS latencies overlap
    if (grp < nm) {
      const int r = rot_r[grp], c0 = rot_c0[grp], z = rot_z[grp];
      const T c = rot_c[grp];
      const cx<T> sr = rot_s[grp];
      cx<T> a[RI], b[RI];
#pragma unroll
      for (int e = 0; e < RI; ++e) {
        const int j = lane_j + G * e;
        const bool live = j < wl && j >= c0;
        a[e] = live ? h[r + j * ldh] : cx<T>{T(0), T(0)};
        b[e] = live ? h[r + 1 + j * ldh] : cx<T>{T(0), T(0)};
      }
#pragma unroll
      for (int e = 0; e < RI; ++e) {
        const int j = lane_j + G * e;
        if (j < wl && j >= c0) {
          rot_rows(c, sr, a[e], b[e]);
          h[r + j * ldh] = a[e];
          h[r + 1 + j * ldh] = j == z ? cx<T>{T(0), T(0)} : b[e];
        }
      }
    }
    __syncthreads();
    // all column rotations of H (rows <= r1) and U (columns r, r+1; disjoint)
    if (grp < nm) {
      const int r = rot_r[grp], r1 = rot_r1[grp];
      const T c = rot_c[grp];
      const cx<T> sr = rot_s[grp];
      cx<T> ha[RI], hb[RI], ua[RI], ub[RI];
#pragma unroll
      for (int e = 0; e < RI; ++e) {
        const int i = lane_j + G * e;
        const bool lh = i < wl && i <= r1, lu = i < wl;
        ha[e] = lh ? h[i + r * ldh] : cx<T>{T(0), T(0)};
        hb[e] = lh ? h[i + (r + 1) * ldh] : cx<T>{T(0), T(0)};
        ua[e] = lu ? u[i + r * ldh] : cx<T>{T(0), T(0)};
        ub[e] = lu ? u[i + (r + 1) * ldh] : cx<T>{T(0), T(0)};
      }
#pragma unroll
      for (int e = 0; e < RI; ++e) {
        const int i = lane_j + G * e;
        if (i < wl && i <= r1) {
          rot_cols(c, sr, ha[e], hb[e]);
          h[i + r * ldh] = ha[e];
          h[i + (r + 1) * ldh] = hb[e];
        }
        if (i < wl) {
          rot_cols(c, sr, ua[e], ub[e]);
          u[i + r * ldh] = ua[e];
          u[i + (r + 1) * ldh] = ub[e];
        }
      }
    }
    __syncthreads();
  }
  win_store<T, W, kChaseThreads>(h, u, H, ld, s, wl, 2, Uo);
}

// Off-window update with U (order bl, stacked, ld 2W):
//   region R: H(b0:b0+bl, b0+bl:n) <- U^* H(...)       (column blocks of 32)
//   region A: H(0:b0, b0:b0+bl)    <- H(...) U          (row blocks of 32)
//   region Z: Z(0:n, b0:b0+bl)     <- Z(...) U          (row blocks of 32)
template <typename T>
__global__ __launch_bounds__(kApplyThreads) void apply_u_kernel(int n, T* H, T* Z, int b0, int bl,
                                                             const T* Uo, int gR, int gA) {
  constexpr int W = Win<T>::W;
  constexpr int RS = kApplyThreads / 32;  // thread rows
  constexpr int Q = W / RS;                // outputs per thread along the window index
  extern __shared__ unsigned char smem_raw[];
  cx<T>* u = reinterpret_cast<cx<T>*>(smem_raw);  // (W + 1) x W
  cx<T>* pnl = u + (W + 1) * W;                    // 32 x W panel, stride W + 1 or 33
  const int ldu = W + 1;
  const int64_t ld = 2 * (int64_t)n;
  const int t = threadIdx.x;
  {
    // the whole W x W buffer (entries beyond bl are never used), all loads
    // in flight together
    constexpr int E = (W * W + kApplyThreads - 1) / kApplyThreads;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kApplyThreads * e;
      const int i = x % W, j = x / W;
      v[e] = x < W * W ? cx<T>{Uo[i + (int64_t)j * 2 * W], Uo[i + (int64_t)j * 2 * W + W]}
                       : cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kApplyThreads * e;
      if (x < W * W) u[x % W + (x / W) * ldu] = v[e];
    }
  }
  const int b = blockIdx.x;
  if (b < gR) {
    // columns c0 .. c0+31 of the rows b0 .. b0+bl
    const int c0 = b0 + bl + 32 * b;
    const int nc = min(32, n - c0);
    {
      constexpr int E = (W * 32 + kApplyThreads - 1) / kApplyThreads;
      cx<T> v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = t + kApplyThreads * e;
        const int i = x % W, j = x / W;
        v[e] = (i < bl && j < nc) ? gload(H, ld, b0 + i, c0 + j) : cx<T>{T(0), T(0)};
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = t + kApplyThreads * e;
        pnl[x % W + (x / W) * ldu] = v[e];
      }
    }
    __syncthreads();
    const int jj = t % 32, i0 = t / 32;
    cx<T> acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = {T(0), T(0)};
    for (int k = 0; k < bl; ++k) {
      const cx<T> hv = pnl[k + jj * ldu];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = i0 + RS * q;
        if (i < bl) acc[q] = cadd(acc[q], cmulc(u[k + i * ldu], hv));
      }
    }
    if (jj < nc) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = i0 + RS * q;
        if (i < bl) gstore(H, ld, b0 + i, c0 + jj, acc[q]);
      }
    }
    return;
  }
  // row block: region A (H rows 0..b0) or Z (rows 0..n)
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
    constexpr int E = (W * 32 + kApplyThreads - 1) / kApplyThreads;
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kApplyThreads * e;
      const int i = x % 32, j = x / 32;
      v[e] = (i < nr && j < bl) ? gload(M, ld, r0 + i, b0 + j) : cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = t + kApplyThreads * e;
      pnl[x % 32 + (x / 32) * ldp] = v[e];
    }
  }
  __syncthreads();
  const int ii = t % 32, j0 = t / 32;
  cx<T> acc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = {T(0), T(0)};
  for (int k = 0; k < bl; ++k) {
    const cx<T> hv = pnl[ii + k * ldp];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = j0 + RS * q;
      if (j < bl) acc[q] = cadd(acc[q], cmul(hv, u[k + j * ldu]));
    }
  }
  if (ii < nr) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = j0 + RS * q;
      if (j < bl) gstore(M, ld, r0 + ii, b0 + j, acc[q]);
    }
  }
}

// Zero negligible subdiagonal entries in (lo, hi] and report the largest such
// index (or lo) in out[0].  Negligible: below ulp times the two adjacent
// diagonal entries, or below ulp ||H||_F -- a perturbation of that size is
// within the backward error the factorisation has anyway, and without the
// norm-wise floor subdiagonals next to eigenvalues much smaller than ||H||
// can stall above the local threshold in float32 (seen with one large
// outlier eigenvalue, e.g. a uniform(0, 1) matrix plus shift).
template <typename T>
__global__ __launch_bounds__(1024) void deflate_kernel(int n, T* H, int lo, int hi, int* out,
                                                      T hnorm) {
  __shared__ int best;
  const int64_t ld = 2 * (int64_t)n;
  if (threadIdx.x == 0) best = lo;
  __syncthreads();
  const T ulp = eps_of<T>(), small = max(tiny_of<T>() * T(1e4), ulp * hnorm);
  for (int k = lo + 1 + threadIdx.x; k <= hi; k += blockDim.x) {
    const cx<T> sub = gload(H, ld, k, k - 1);
    const T tst = cabs1(gload(H, ld, k - 1, k - 1)) + cabs1(gload(H, ld, k, k));
    const T a = cabs1(sub);
    if (a <= ulp * tst || a <= small) {
      gstore(H, ld, k, k - 1, cx<T>{T(0), T(0)});
      atomicMax(&best, k);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) out[0] = best;
}

// dynamic LDS of the window kernels: H and U windows (+ the schedule for
// the chase kernel)
template <typename T>
size_t win_lds() {
  constexpr int W = Win<T>::W;
  return sizeof(cx<T>) * (size_t)(W + 1) * W * 2;
}
template <typename T>
size_t chase_lds() {
  return win_lds<T>() + sizeof(int) * kSchedCap;
}
template <typename T>
size_t apply_lds() {
  constexpr int W = Win<T>::W;
  return sizeof(cx<T>) * ((size_t)(W + 1) * W + std::max<size_t>((size_t)(W + 1) * 32, 33 * (size_t)W));
}

template <typename T>
void launch_apply(hipStream_t st, int n, T* H, T* Z, int b0, int bl, const T* U) {
  const int gR = (int)ceil_div(n - b0 - bl, 32);
  const int gA = (int)ceil_div(b0, 32);
  const int gZ = (int)ceil_div(n, 32);
  const int g = gR + gA + gZ;
  if (g == 0) return;
  hipLaunchKernelGGL(apply_u_kernel<T>, dim3(g), dim3(kApplyThreads), apply_lds<T>(), st, n, H, Z, b0,
                     bl, U, gR, gA);
  MSQRT_LAUNCH_CHECK();
}

}  // namespace

template <typename T>
bool hseqr(hipStream_t st, int n, T* H, T* Z, HseqrWork& w, T hnorm) {
  constexpr int W = Win<T>::W, NS = Win<T>::NS;
  static bool attr_set = false;
  if (!attr_set) {
    MSQRT_HIP(hipFuncSetAttribute((const void*)small_schur_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)win_lds<T>()));
    MSQRT_HIP(hipFuncSetAttribute((const void*)chase_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)chase_lds<T>()));
    MSQRT_HIP(hipFuncSetAttribute((const void*)apply_u_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)apply_lds<T>()));
    attr_set = true;
  }
  if (n <= 0) return true;
  Sweep w_sweep;
  T* U = w.U.ensure<T>((int64_t)2 * W * W);
  cx<T>* shifts = w.shifts.ensure<cx<T>>(kMaxNs);
  int* flag = w.flag.ensure<int>(4);
  MSQRT_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, st));
  int hi = n - 1;
  int sweeps = 0, stuck = 0, last_hi = -1, last_lo = -1;
  const int max_sweeps = 30 * std::max(10, n / NS) + 100;
  while (hi >= 0) {
    int lo = 0;
    if (hi > 0) {
      hipLaunchKernelGGL(deflate_kernel<T>, dim3(1), dim3(1024), 0, st, n, H, 0, hi, flag + 1, hnorm);
      MSQRT_LAUNCH_CHECK();
      MSQRT_HIP(hipMemcpyAsync(&lo, flag + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      MSQRT_HIP(hipStreamSynchronize(st));
    }
    const int m = hi - lo + 1;
    if (m <= W) {
      if (m > 1) {
        hipLaunchKernelGGL(small_schur_kernel<T>, dim3(1), dim3(kQrThreads), win_lds<T>(), st, n, H,
                           lo, m, 0, U, shifts, flag, hnorm);
        MSQRT_LAUNCH_CHECK();
        launch_apply<T>(st, n, H, Z, lo, m, U);
      }
      hi = lo - 1;
      continue;
    }
    if (++sweeps > max_sweeps) return false;
    if (hi == last_hi && lo == last_lo) ++stuck;
    else stuck = 0;
    if (stuck > 300) return false;  // no deflation for 300 sweeps: give up early
    last_hi = hi;
    last_lo = lo;
    // shifts: eigenvalues of the trailing NS x NS block
    const int ns = NS;
    hipLaunchKernelGGL(small_schur_kernel<T>, dim3(1), dim3(kQrThreads), win_lds<T>(), st, n, H,
                       hi - ns + 1, ns, 1, U, shifts, flag, hnorm);
    MSQRT_LAUNCH_CHECK();
    if (stuck > 0 && stuck % 6 == 0) {
      // exceptional sweep: perturb the shifts by a multiple of the coupling
      std::vector<cx<T>> hs(ns);
      MSQRT_HIP(hipMemcpyAsync(hs.data(), shifts, sizeof(cx<T>) * ns, hipMemcpyDeviceToHost, st));
      T sub[2] = {0, 0};
      MSQRT_HIP(hipMemcpyAsync(&sub[0], H + hi + (int64_t)(hi - 1) * 2 * n, sizeof(T),
                               hipMemcpyDeviceToHost, st));
      MSQRT_HIP(hipMemcpyAsync(&sub[1], H + n + hi + (int64_t)(hi - 1) * 2 * n, sizeof(T),
                               hipMemcpyDeviceToHost, st));
      MSQRT_HIP(hipStreamSynchronize(st));
      const T e = T(0.75) * (std::fabs(sub[0]) + std::fabs(sub[1]));
      for (int j = 0; j < ns; ++j) hs[j].r += (j % 2 ? -e : e), hs[j].i += T(0.5) * e;
      MSQRT_HIP(hipMemcpyAsync(shifts, hs.data(), sizeof(cx<T>) * ns, hipMemcpyHostToDevice, st));
      MSQRT_HIP(hipStreamSynchronize(st));
    }
    Sweep& sw = w_sweep;
    build_sweep(lo, hi, ns, W, sw);
    // upload the sweep's rounds and moves (stream-ordered, from a host
    // staging copy that lives until the next synchronisation)
    const int nr = (int)sw.rnd.size(), nm = (int)sw.mv.size();
    int* dsched = w.scratch.ensure<int>(nr + nm + 64);
    MSQRT_HIP(hipMemcpyAsync(dsched, sw.rnd.data(), sizeof(int) * nr, hipMemcpyHostToDevice, st));
    MSQRT_HIP(hipMemcpyAsync(dsched + nr, sw.mv.data(), sizeof(int) * nm, hipMemcpyHostToDevice, st));
    for (size_t wi = 0; wi < sw.win.size(); wi += 4) {
      const int s = sw.win[wi], wl = sw.win[wi + 1], r0 = sw.win[wi + 2], nrw = sw.win[wi + 3];
      // launch the window's rounds in pieces whose schedule fits in LDS
      for (int ra = 0; ra < nrw;) {
        int rb = ra, used = 0;
        while (rb < nrw) {
          const int cnt = sw.rnd[2 * (r0 + rb) + 1];
          if (used + 2 + cnt > kSchedCap) break;
          used += 2 + cnt;
          ++rb;
        }
        if (rb == ra) throw Error{MSQRT_ERR_DEVICE, "Schur QR: round larger than the LDS schedule"};
        const int mv0 = sw.rnd[2 * (r0 + ra)];
        const int mv1 = sw.rnd[2 * (r0 + rb - 1)] + sw.rnd[2 * (r0 + rb - 1) + 1];
        hipLaunchKernelGGL(chase_kernel<T>, dim3(1), dim3(kChaseThreads), chase_lds<T>(), st, n, H, s, wl,
                           rb - ra, (const int*)(dsched + 2 * (r0 + ra)), (const int*)(dsched + nr),
                           mv0, mv1 - mv0, (const cx<T>*)shifts, U);
        MSQRT_LAUNCH_CHECK();
        launch_apply<T>(st, n, H, Z, s, wl, U);
        ra = rb;
      }
    }
    // the staging vectors are reused by the next sweep: wait for the copies
    MSQRT_HIP(hipStreamSynchronize(st));
  }
  int hflag = 0;
  MSQRT_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipStreamSynchronize(st));
  return hflag == 0;
}

template bool hseqr<float>(hipStream_t, int, float*, float*, HseqrWork&, float);
template bool hseqr<double>(hipStream_t, int, double*, double*, HseqrWork&, double);

}  // namespace msqrt
