// Divide-and-conquer eigensolver for a symmetric tridiagonal matrix
// (Cuppen's tearing, deflation, secular equation, Gu-Eisenstat eigenvectors).
//
// All scalar work (eigenvalues, secular roots, deflation) is float64 on the
// device; the eigenvector matrices and the merge products use the factor
// precision T on the MFMA GEMM.  Every merge of a level is processed by the
// same launches: one workgroup per merge for the deflation scan, one wave per
// secular root, one GEMM per merge for the eigenvector update.
//
// Merge of two solved halves (T1' = Q1 D1 Q1^T, T2' = Q2 D2 Q2^T) coupled by
// beta:  T = diag(Q1, Q2) (D + rho z z^T) diag(Q1, Q2)^T with
// z = [last row of Q1, sign(beta) first row of Q2] / sqrt(2), rho = 2|beta|.
// The merged eigenvectors are diag(Q1, Q2) (after the deflation rotations)
// times M, where M holds the normalised vectors z_i / (d_i - lambda_j) of the
// non-deflated secular problem and unit columns for deflated entries, both
// placed in ascending order of the merged eigenvalues.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"
#include "tridiag.hpp"

namespace msqrt {

namespace {

constexpr int kLeaf = 32;

struct MergeDesc {
  int s, n1, m;  // start, left size, total size
};

// A batch of tridiagonal matrices of order n is solved as one matrix of
// order batch * n whose off-diagonal vanishes at the entry boundaries: every
// position s of the concatenated index space belongs to entry s / n, and no
// leaf or merge straddles two entries.  The eigenvector matrices stay n x n
// per entry (stride n * n); this is the offset of the diagonal block that
// starts at position s.
__host__ __device__ inline int64_t blk_off(int s, int n) {
  const int e = s / n, sl = s - e * n;
  return (int64_t)e * n * n + sl + (int64_t)sl * n;
}

// Per-position metadata arrays (all length n, indexed by s + local index).
struct Meta {
  double* dl;      // non-deflated poles, ascending
  double* zl;      // their z components
  int* cl;         // their original local column
  double* defd;    // deflated eigenvalues, ascending
  int* defc;       // their original local column
  int* rota;       // rotation list: columns a, b
  int* rotb;
  double* rotc;
  double* rots;
  int* kcnt;       // per merge: k, number of deflated, number of rotations
  double* rho;     // per merge
  int* org;        // per root: origin pole index
  double* tau;     // per root: lambda - d_org
  double* lamr;    // per root: lambda
  double* zhat;    // per non-deflated index: recomputed z
  double* tmpd;    // scratch (sorted d), length n
  double* tmpz;    // scratch (sorted z)
  int* tmpc;       // scratch (sorted columns)
};

// ---------------------------------------------------------------------------
// Tearing: for every split point q, d[q-1] -= |e[q-1]| and d[q] -= |e[q-1]|.

__global__ void tear_kernel(int nsplit, const int* splits, double* d, const double* e) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsplit) return;
  const int q = splits[t];
  const double b = fabs(e[q - 1]);
  d[q - 1] -= b;
  d[q] -= b;
}

// ---------------------------------------------------------------------------
// Leaf eigensolver: implicit symmetric QR with Wilkinson shifts on a leaf of
// size L <= 32.  One wave per leaf; every lane runs the scalar recurrence
// redundantly (identical values) and lane r applies the rotations to row r of
// the eigenvector block.

template <typename T>
__global__ __launch_bounds__(64) void leaf_kernel(const int* leaf_start, const int* leaf_size,
                                                  const double* dg, const double* eg, double* lam,
                                                  T* Z, int n) {
  __shared__ double d[kLeaf], e[kLeaf], Zl[kLeaf][kLeaf + 1];
  const int lf = blockIdx.x, lane = threadIdx.x;
  const int s = leaf_start[lf], L = leaf_size[lf];
  if (lane < L) {
    d[lane] = dg[s + lane];
    e[lane] = (lane + 1 < L) ? eg[s + lane] : 0.0;
    for (int c = 0; c < L; ++c) Zl[lane][c] = (c == lane) ? 1.0 : 0.0;
  }
  __syncthreads();
  const double eps = 1.1102230246251565e-16;
  static_assert(kLeaf <= kWave, "one lane per off-diagonal entry of a leaf");
  int hi = L - 1, iters = 0;
  while (hi > 0 && iters < 60 * kLeaf) {
    // lo = 1 + the last negligible e[l] below hi (0 if none): every lane
    // tests its own entry and a ballot finds the last one
    const bool small = lane < hi && fabs(e[lane]) <= eps * (fabs(d[lane]) + fabs(d[lane + 1]));
    const unsigned long long sm = __ballot(small);
    const int lo = sm ? 64 - __clzll(sm) : 0;
    if (lo == hi) { --hi; continue; }
    ++iters;
    const double dd = (d[hi - 1] - d[hi]) * 0.5;
    const double b2 = e[hi - 1] * e[hi - 1];
    const double den = dd + copysign(sqrt(dd * dd + b2), dd);
    const double mu = (den == 0.0) ? d[hi] : d[hi] - b2 / den;
    double x = d[lo] - mu, z = e[lo];
    // d[k] and e[k] were written by the previous step and are carried in
    // registers; d[k+1] and e[k+1] are not touched before step k
    double cd = d[lo], ce = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double dk1 = d[k + 1];
      const double ek1 = (k + 1 < hi) ? e[k + 1] : 0.0;
      const double r = hypot(x, z);
      const double c = (r == 0.0) ? 1.0 : x / r;
      const double sn = (r == 0.0) ? 0.0 : z / r;
      const double dk = cd, ek = ce;
      const double ekm = (k > lo) ? r : 0.0;
      const double nd0 = c * c * dk + 2.0 * c * sn * ek + sn * sn * dk1;
      const double nd1 = sn * sn * dk - 2.0 * c * sn * ek + c * c * dk1;
      const double ne = c * sn * (dk1 - dk) + (c * c - sn * sn) * ek;
      double nx = 0.0, nz = 0.0, nek1 = 0.0;
      if (k + 1 < hi) {
        nx = ne;
        nz = sn * ek1;
        nek1 = c * ek1;
      }
      cd = nd1;
      ce = nek1;
      // Every lane computed the same scalars and writes them itself, so each
      // lane's later reads depend only on its own writes (no barrier).
      if (k > lo) e[k - 1] = ekm;
      d[k] = nd0;
      d[k + 1] = nd1;
      e[k] = ne;
      if (k + 1 < hi) e[k + 1] = nek1;
      if (lane < L) {
        const double qa = Zl[lane][k], qb = Zl[lane][k + 1];
        Zl[lane][k] = c * qa + sn * qb;
        Zl[lane][k + 1] = -sn * qa + c * qb;
      }
      x = nx;
      z = nz;
    }
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) e[hi - 1] = 0.0;
  }
  __syncthreads();
  // Ascending order: rank of eigenvalue c (ties by index).
  __shared__ int rank[kLeaf];
  if (lane < L) {
    int r = 0;
    for (int i = 0; i < L; ++i) r += (d[i] < d[lane]) || (d[i] == d[lane] && i < lane);
    rank[lane] = r;
  }
  __syncthreads();
  if (lane < L) {
    lam[s + rank[lane]] = d[lane];
    T* Zb = Z + blk_off(s, n);
    for (int c = 0; c < L; ++c) Zb[lane + (int64_t)rank[c] * n] = (T)Zl[lane][c];
  }
}

// ---------------------------------------------------------------------------
// Merge preparation: z vector, merge of the two sorted halves, deflation scan.
// One workgroup per merge.

template <typename T>
__global__ __launch_bounds__(256) void merge_prep_kernel(const MergeDesc* md, const double* eg,
                                                         const double* lam, const T* Z, int n,
                                                         Meta mt) {
  const MergeDesc g = md[blockIdx.x];
  const int s = g.s, n1 = g.n1, m = g.m, n2 = m - n1;
  const double beta = eg[s + n1 - 1];
  const double sgn = beta >= 0.0 ? 1.0 : -1.0;
  const double rho = 2.0 * fabs(beta);
  const double r2 = 0.7071067811865476;
  const T* Zg = Z + blk_off(s, n);
  __shared__ double red[4];
  // merge-path placement of the two ascending halves
  double dmax = 0.0, zmax = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    double di, zi;
    int pos;
    if (i < n1) {
      di = lam[s + i];
      zi = r2 * (double)Zg[(n1 - 1) + (int64_t)i * n];
      int lo = 0, hi = n2;  // count right values < di
      while (lo < hi) { const int mid = (lo + hi) / 2; if (lam[s + n1 + mid] < di) lo = mid + 1; else hi = mid; }
      pos = i + lo;
    } else {
      const int jr = i - n1;
      di = lam[s + i];
      zi = sgn * r2 * (double)Zg[n1 + (int64_t)i * n];
      int lo = 0, hi = n1;  // count left values <= di
      while (lo < hi) { const int mid = (lo + hi) / 2; if (lam[s + mid] <= di) lo = mid + 1; else hi = mid; }
      pos = jr + lo;
    }
    mt.tmpd[s + pos] = di;
    mt.tmpz[s + pos] = zi;
    mt.tmpc[s + pos] = i;
    dmax = fmax(dmax, fabs(di));
    zmax = fmax(zmax, fabs(zi));
  }
  dmax = block_max(dmax, red);
  zmax = block_max(zmax, red);
  __syncthreads();
  // Stage the sorted (d, z, column) triples in LDS for the sequential scan;
  // outputs go straight to global memory (stores only).
  extern __shared__ unsigned char lds_raw[];
  double* d = reinterpret_cast<double*>(lds_raw);
  double* z = d + m;
  int* c = reinterpret_cast<int*>(z + m);
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    d[i] = mt.tmpd[s + i];
    z[i] = mt.tmpz[s + i];
    c[i] = mt.tmpc[s + i];
  }
  __syncthreads();
  __shared__ int counts[3];
  const double eps = 1.1102230246251565e-16;
  const double tol = 8.0 * eps * fmax(dmax, zmax);
  // Rotation test of the scan below for a pair of consecutive survivors
  // (identical arithmetic, so the flags agree with it).
  auto rot_test = [&](double dp, double zp, double dj, double zj) {
    double sn = zp, cs = zj;
    const double tau = hypot(cs, sn);
    const double t = dj - dp;
    cs /= tau;
    sn = -sn / tau;
    return fabs(t * cs * sn) <= tol;
  };
  // Parallel pass: each thread takes a contiguous chunk, survivors of the
  // z-test and deflated entries are placed by block prefix sums, and every
  // pair of consecutive survivors is tested with its original values.  When
  // no pair calls for a rotation this is exactly the scan's result (kept
  // values in order, deflated values ascending); otherwise the sequential
  // scan below redoes the merge.
  __shared__ int scan_k[256], scan_d[256], scan_last[256];
  __shared__ int any_rot;
  const int nt = blockDim.x, tid = threadIdx.x;  // nt <= 256
  const int chunk = (m + nt - 1) / nt, c0 = min(m, tid * chunk), c1 = min(m, c0 + chunk);
  int nk = 0, ndf = 0, last = -1;
  for (int j = c0; j < c1; ++j) {
    if (rho * fabs(z[j]) <= tol) ++ndf;
    else { ++nk; last = j; }
  }
  scan_k[tid] = nk;
  scan_d[tid] = ndf;
  scan_last[tid] = last;
  if (tid == 0) any_rot = 0;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {  // inclusive scans (sum, max)
    const int a = tid >= off ? scan_k[tid - off] : 0, b = tid >= off ? scan_d[tid - off] : 0;
    const int l = tid >= off ? scan_last[tid - off] : -1;
    __syncthreads();
    scan_k[tid] += a;
    scan_d[tid] += b;
    scan_last[tid] = max(scan_last[tid], l);
    __syncthreads();
  }
  {
    int kpos = scan_k[tid] - nk, dpos = scan_d[tid] - ndf;
    int prev = tid > 0 ? scan_last[tid - 1] : -1;
    bool rot = false;
    for (int j = c0; j < c1; ++j) {
      if (rho * fabs(z[j]) <= tol) {
        mt.defd[s + dpos] = d[j];
        mt.defc[s + dpos] = c[j];
        ++dpos;
      } else {
        if (prev >= 0) rot = rot || rot_test(d[prev], z[prev], d[j], z[j]);
        mt.dl[s + kpos] = d[j];
        mt.zl[s + kpos] = z[j];
        mt.cl[s + kpos] = c[j];
        ++kpos;
        prev = j;
      }
    }
    if (rot) any_rot = 1;
  }
  __syncthreads();
  const bool need_scan = any_rot != 0;
  if (!need_scan && tid == 0) {
    counts[0] = scan_k[nt - 1]; counts[1] = scan_d[nt - 1]; counts[2] = 0;
    mt.kcnt[3 * blockIdx.x + 0] = scan_k[nt - 1];
    mt.kcnt[3 * blockIdx.x + 1] = scan_d[nt - 1];
    mt.kcnt[3 * blockIdx.x + 2] = 0;
    mt.rho[blockIdx.x] = rho;
  }
  if (need_scan && tid == 0) {
    int k = 0, nd = 0, nr = 0, pj = -1;
    double dp = 0.0, zp = 0.0;
    int cp = 0;
    for (int j = 0; j < m; ++j) {
      const double dj = d[j], zj = z[j];
      const int cj = c[j];
      if (rho * fabs(zj) <= tol) {
        mt.defd[s + nd] = dj;
        mt.defc[s + nd] = cj;
        ++nd;
        continue;
      }
      if (pj < 0) { pj = j; dp = dj; zp = zj; cp = cj; continue; }
      double sn = zp, cs = zj;
      const double tau = hypot(cs, sn);
      const double t = dj - dp;
      cs /= tau;
      sn = -sn / tau;
      if (fabs(t * cs * sn) <= tol) {
        // Rotate columns pj, j so that z[pj] vanishes; pj deflates.
        mt.rota[s + nr] = cp;
        mt.rotb[s + nr] = cj;
        mt.rotc[s + nr] = cs;
        mt.rots[s + nr] = sn;
        ++nr;
        const double tt = dp * cs * cs + dj * sn * sn;
        const double dnew = dp * sn * sn + dj * cs * cs;
        mt.defd[s + nd] = tt;
        mt.defc[s + nd] = cp;
        ++nd;
        pj = j; dp = dnew; zp = tau; cp = cj;
      } else {
        mt.dl[s + k] = dp;
        mt.zl[s + k] = zp;
        mt.cl[s + k] = cp;
        ++k;
        pj = j; dp = dj; zp = zj; cp = cj;
      }
    }
    if (pj >= 0) {
      mt.dl[s + k] = dp;
      mt.zl[s + k] = zp;
      mt.cl[s + k] = cp;
      ++k;
    }
    counts[0] = k; counts[1] = nd; counts[2] = nr;
    mt.kcnt[3 * blockIdx.x + 0] = k;
    mt.kcnt[3 * blockIdx.x + 1] = nd;
    mt.kcnt[3 * blockIdx.x + 2] = nr;
    mt.rho[blockIdx.x] = rho;
  }
  __syncthreads();
  // Deflated values in ascending order: rank sort in LDS (ties by index).
  // Without rotations they are already in order (d ascending).
  const int nd = counts[1];
  if (need_scan && nd > 1) {
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      d[i] = mt.defd[s + i];
      c[i] = mt.defc[s + i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      const double v = d[i];
      int r = 0;
      for (int q = 0; q < nd; ++q) r += (d[q] < v) || (d[q] == v && q < i);
      mt.defd[s + r] = v;
      mt.defc[s + r] = c[i];
    }
  }
}

// Deflation rotations on the rows of each merge block (one thread per row).
template <typename T>
__global__ void merge_rot_kernel(const MergeDesc* md, int nmerge_rows, const int* row_merge,
                                 Meta mt, T* Z, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nmerge_rows) return;
  const int b = row_merge[r];
  if (b < 0) return;
  const MergeDesc g = md[b];
  const int nr = mt.kcnt[3 * b + 2];
  T* Zr = Z + blk_off(g.s, n) + (r - g.s);  // row r of the merge block
  for (int q = 0; q < nr; ++q) {
    const int64_t ca = (int64_t)mt.rota[g.s + q] * n, cb = (int64_t)mt.rotb[g.s + q] * n;
    const double c = mt.rotc[g.s + q], sn = mt.rots[g.s + q];
    const double x = (double)Zr[ca], y = (double)Zr[cb];
    Zr[ca] = (T)(c * x + sn * y);
    Zr[cb] = (T)(c * y - sn * x);
  }
}

// ---------------------------------------------------------------------------
// Secular equation 1/rho + sum_i z_i^2 / (d_i - lambda) = 0, one wave per
// root j (root j lies in (d_j, d_{j+1}), the last one in (d_k, d_k + rho)).
// The root is represented as lambda = d_org + tau with org the nearer pole so
// that d_i - lambda = (d_i - d_org) - tau is computed to high relative
// accuracy.  Iteration: a two-pole rational model fitted to the value and the
// derivatives of the left and right partial sums (Gragg's scheme), solved as
// a quadratic, safeguarded by a bracket that is bisected whenever the model
// step leaves it.

__device__ inline void secular_eval(const double* dl, const double* zl, int k, int org, int j,
                                    double tau, int lane, double& psi, double& phi, double& dpsi,
                                    double& dphi) {
  psi = phi = dpsi = dphi = 0.0;
  const double dorg = dl[org];
  for (int i = lane; i < k; i += kWave) {
    const double del = (dl[i] - dorg) - tau;
    const double w = zl[i] / del;
    if (i <= j) { psi += zl[i] * w; dpsi += w * w; }
    else { phi += zl[i] * w; dphi += w * w; }
  }
  psi = wave_sum(psi);
  phi = wave_sum(phi);
  dpsi = wave_sum(dpsi);
  dphi = wave_sum(dphi);
}

__global__ __launch_bounds__(64) void secular_kernel(const MergeDesc* md, const int* pos_merge,
                                                     Meta mt, int n) {
  const int w = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = pos_merge[w];
  if (b < 0) return;
  const MergeDesc g = md[b];
  const int j = w - g.s;
  const int k = mt.kcnt[3 * b];
  if (j >= k) return;
  const double* dl = mt.dl + g.s;
  const double* zl = mt.zl + g.s;
  const double rho = mt.rho[b];
  const double eps = 1.1102230246251565e-16;
  int org;
  double lo, hi, tau;
  if (k == 1) {
    if (lane == 0) {
      mt.org[g.s + j] = 0;
      mt.tau[g.s + j] = rho * zl[0] * zl[0];
      mt.lamr[g.s + j] = dl[0] + rho * zl[0] * zl[0];
    }
    return;
  }
  if (j < k - 1) {
    const double gap = dl[j + 1] - dl[j];
    // f at the midpoint decides the nearer pole
    double psi, phi, dpsi, dphi;
    secular_eval(dl, zl, k, j, j, 0.5 * gap, lane, psi, phi, dpsi, dphi);
    const double fmid = 1.0 / rho + psi + phi;
    if (fmid >= 0.0) { org = j; lo = 0.0; hi = 0.5 * gap; }
    else { org = j + 1; lo = -0.5 * gap; hi = 0.0; }
  } else {
    org = k - 1;
    double zz = 0.0;
    for (int i = lane; i < k; i += kWave) zz += zl[i] * zl[i];
    zz = wave_sum(zz);
    lo = 0.0;
    hi = rho * zz * (1.0 + 4.0 * eps) + 1e-300;
  }
  tau = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double psi, phi, dpsi, dphi;
    secular_eval(dl, zl, k, org, j, tau, lane, psi, phi, dpsi, dphi);
    const double f = 1.0 / rho + psi + phi;
    if (f == 0.0) break;
    if (f < 0.0) lo = tau; else hi = tau;
    // convergence: |f| below the rounding level of its terms, or bracket tight
    const double erret = 8.0 * (phi - psi) + 2.0 / rho + fabs(tau) * (dpsi + dphi);
    if (fabs(f) <= eps * erret * 4.0) break;
    if (hi - lo <= 4.0 * eps * fmax(fabs(lo), fabs(hi))) break;
    // model poles relative to the current point
    const double dorg = dl[org];
    const double a0 = (dl[j] - dorg) - tau;  // < 0
    double step_tau;
    bool ok = false;
    if (j < k - 1) {
      const double b0 = (dl[j + 1] - dorg) - tau;  // > 0
      const double s1 = a0 * a0 * dpsi, s2 = b0 * b0 * dphi;
      const double c0 = f - a0 * dpsi - b0 * dphi;
      // c0 eta^2 - B eta + C = 0, eta in (a0, b0)
      const double B = c0 * (a0 + b0) + s1 + s2;
      const double C = c0 * a0 * b0 + s1 * b0 + s2 * a0;
      double eta = 0.0;
      if (c0 == 0.0) {
        if (B != 0.0) { eta = C / B; ok = true; }
      } else {
        const double disc = B * B - 4.0 * c0 * C;
        if (disc >= 0.0) {
          const double q = 0.5 * (B + copysign(sqrt(disc), B));
          const double e1 = q / c0, e2 = (q != 0.0) ? C / q : e1;
          if (e1 > a0 && e1 < b0) { eta = e1; ok = true; }
          else if (e2 > a0 && e2 < b0) { eta = e2; ok = true; }
        }
      }
      step_tau = tau + eta;
    } else {
      const double s1 = a0 * a0 * dpsi;
      const double c0 = f - a0 * dpsi;
      double eta = 0.0;
      if (c0 > 0.0) { eta = a0 + s1 / c0; ok = true; }
      step_tau = tau + eta;
    }
    if (!ok || !(step_tau > lo && step_tau < hi)) {
      // bisection (geometric when the bracket excludes zero)
      if (lo > 0.0 && hi > 0.0 && hi > 4.0 * lo) step_tau = sqrt(lo * hi);
      else if (lo < 0.0 && hi < 0.0 && lo < 4.0 * hi) step_tau = -sqrt(lo * hi);
      else step_tau = 0.5 * (lo + hi);
    }
    if (step_tau == tau) break;
    tau = step_tau;
  }
  if (lane == 0) {
    mt.org[g.s + j] = org;
    mt.tau[g.s + j] = tau;
    mt.lamr[g.s + j] = dl[org] + tau;
  }
}

// Gu-Eisenstat: z_i recomputed from the computed roots so that the computed
// eigenvectors are numerically orthogonal:
//   zhat_i^2 = (lambda_i - d_i)/rho * prod_{j != i} (lambda_j - d_i)/(d_j - d_i).
__global__ __launch_bounds__(64) void lowner_kernel(const MergeDesc* md, const int* pos_merge,
                                                    Meta mt, int n) {
  const int p = blockIdx.x, lane = threadIdx.x;
  const int b = pos_merge[p];
  if (b < 0) return;
  const MergeDesc g = md[b];
  const int i = p - g.s;
  const int k = mt.kcnt[3 * b];
  if (i >= k) return;
  const double* dl = mt.dl + g.s;
  const double di = dl[i];
  double prod = 1.0;
  for (int j = lane; j < k; j += kWave) {
    const double lj_di = (dl[mt.org[g.s + j]] - di) + mt.tau[g.s + j];
    prod *= (j == i) ? lj_di / mt.rho[b] : lj_di / (dl[j] - di);
  }
  // product over the wave
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) prod *= __shfl_xor(prod, off, kWave);
  if (lane == 0) {
    const double zh = sqrt(fmax(prod, 0.0));
    mt.zhat[g.s + i] = mt.zl[g.s + i] >= 0.0 ? zh : -zh;
  }
}

// Columns of M: secular eigenvectors (normalised) and unit vectors for the
// deflated entries, at the rank of their eigenvalue; new eigenvalue array.
template <typename T>
__global__ __launch_bounds__(64) void vectors_kernel(const MergeDesc* md, const int* pos_merge,
                                                     Meta mt, T* M, double* lam_new, int n) {
  const int w = blockIdx.x, lane = threadIdx.x;
  const int b = pos_merge[w];
  if (b < 0) return;
  const MergeDesc g = md[b];
  const int q = w - g.s;
  const int k = mt.kcnt[3 * b], nd = mt.kcnt[3 * b + 1];
  T* Mb = M + (int64_t)g.s * n;  // m x m, ld m
  const int m = g.m;
  if (q < k) {
    const int j = q;
    const double* dl = mt.dl + g.s;
    const double dorg = dl[mt.org[g.s + j]], tau = mt.tau[g.s + j];
    const double lj = mt.lamr[g.s + j];
    double nrm = 0.0;
    for (int i = lane; i < k; i += kWave) {
      const double v = mt.zhat[g.s + i] / ((dl[i] - dorg) - tau);
      nrm += v * v;
    }
    nrm = sqrt(wave_sum(nrm));
    // rank among deflated values (strictly smaller)
    int lo = 0, hi = nd;
    while (lo < hi) { const int mid = (lo + hi) / 2; if (mt.defd[g.s + mid] < lj) lo = mid + 1; else hi = mid; }
    const int col = j + lo;
    for (int i = lane; i < k; i += kWave) {
      const double v = mt.zhat[g.s + i] / ((dl[i] - dorg) - tau) / nrm;
      Mb[mt.cl[g.s + i] + (int64_t)col * m] = (T)v;
    }
    if (lane == 0) lam_new[g.s + col] = lj;
  } else if (q < k + nd) {
    const int t = q - k;
    const double v = mt.defd[g.s + t];
    int lo = 0, hi = k;  // roots <= v
    while (lo < hi) { const int mid = (lo + hi) / 2; if (mt.lamr[g.s + mid] <= v) lo = mid + 1; else hi = mid; }
    const int col = t + lo;
    if (lane == 0) {
      Mb[mt.defc[g.s + t] + (int64_t)col * m] = T(1);
      lam_new[g.s + col] = v;
    }
  }
}

// Concatenated float64 copies of the batch's diagonals; the coupling at the
// end of every entry is zero.
template <typename T>
__global__ void cast_tridiag(int n, const T* d, const T* e, int64_t sD, double* dd, double* ee) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i < n) {
    dd[(int64_t)b * n + i] = (double)d[b * sD + i];
    ee[(int64_t)b * n + i] = (i + 1 < n) ? (double)e[b * sD + i] : 0.0;
  }
}

// Copies the diagonal block [r0, r0+sz) of entry blockIdx.y of Za (and its
// eigenvalues) to Zb.
template <typename T>
__global__ void copy_block(int n, int r0, int sz, const T* Za, T* Zb, const double* la,
                           double* lb) {
  const int c = r0 + blockIdx.x;
  const int64_t zo = (int64_t)blockIdx.y * n * n;
  for (int i = threadIdx.x; i < sz; i += blockDim.x)
    Zb[zo + (int64_t)(r0 + i) + (int64_t)c * n] = Za[zo + (int64_t)(r0 + i) + (int64_t)c * n];
  if (threadIdx.x == 0) lb[(int64_t)blockIdx.y * n + c] = la[(int64_t)blockIdx.y * n + c];
}

template <typename T>
__global__ void copy_mat(int64_t cnt, const T* a, T* b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = a[i];
}

}  // namespace

template <typename T>
void stedc_batched(hipStream_t st, int n, int batch, const T* d, const T* e, int64_t sD,
                   double* lam, T* Z, StedcWork& w) {
  if (n <= 0 || batch <= 0) return;
  const int64_t nn = (int64_t)n * n;
  const int64_t N64 = (int64_t)n * batch;
  if (N64 > (int64_t)1 << 30 || nn * batch > ((int64_t)1 << 40))
    throw Error{MSQRT_ERR_UNSUPPORTED, "tridiagonal eigensolver: batch too large"};
  const int N = (int)N64;
  double* dd = w.dd.ensure<double>(N);
  double* ee = w.ee.ensure<double>(N);
  hipLaunchKernelGGL(cast_tridiag<T>, dim3((unsigned)ceil_div(n, 256), (unsigned)batch), dim3(256), 0,
                     st, n, d, e, sD, dd, ee);
  MSQRT_LAUNCH_CHECK();

  // Static recursion tree of one entry: halve until the pieces are at most
  // kLeaf.  Every entry has the same tree, shifted by a multiple of n.
  std::vector<std::vector<MergeDesc>> levels;  // levels[0] = leaves' parents ... top
  std::vector<std::pair<int, int>> cur{{0, n}};
  std::vector<std::vector<std::pair<int, int>>> tree{cur};
  while (true) {
    bool split = false;
    std::vector<std::pair<int, int>> nxt;
    for (auto& pr : tree.back()) {
      if (pr.second > kLeaf) {
        const int h = pr.second / 2;
        nxt.push_back({pr.first, h});
        nxt.push_back({pr.first + h, pr.second - h});
        split = true;
      } else {
        nxt.push_back(pr);
      }
    }
    if (!split) break;
    tree.push_back(nxt);
  }
  // leaves = tree.back(); merges: for level L from deepest-1 up to 0, every
  // node of tree[L] that was split.
  const auto& leaves = tree.back();
  std::vector<int> lst, lsz, splits;
  for (int b = 0; b < batch; ++b)
    for (auto& pr : leaves) { lst.push_back(b * n + pr.first); lsz.push_back(pr.second); }
  // Nodes of a tree level that are not split are already solved leaves; they
  // are carried unchanged through that level's merge step.
  std::vector<std::vector<std::pair<int, int>>> carried;
  for (size_t li = 0; li + 1 < tree.size(); ++li) {
    std::vector<MergeDesc> lv;
    std::vector<std::pair<int, int>> cv;
    for (auto& pr : tree[li]) {
      if (pr.second > kLeaf) {
        const int h = pr.second / 2;
        lv.push_back({pr.first, h, pr.second});
        for (int b = 0; b < batch; ++b) splits.push_back(b * n + pr.first + h);
      } else {
        cv.push_back(pr);
      }
    }
    levels.push_back(lv);
    carried.push_back(cv);
  }
  std::reverse(levels.begin(), levels.end());  // bottom-up
  std::reverse(carried.begin(), carried.end());

  // device metadata
  const int nl = (int)lst.size();
  int* dmeta = w.meta.ensure<int>(2 * (int64_t)nl + (int64_t)splits.size() + 4 * N64 + 8);
  int* dlst = dmeta;
  int* dlsz = dmeta + nl;
  int* dspl = dmeta + 2 * nl;
  int* pos_merge = dspl + splits.size();
  std::vector<int> hmeta(2 * nl + splits.size());
  std::copy(lst.begin(), lst.end(), hmeta.begin());
  std::copy(lsz.begin(), lsz.end(), hmeta.begin() + nl);
  std::copy(splits.begin(), splits.end(), hmeta.begin() + 2 * nl);
  MSQRT_HIP(hipMemcpyAsync(dmeta, hmeta.data(), sizeof(int) * hmeta.size(), hipMemcpyHostToDevice, st));
  if (!splits.empty()) {
    hipLaunchKernelGGL(tear_kernel, dim3((unsigned)ceil_div(splits.size(), 64)), dim3(64), 0, st,
                       (int)splits.size(), dspl, dd, ee);
    MSQRT_LAUNCH_CHECK();
  }
  T* Za = Z;
  T* Zb = w.Z2.ensure<T>(nn * batch);
  MSQRT_HIP(hipMemsetAsync(Za, 0, sizeof(T) * nn * batch, st));
  MSQRT_HIP(hipMemsetAsync(Zb, 0, sizeof(T) * nn * batch, st));
  double* lamA = lam;
  double* lamB = w.lam.ensure<double>(N);
  hipLaunchKernelGGL(leaf_kernel<T>, dim3(nl), dim3(64), 0, st, dlst, dlsz, dd, ee, lamA, Za, n);
  MSQRT_LAUNCH_CHECK();
  if (levels.empty()) return;

  // metadata buffers, indexed by concatenated position (per merge: by the
  // merge's index in its level, entry-major)
  Meta mt;
  double* fb = w.roots.ensure<double>((int64_t)12 * N + 16);
  int* ib = w.rot.ensure<int>((int64_t)10 * N + 16);
  mt.dl = fb; mt.zl = fb + N; mt.defd = fb + 2 * N; mt.rotc = fb + 3 * N; mt.rots = fb + 4 * N;
  mt.tau = fb + 5 * N; mt.lamr = fb + 6 * N; mt.zhat = fb + 7 * N; mt.tmpd = fb + 8 * N;
  mt.tmpz = fb + 9 * N; mt.rho = fb + 10 * N;
  mt.cl = ib; mt.defc = ib + N; mt.rota = ib + 2 * N; mt.rotb = ib + 3 * N; mt.org = ib + 4 * N;
  mt.tmpc = ib + 5 * N; mt.kcnt = ib + 6 * N;
  MergeDesc* dmd = (MergeDesc*)w.zhat.ensure<int>((int64_t)3 * N + 16);
  // M: the m x m secular eigenvector block of the merge at position s sits
  // at M + s * n (ld m)
  T* M = w.M.ensure<T>(nn * batch);

  static bool prep_attr[2] = {false, false};
  if (!prep_attr[sizeof(T) == 8]) {
    MSQRT_HIP(hipFuncSetAttribute((const void*)merge_prep_kernel<T>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024));
    prep_attr[sizeof(T) == 8] = true;
  }
  std::vector<int> posm(N);
  std::vector<MergeDesc> all;
  for (size_t L = 0; L < levels.size(); ++L) {
    const auto& lv = levels[L];
    const int nm1 = (int)lv.size();
    const int nm = nm1 * batch;
    all.clear();
    for (int b = 0; b < batch; ++b)
      for (auto g : lv) { g.s += b * n; all.push_back(g); }
    std::fill(posm.begin(), posm.end(), -1);
    for (int b = 0; b < nm; ++b)
      for (int i = 0; i < all[b].m; ++i) posm[all[b].s + i] = b;
    MSQRT_HIP(hipMemcpyAsync(dmd, all.data(), sizeof(MergeDesc) * nm, hipMemcpyHostToDevice, st));
    MSQRT_HIP(hipMemcpyAsync(pos_merge, posm.data(), sizeof(int) * N, hipMemcpyHostToDevice, st));
    int mmax = 0;
    for (auto& g : lv) mmax = std::max(mmax, g.m);
    const size_t prep_lds = (size_t)mmax * (2 * sizeof(double) + sizeof(int));
    if (prep_lds > 140 * 1024) throw Error{MSQRT_ERR_UNSUPPORTED, "tridiagonal eigensolver supports n <= 7000"};
    hipLaunchKernelGGL(merge_prep_kernel<T>, dim3(nm), dim3(256), prep_lds, st, dmd, ee, lamA, Za, n, mt);
    MSQRT_LAUNCH_CHECK();
    hipLaunchKernelGGL(merge_rot_kernel<T>, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, st, dmd, N,
                       pos_merge, mt, Za, n);
    MSQRT_LAUNCH_CHECK();
    hipLaunchKernelGGL(secular_kernel, dim3(N), dim3(64), 0, st, dmd, pos_merge, mt, n);
    MSQRT_LAUNCH_CHECK();
    hipLaunchKernelGGL(lowner_kernel, dim3(N), dim3(64), 0, st, dmd, pos_merge, mt, n);
    MSQRT_LAUNCH_CHECK();
    MSQRT_HIP(hipMemsetAsync(M, 0, sizeof(T) * nn * batch, st));
    hipLaunchKernelGGL(vectors_kernel<T>, dim3(N), dim3(64), 0, st, dmd, pos_merge, mt, M, lamB, n);
    MSQRT_LAUNCH_CHECK();
    // C = A M for each merge, A the merge's m x m block of eigenvectors, M its
    // secular block.  Before the deflation rotations A = diag(Z1, Z2); a
    // level whose merges rotated no pair of columns keeps that structure, and
    // the product splits into Z1 M(0:n1, :) and Z2 M(n1:m, :) (half the
    // flops).  For a single matrix the rotation counts come to the host once
    // per level; after a rotation the level forms the full products.  (A
    // batch nearly always has a rotation in some entry at every level, so it
    // skips the read and its host synchronisation: for 64 x n = 512 the
    // eigensolver measured 2.49 ms without the read and 2.67 ms with it.)
    bool halves = false;
    if (batch == 1) {
      std::vector<int> kc(3 * (size_t)nm);
      MSQRT_HIP(hipMemcpyAsync(kc.data(), mt.kcnt, sizeof(int) * kc.size(), hipMemcpyDeviceToHost, st));
      MSQRT_HIP(hipStreamSynchronize(st));
      halves = true;
      for (int b = 0; b < nm && halves; ++b) halves = kc[3 * b + 2] == 0;
    }
    auto gemm = [&](int Mr, int Nc, int Kk, const T* A_, int64_t sA_, const T* B_, int ldb_, int64_t sB_,
                    T* C_, int64_t sC_, int nb_) {
      if (std::is_same<T, float>::value)
        gemm_store_f32(st, false, false, Mr, Nc, Kk, (const float*)A_, n, sA_, (const float*)B_, ldb_, sB_,
                       (float*)C_, n, sC_, 1.f, 0.f, nb_, false);
      else
        gemm_store_f64(st, false, false, Mr, Nc, Kk, (const double*)A_, n, sA_, (const double*)B_, ldb_,
                       sB_, (double*)C_, n, sC_, 1.0, 0.0, nb_, false);
    };
    auto merge_product = [&](const MergeDesc& g, const T* Ablk, int64_t sA_, const T* Mb, int64_t sM_,
                             T* Cblk, int64_t sC_, int nb_) {
      if (halves) {
        const int n1 = g.n1, n2 = g.m - g.n1;
        if (n1 > 0) gemm(n1, g.m, n1, Ablk, sA_, Mb, g.m, sM_, Cblk, sC_, nb_);
        if (n2 > 0)
          gemm(n2, g.m, n2, Ablk + blk_off(n1, n), sA_, Mb + n1, g.m, sM_, Cblk + n1, sC_, nb_);
      } else {
        gemm(g.m, g.m, g.m, Ablk, sA_, Mb, g.m, sM_, Cblk, sC_, nb_);
      }
    };
    // One product per merge of the level, batched over the entries; a single
    // entry whose merges are equal and adjacent (n a power of two times the
    // leaf size) takes the whole level as one batch instead.
    bool uniform = batch == 1 && nm1 > 1;
    for (int b = 1; b < nm1 && uniform; ++b)
      uniform = lv[b].m == lv[0].m && lv[b].n1 == lv[0].n1 && lv[b].s == lv[0].s + b * lv[0].m;
    if (uniform) {
      const MergeDesc& g = lv[0];
      const int64_t sBlk = (int64_t)g.m * (n + 1), sM = (int64_t)g.m * n;
      merge_product(g, Za + blk_off(g.s, n), sBlk, M + (int64_t)g.s * n, sM, Zb + blk_off(g.s, n), sBlk, nm1);
    }
    for (int b = 0; b < nm1 && !uniform; ++b) {
      const MergeDesc& g = lv[b];
      merge_product(g, Za + blk_off(g.s, n), nn, M + (int64_t)g.s * n, nn, Zb + blk_off(g.s, n), nn, batch);
    }
    for (auto& pr : carried[L]) {
      hipLaunchKernelGGL(copy_block<T>, dim3((unsigned)pr.second, (unsigned)batch), dim3(64), 0, st, n,
                         pr.first, pr.second, (const T*)Za, Zb, (const double*)lamA, lamB);
      MSQRT_LAUNCH_CHECK();
    }
    std::swap(Za, Zb);
    std::swap(lamA, lamB);
  }
  if (Za != Z) {
    const int64_t cnt = nn * batch;
    hipLaunchKernelGGL(copy_mat<T>, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, cnt,
                       (const T*)Za, Z);
    MSQRT_LAUNCH_CHECK();
  }
  if (lamA != lam) MSQRT_HIP(hipMemcpyAsync(lam, lamA, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
}

template <typename T>
void stedc(hipStream_t st, int n, const T* d, const T* e, double* lam, T* Z, StedcWork& w) {
  stedc_batched<T>(st, n, 1, d, e, 0, lam, Z, w);
}

template void stedc<float>(hipStream_t, int, const float*, const float*, double*, float*, StedcWork&);
template void stedc<double>(hipStream_t, int, const double*, const double*, double*, double*, StedcWork&);
template void stedc_batched<float>(hipStream_t, int, int, const float*, const float*, int64_t, double*,
                                   float*, StedcWork&);
template void stedc_batched<double>(hipStream_t, int, int, const double*, const double*, int64_t,
                                    double*, double*, StedcWork&);

}  // namespace msqrt
