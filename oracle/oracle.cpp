// Plain CPU oracle for the principal matrix square root and the linear solves
// that the mixed-precision method (Gao, Kressner, Shao) is built from.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code with
// the HIP path: no headers, kernels, tables or helpers.
//
// Everything here is unblocked, textbook and slow on purpose, so that a reader
// can check it against the paper by eye:
//   * complex Schur form by Householder Hessenberg reduction followed by the
//     implicit single-shift complex QR iteration (Wilkinson shift, Givens
//     rotations, accumulated unitary factor) -- the decomposition A = Q T Q^H
//     that the paper's Schur algorithm starts from (Sec. 1, Sec. 2.1);
//   * the column recurrence for the square root of an upper triangular matrix
//     (Eq. (subst), Sec. 2.2.1);
//   * the symmetric spectral decomposition by Householder tridiagonalisation
//     and implicit symmetric QR with Wilkinson shifts, the factorisation that
//     the SPD algorithm (Alg. 3) starts from;
//   * the triangular Sylvester equation S Y + Y St = C by plain
//     back-substitution (Bartels-Stewart on triangular factors, Sec. 2.2.2) and
//     the block recursion of Alg. 1 on top of it;
//   * the adjoint solve X^H G + G X^H = Gbar used for differentiation.
//
// All routines are templated on the real type so that the mixed-precision
// emulator can run the *same* textbook factorisation in single precision.
// Loops over independent entries run on OpenMP threads, and the QR sweeps
// apply their rotations lazily where the chase does not read them (see
// g_deferred); neither changes any entry's arithmetic, so every result is
// bitwise that of the plain serial loops, which stay selectable.
// Matrices are column-major: element (i,j) of an n-by-n matrix is a[i + j*n].

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include <omp.h>

namespace orc {

template <class R> using C = std::complex<R>;

// Execution mode.  Every loop that OpenMP splits below runs over independent
// elements (rows, columns or entries of one superdiagonal), and each element
// receives exactly the same floating-point operations in the same order as in
// a serial run, so the results do not depend on the thread count.  With
// g_deferred set, the plane rotations of the QR iterations are applied at
// once only to the entries that the iteration itself reads; the others (the
// rows of Q, and the parts of H outside the active block) are logged and
// applied later, in log order, row block by row block.  Each entry still sees
// the same rotations in the same order, so the result is bitwise that of the
// immediate application (g_deferred = 0), which is kept for that comparison.
static int g_deferred = 1;

// Rows (or columns) per OpenMP work item in the blocked loops.
constexpr int kChunk = 32;

// ---------------------------------------------------------------------------
// Principal complex square root by the half-angle formula.  For z = x + i y
// with |z| = r:  t = sqrt((|x| + r)/2);  x >= 0 -> (t, y/(2t)),
// x < 0 -> (|y|/(2t), sign(y) t).  The result has non-negative real part; the
// branch cut is the non-positive real axis, matching the definition of the
// principal root in Sec. 1.
template <class R> C<R> csqrt_principal(C<R> z) {
  R x = z.real(), y = z.imag();
  if (x == R(0) && y == R(0)) return C<R>(0, 0);
  R r = std::hypot(x, y);
  R t = std::sqrt((std::fabs(x) + r) / R(2));
  if (x >= R(0)) return C<R>(t, y / (R(2) * t));
  return C<R>(std::fabs(y) / (R(2) * t), (y >= R(0) ? t : -t));
}

// ---------------------------------------------------------------------------
// Complex Householder reflector P = I - 2 u u^H / (u^H u) that maps x (length
// len) onto a multiple of e_1.  u = x + e^{i arg x_0} ||x|| e_1.  Returns false
// when x is already zero below its first entry (no reflection needed).
template <class R>
bool householder(int len, const C<R>* x, C<R>* u, R* unorm2) {
  R nx2 = 0;
  for (int i = 0; i < len; ++i) nx2 += std::norm(x[i]);
  R tail = nx2 - std::norm(x[0]);
  if (tail <= R(0)) return false;
  R nx = std::sqrt(nx2);
  R a0 = std::abs(x[0]);
  C<R> phase = a0 > R(0) ? x[0] / a0 : C<R>(1, 0);
  for (int i = 0; i < len; ++i) u[i] = x[i];
  u[0] += phase * nx;
  R s = 0;
  for (int i = 0; i < len; ++i) s += std::norm(u[i]);
  *unorm2 = s;
  return true;
}

// Hessenberg reduction A <- P^H A P with Q accumulating the reflectors, so
// that on exit A_in = Q H Q^H.
template <class R> void hessenberg(int n, C<R>* a, C<R>* q) {
  std::vector<C<R>> u(n), x(n), r(n);
  for (int k = 0; k + 2 < n; ++k) {
    int len = n - k - 1;
    for (int i = 0; i < len; ++i) x[i] = a[(k + 1 + i) + (size_t)k * n];
    R un2;
    if (!householder<R>(len, x.data(), u.data(), &un2)) continue;
    R f = R(2) / un2;
    // Left: rows k+1..n-1, all columns.  A <- (I - f u u^H) A (columns are
    // independent).
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
      C<R> s = 0;
      for (int i = 0; i < len; ++i) s += std::conj(u[i]) * a[(k + 1 + i) + (size_t)j * n];
      s *= f;
      for (int i = 0; i < len; ++i) a[(k + 1 + i) + (size_t)j * n] -= u[i] * s;
    }
    // Right: columns k+1..n-1, all rows.  A <- A (I - f u u^H), and the
    // same for Q.  r = M u is formed column by column (rows independent),
    // then M -= f r u^H (columns independent).
    for (C<R>* m : {a, q}) {
#pragma omp parallel for schedule(static)
      for (int i0 = 0; i0 < n; i0 += kChunk) {
        const int i1 = std::min(n, i0 + kChunk);
        for (int i = i0; i < i1; ++i) r[i] = C<R>(0, 0);
        for (int jj = 0; jj < len; ++jj)
          for (int i = i0; i < i1; ++i) r[i] += m[i + (size_t)(k + 1 + jj) * n] * u[jj];
      }
#pragma omp parallel for schedule(static)
      for (int jj = 0; jj < len; ++jj) {
        C<R> cu = f * std::conj(u[jj]);
        for (int i = 0; i < n; ++i) m[i + (size_t)(k + 1 + jj) * n] -= r[i] * cu;
      }
    }
    for (int i = k + 2; i < n; ++i) a[i + (size_t)k * n] = 0;
  }
}

// Givens rotation G = [[c, s], [-conj(s), c]] (c real) with G [a; b] = [r; 0].
template <class R> void givens(C<R> a, C<R> b, R* c, C<R>* s) {
  R aa = std::abs(a), bb = std::abs(b);
  if (bb == R(0)) { *c = 1; *s = 0; return; }
  if (aa == R(0)) { *c = 0; *s = 1; return; }
  R rho = std::hypot(aa, bb);
  *c = aa / rho;
  *s = (a / aa) * std::conj(b) / rho;
}

// Similarity with G acting on indices (p, p+1): H <- G H G^H restricted to the
// columns/rows that can be non-zero, Q <- Q G^H.  The three parts: rows p, p+1
// of H for columns j0..j1-1; columns p, p+1 of H for rows i0..i1-1; columns p,
// p+1 of Q for all rows.
template <class R>
inline void rot_rows(int n, C<R>* h, int p, R c, C<R> s, int j0, int j1) {
  for (int j = j0; j < j1; ++j) {
    C<R> x = h[p + (size_t)j * n], y = h[p + 1 + (size_t)j * n];
    h[p + (size_t)j * n] = c * x + s * y;
    h[p + 1 + (size_t)j * n] = -std::conj(s) * x + c * y;
  }
}
template <class R>
inline void rot_cols(int n, C<R>* m, int p, R c, C<R> s, int i0, int i1) {
  for (int i = i0; i < i1; ++i) {
    C<R> x = m[i + (size_t)p * n], y = m[i + (size_t)(p + 1) * n];
    m[i + (size_t)p * n] = x * c + y * std::conj(s);
    m[i + (size_t)(p + 1) * n] = -x * s + y * c;
  }
}

// One logged rotation of a QR sweep on the active block [lo, hi].
template <class R> struct RotLog {
  int p, lo, hi;
  R c;
  C<R> s;
};

// Applies the logged rotations, in log order, to the entries the sweep left
// out: rows p, p+1 of H right of the active block (columns > hi), columns p,
// p+1 of H above it (rows < lo) and columns p, p+1 of Q (all rows).  Entries
// are independent, so row (column) blocks run in parallel.
template <class R>
void flush_rotations(int n, C<R>* h, C<R>* q, std::vector<RotLog<R>>& log) {
  if (log.empty()) return;
  const int nl = (int)log.size();
  const int nb = (n + kChunk - 1) / kChunk;
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < 3 * nb; ++b) {
    const int part = b / nb;
    const int x0 = (b % nb) * kChunk, x1 = std::min(n, x0 + kChunk);
    if (part == 0) {  // rows x0..x1-1 of Q
      for (int t = 0; t < nl; ++t) rot_cols<R>(n, q, log[t].p, log[t].c, log[t].s, x0, x1);
    } else if (part == 1) {  // rows x0..x1-1 of H above the active block
      for (int t = 0; t < nl; ++t)
        rot_cols<R>(n, h, log[t].p, log[t].c, log[t].s, x0, std::min(x1, log[t].lo));
    } else {  // columns x0..x1-1 of H right of the active block
      for (int t = 0; t < nl; ++t)
        rot_rows<R>(n, h, log[t].p, log[t].c, log[t].s, std::max(x0, log[t].hi + 1), x1);
    }
  }
  log.clear();
}

// Complex Schur decomposition.  On entry a holds A; on exit a holds the upper
// triangular T and q the unitary Q with A = Q T Q^H.  Returns 0 on success,
// 1 if the QR iteration failed to converge within 30 n iterations.
template <class R> int schur(int n, C<R>* a, C<R>* q) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) q[i + (size_t)j * n] = (i == j) ? C<R>(1, 0) : C<R>(0, 0);
  if (n <= 1) return 0;
  hessenberg<R>(n, a, q);
  const R eps = std::numeric_limits<R>::epsilon() / 2;
  auto H = [&](int i, int j) -> C<R>& { return a[i + (size_t)j * n]; };
  std::vector<RotLog<R>> log;
  const size_t log_cap = (size_t)1 << 20;
  std::vector<R> rc(n);
  std::vector<C<R>> rs(n);
  std::vector<int> next_row(n);
  int hi = n - 1, iter = 0, total = 0, st = 0;
  while (hi > 0) {
    // Find the start of the active unreduced block by scanning for negligible
    // subdiagonal entries.
    int lo = hi;
    while (lo > 0) {
      R scale = std::abs(H(lo, lo)) + std::abs(H(lo - 1, lo - 1));
      if (scale == R(0)) scale = 1;
      if (std::abs(H(lo, lo - 1)) <= eps * scale) { H(lo, lo - 1) = 0; break; }
      --lo;
    }
    if (lo == hi) { --hi; iter = 0; continue; }
    if (++total > 30 * n) { st = 1; break; }
    ++iter;
    // Wilkinson shift: eigenvalue of the trailing 2x2 block closest to H(hi,hi).
    C<R> mu;
    if (iter % 10 == 0) {
      // Exceptional shift after 10 iterations without deflation.
      mu = H(hi, hi) + C<R>(R(0.75) * std::abs(H(hi, hi - 1)), 0);
    } else {
      C<R> a11 = H(hi - 1, hi - 1), a12 = H(hi - 1, hi), a21 = H(hi, hi - 1), a22 = H(hi, hi);
      C<R> tr = a11 + a22, det = a11 * a22 - a12 * a21;
      C<R> disc = std::sqrt(tr * tr / R(4) - det);
      C<R> l1 = tr / R(2) + disc, l2 = tr / R(2) - disc;
      mu = (std::abs(l1 - a22) < std::abs(l2 - a22)) ? l1 : l2;
    }
    // Implicit single-shift sweep over the active block [lo, hi]: each
    // rotation acts on rows k, k+1 from column col_lo on and on columns k, k+1
    // down to row row_hi (the only entries that can be non-zero), and on Q.
    C<R> x = H(lo, lo) - mu, y = H(lo + 1, lo);
    if (!g_deferred) {
      for (int k = lo; k < hi; ++k) {
        R c; C<R> s;
        givens<R>(x, y, &c, &s);
        int col_lo = (k > lo) ? k - 1 : lo;
        int row_hi = std::min(k + 2, hi);
        rot_rows<R>(n, a, k, c, s, col_lo, n);
        rot_cols<R>(n, a, k, c, s, 0, row_hi + 1);
        rot_cols<R>(n, q, k, c, s, 0, n);
        if (k > lo) H(k + 1, k - 1) = 0;
        if (k + 1 < hi) { x = H(k + 1, k); y = H(k + 2, k); }
      }
    } else {
      // The same sweep, with every rotation applied at once only where the
      // chase reads it next, and the rest later in an order that gives every
      // entry the same operations in the same sequence:
      //  * rows: column j of the block receives row rotations lo..j+1; it is
      //    brought up to date (in rotation order, down the column) just before
      //    a column rotation or the chase reads it, and every kLook rotations
      //    all columns right of the bulge are brought up to date in parallel;
      //  * columns: rotation k is applied at once to rows k-1..k+2; rows
      //    lo..k-2 (all of whose row rotations come earlier) are rotated after
      //    the sweep, row blocks in parallel;
      //  * entries above the block (rows < lo), right of it (columns > hi) and
      //    all of Q go to the log.  Within one log lo is fixed, so those two
      //    parts never share an entry; an entry above an earlier block can lie
      //    right of a later one, so the log is applied before lo changes.
      if (!log.empty() && log.back().lo != lo) flush_rotations<R>(n, a, q, log);
      for (int j = lo; j <= hi; ++j) next_row[j] = lo;
      auto catch_up = [&](int j, int kmax) {
        const int kend = std::min(kmax, j + 1);
        for (int k = next_row[j]; k <= kend; ++k) {
          C<R> u = H(k, j), v = H(k + 1, j);
          H(k, j) = rc[k] * u + rs[k] * v;
          H(k + 1, j) = -std::conj(rs[k]) * u + rc[k] * v;
        }
        if (kend + 1 > next_row[j]) next_row[j] = kend + 1;
      };
      constexpr int kLook = 64;
      for (int k = lo; k < hi; ++k) {
        R c; C<R> s;
        givens<R>(x, y, &c, &s);
        rc[k] = c;
        rs[k] = s;
        if (k > lo) catch_up(k - 1, k);
        catch_up(k, k);
        catch_up(k + 1, k);
        rot_cols<R>(n, a, k, c, s, std::max(lo, k - 1), std::min(k + 2, hi) + 1);
        log.push_back({k, lo, hi, c, s});
        if (k > lo) H(k + 1, k - 1) = 0;
        if (k + 1 < hi) { x = H(k + 1, k); y = H(k + 2, k); }
        if ((k - lo) % kLook == kLook - 1) {
#pragma omp parallel for schedule(static)
          for (int j = k + 2; j <= hi; ++j) catch_up(j, k);
        }
      }
#pragma omp parallel for schedule(static)
      for (int j = lo; j <= hi; ++j) catch_up(j, hi - 1);
      const int nb = (hi - lo + 1 + kChunk - 1) / kChunk;
#pragma omp parallel for schedule(dynamic)
      for (int b = 0; b < nb; ++b) {
        const int i0 = lo + b * kChunk, i1 = std::min(hi + 1, i0 + kChunk);
        for (int k = std::max(lo, i0 + 2); k < hi; ++k)
          rot_cols<R>(n, a, k, rc[k], rs[k], i0, std::min(i1, k - 1));
      }
    }
    if (log.size() >= log_cap) flush_rotations<R>(n, a, q, log);
  }
  flush_rotations<R>(n, a, q, log);
  if (st) return st;
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) a[i + (size_t)j * n] = 0;
  return 0;
}

// Square root of an upper triangular matrix by the column recurrence
// (Eq. (subst)): s_ii = t_ii^{1/2}; for j = 2..n and i = j-1 down to 1,
// s_ij = (t_ij - sum_{k=i+1}^{j-1} s_ik s_kj) / (s_ii + s_jj).
// Returns 2 if a diagonal entry lies on the closed negative real axis.
template <class R> int trsqrt(int n, const C<R>* t, C<R>* s) {
  for (size_t k = 0; k < (size_t)n * n; ++k) s[k] = 0;
  for (int i = 0; i < n; ++i) {
    C<R> d = t[i + (size_t)i * n];
    if (d.imag() == R(0) && d.real() <= R(0)) return 2;
    s[i + (size_t)i * n] = csqrt_principal<R>(d);
  }
  auto entry = [&](int i, int j) {
    C<R> acc = t[i + (size_t)j * n];
    for (int k = i + 1; k <= j - 1; ++k) acc -= s[i + (size_t)k * n] * s[k + (size_t)j * n];
    s[i + (size_t)j * n] = acc / (s[i + (size_t)i * n] + s[j + (size_t)j * n]);
  };
  if (!g_deferred) {
    for (int j = 1; j < n; ++j)
      for (int i = j - 1; i >= 0; --i) entry(i, j);
    return 0;
  }
  // s_ij reads only entries of lower superdiagonals (s_ik and s_kj with
  // i < k < j), so the entries of one superdiagonal are independent.
  for (int d = 1; d < n; ++d) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n - d; ++i) entry(i, i + d);
  }
  return 0;
}

// C = A * B (n x n, complex), plain triple loop.
// Columns of C are independent.
template <class R> void cgemm(int n, const C<R>* a, const C<R>* b, C<R>* c) {
  for (size_t k = 0; k < (size_t)n * n; ++k) c[k] = 0;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      C<R> bkj = b[k + (size_t)j * n];
      for (int i = 0; i < n; ++i) c[i + (size_t)j * n] += a[i + (size_t)k * n] * bkj;
    }
}

// Triangular Sylvester equation S Y + Y St = Cm with S (m x m) and St (n x n)
// upper triangular, solved by back-substitution: columns left to right, rows
// bottom to top,
//   y_ij = (c_ij - sum_{k>i} s_ik y_kj - sum_{k<j} y_ik st_kj) / (s_ii + st_jj).
// Leading dimensions ldS, ldT, ldC, ldY allow operating on sub-blocks.
template <class R>
void trsyl(int m, int n, const C<R>* S, int ldS, const C<R>* St, int ldT, const C<R>* Cm,
           int ldC, C<R>* Y, int ldY) {
  for (int j = 0; j < n; ++j) {
    for (int i = m - 1; i >= 0; --i) {
      C<R> acc = Cm[i + (size_t)j * ldC];
      for (int k = i + 1; k < m; ++k) acc -= S[i + (size_t)k * ldS] * Y[k + (size_t)j * ldY];
      for (int k = 0; k < j; ++k) acc -= Y[i + (size_t)k * ldY] * St[k + (size_t)j * ldT];
      Y[i + (size_t)j * ldY] = acc / (S[i + (size_t)i * ldS] + St[j + (size_t)j * ldT]);
    }
  }
}

// Cm(mxn) -= A(mxk) * B(kxn) for sub-blocks with leading dimensions.
template <class R>
void sub_gemm(int m, int n, int k, const C<R>* A, int lda, const C<R>* B, int ldb, C<R>* Cm,
              int ldc) {
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < k; ++l) {
      C<R> b = B[l + (size_t)j * ldb];
      for (int i = 0; i < m; ++i) Cm[i + (size_t)j * ldc] -= A[i + (size_t)l * lda] * b;
    }
}

// Block recursion of Alg. 1: solves S Y + Y St = Cm, overwriting Cm with Y.
// The split point of a dimension m is floor(m/2); "n <= m/2" and "m <= n/2"
// are tested as 2n <= m and 2m <= n.
template <class R>
void rtrsyl(int m, int n, const C<R>* S, int ldS, const C<R>* St, int ldT, C<R>* Cm, int ldC,
            int blks) {
  if (m <= 0 || n <= 0) return;
  if (m <= blks && n <= blks) {
    std::vector<C<R>> y((size_t)m * n);
    trsyl<R>(m, n, S, ldS, St, ldT, Cm, ldC, y.data(), m);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < m; ++i) Cm[i + (size_t)j * ldC] = y[i + (size_t)j * m];
    return;
  }
  if (2 * n <= m) {
    // Split rows only: S = [S11 S12; 0 S22], Cm = [C1; C2].
    int m1 = m / 2, m2 = m - m1;
    const C<R>* S11 = S;
    const C<R>* S12 = S + (size_t)m1 * ldS;
    const C<R>* S22 = S + m1 + (size_t)m1 * ldS;
    C<R>* C1 = Cm;
    C<R>* C2 = Cm + m1;
    rtrsyl<R>(m2, n, S22, ldS, St, ldT, C2, ldC, blks);
    sub_gemm<R>(m1, n, m2, S12, ldS, C2, ldC, C1, ldC);
    rtrsyl<R>(m1, n, S11, ldS, St, ldT, C1, ldC, blks);
    return;
  }
  if (2 * m <= n) {
    // Split columns only: St = [St11 St12; 0 St22], Cm = [C1 C2].
    int n1 = n / 2, n2 = n - n1;
    const C<R>* T11 = St;
    const C<R>* T12 = St + (size_t)n1 * ldT;
    const C<R>* T22 = St + n1 + (size_t)n1 * ldT;
    C<R>* C1 = Cm;
    C<R>* C2 = Cm + (size_t)n1 * ldC;
    rtrsyl<R>(m, n1, S, ldS, T11, ldT, C1, ldC, blks);
    // C2 -= Y1 * St12
    sub_gemm<R>(m, n2, n1, C1, ldC, T12, ldT, C2, ldC);
    rtrsyl<R>(m, n2, S, ldS, T22, ldT, C2, ldC, blks);
    return;
  }
  int m1 = m / 2, m2 = m - m1, n1 = n / 2, n2 = n - n1;
  const C<R>* S11 = S;
  const C<R>* S12 = S + (size_t)m1 * ldS;
  const C<R>* S22 = S + m1 + (size_t)m1 * ldS;
  const C<R>* T11 = St;
  const C<R>* T12 = St + (size_t)n1 * ldT;
  const C<R>* T22 = St + n1 + (size_t)n1 * ldT;
  C<R>* C11 = Cm;
  C<R>* C21 = Cm + m1;
  C<R>* C12 = Cm + (size_t)n1 * ldC;
  C<R>* C22 = Cm + m1 + (size_t)n1 * ldC;
  rtrsyl<R>(m2, n1, S22, ldS, T11, ldT, C21, ldC, blks);             // Y21
  sub_gemm<R>(m1, n1, m2, S12, ldS, C21, ldC, C11, ldC);              // C11 -= S12 Y21
  sub_gemm<R>(m2, n2, n1, C21, ldC, T12, ldT, C22, ldC);              // C22 -= Y21 St12
  rtrsyl<R>(m1, n1, S11, ldS, T11, ldT, C11, ldC, blks);             // Y11
  rtrsyl<R>(m2, n2, S22, ldS, T22, ldT, C22, ldC, blks);             // Y22
  sub_gemm<R>(m1, n2, m2, S12, ldS, C22, ldC, C12, ldC);              // C12 -= S12 Y22
  sub_gemm<R>(m1, n2, n1, C11, ldC, T12, ldT, C12, ldC);              // C12 -= Y11 St12
  rtrsyl<R>(m1, n2, S11, ldS, T22, ldT, C12, ldC, blks);             // Y12
}

// ---------------------------------------------------------------------------
// Real quasi-triangular route (remark after the blocked square root in
// Sec. 2.2.1): for real A the real Schur form A = Q T Q^T is used, T
// quasi-upper-triangular with 1x1 and 2x2 diagonal blocks, and a block
// partition never separates the two rows of a 2x2 block.  The square root and
// the Sylvester solves below are the block forms of Eq. (subst) and of the
// back-substitution, with 1x1 / 2x2 blocks in place of scalars.

// Diagonal block structure of an m x m quasi-upper-triangular matrix: the
// block starts, followed by m.  A 2x2 block starts at i when t(i+1, i) != 0.
template <class R> std::vector<int> qt_blocks(int m, const R* t, int ld) {
  std::vector<int> st;
  for (int i = 0; i < m;) {
    st.push_back(i);
    i += (i + 1 < m && t[i + 1 + (size_t)i * ld] != R(0)) ? 2 : 1;
  }
  st.push_back(m);
  return st;
}

// A Y + Y B = Cm for a p x p block A and a q x q block B (p, q <= 2): the
// Kronecker form (I_q kron A + B^T kron I_p) vec(Y) = vec(Cm) (Sec. 3.1's
// vec form, at block size) by Gaussian elimination with partial pivoting.
template <class R>
void sylv_small(int p, int q, const R* A, int lda, const R* B, int ldb, const R* Cm, int ldc, R* Y,
                int ldy) {
  const int N = p * q;
  R M[4][5];
  for (int c = 0; c < q; ++c)
    for (int r = 0; r < p; ++r) {
      const int row = r + p * c;
      for (int l = 0; l < q; ++l)
        for (int k = 0; k < p; ++k) {
          R v = 0;
          if (l == c) v += A[r + (size_t)k * lda];
          if (k == r) v += B[l + (size_t)c * ldb];
          M[row][k + p * l] = v;
        }
      M[row][N] = Cm[r + (size_t)c * ldc];
    }
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int i = k + 1; i < N; ++i)
      if (std::abs(M[i][k]) > std::abs(M[piv][k])) piv = i;
    if (piv != k)
      for (int j = 0; j <= N; ++j) std::swap(M[k][j], M[piv][j]);
    for (int i = k + 1; i < N; ++i) {
      const R f = M[i][k] / M[k][k];
      for (int j = k; j <= N; ++j) M[i][j] -= f * M[k][j];
    }
  }
  R x[4];
  for (int i = N - 1; i >= 0; --i) {
    R acc = M[i][N];
    for (int j = i + 1; j < N; ++j) acc -= M[i][j] * x[j];
    x[i] = acc / M[i][i];
  }
  for (int c = 0; c < q; ++c)
    for (int r = 0; r < p; ++r) Y[r + (size_t)c * ldy] = x[r + p * c];
}

// Principal square root of a 2x2 real block B without eigenvalues on R<=0.
// For X = B^{1/2}, Cayley-Hamilton gives X^2 - tr(X) X + det(X) I = 0, i.e.
// B + det(X) I = tr(X) X; det(X)^2 = det B and, taking traces,
// tr(X)^2 = tr B + 2 det(X).  The principal root has both eigenvalues in the
// open right half-plane, so det(X) and tr(X) are the positive roots:
//   X = (B + d I) / t,  d = sqrt(det B),  t = sqrt(tr B + 2 d).
// Returns false when det B <= 0 or tr B + 2 d <= 0 (no real principal root).
template <class R> bool sqrt_2x2(const R* b, int ldb, R* x, int ldx) {
  const R a11 = b[0], a21 = b[1], a12 = b[ldb], a22 = b[1 + ldb];
  const R det = a11 * a22 - a12 * a21;
  if (!(det > R(0))) return false;
  const R d = std::sqrt(det);
  const R t2 = a11 + a22 + R(2) * d;
  if (!(t2 > R(0))) return false;
  const R t = std::sqrt(t2);
  x[0] = (a11 + d) / t;
  x[1] = a21 / t;
  x[ldx] = a12 / t;
  x[1 + ldx] = (a22 + d) / t;
  return true;
}

// Square root U of a quasi-upper-triangular T by blocks (Eq. (subst) with
// the diagonal blocks as units): U_ii = T_ii^{1/2} (scalar root, or the 2x2
// closed form above), and for i < j
//   U_ii U_ij + U_ij U_jj = T_ij - sum_{i<k<j} U_ik U_kj.
// Returns 2 when a diagonal block has an eigenvalue on R<=0.
template <class R> int trsqrt_quasi(int n, const R* t, R* u) {
  for (size_t k = 0; k < (size_t)n * n; ++k) u[k] = 0;
  const std::vector<int> bs = qt_blocks<R>(n, t, n);
  const int nb = (int)bs.size() - 1;
  for (int b = 0; b < nb; ++b) {
    const int i = bs[b], p = bs[b + 1] - i;
    if (p == 1) {
      const R d = t[i + (size_t)i * n];
      if (!(d > R(0))) return 2;
      u[i + (size_t)i * n] = std::sqrt(d);
    } else if (!sqrt_2x2<R>(t + i + (size_t)i * n, n, u + i + (size_t)i * n, n)) {
      return 2;
    }
  }
  auto block = [&](int bi, int bj) {
    const int i0 = bs[bi], p = bs[bi + 1] - i0, j0 = bs[bj], q = bs[bj + 1] - j0;
    R rhs[4];
    for (int c = 0; c < q; ++c)
      for (int r = 0; r < p; ++r) {
        R acc = t[i0 + r + (size_t)(j0 + c) * n];
        for (int k = bs[bi + 1]; k < j0; ++k)
          acc -= u[i0 + r + (size_t)k * n] * u[k + (size_t)(j0 + c) * n];
        rhs[r + p * c] = acc;
      }
    sylv_small<R>(p, q, u + i0 + (size_t)i0 * n, n, u + j0 + (size_t)j0 * n, n, rhs, p,
                  u + i0 + (size_t)j0 * n, n);
  };
  // block (bi, bj) reads only blocks of lower block superdiagonals
  for (int d = 1; d < nb; ++d) {
#pragma omp parallel for schedule(static) if (g_deferred)
    for (int bi = 0; bi < nb - d; ++bi) block(bi, bi + d);
  }
  return 0;
}

// S Y + Y St = Cm with S (m x m) and St (n x n) quasi-upper-triangular, by
// block back-substitution: block columns left to right, block rows bottom to
// top,
//   S_ii Y_ij + Y_ij St_jj = C_ij - sum_{k>i} S_ik Y_kj - sum_{l<j} Y_il St_lj.
template <class R>
void trsyl_quasi(int m, int n, const R* S, int ldS, const R* St, int ldT, const R* Cm, int ldC,
                 R* Y, int ldY) {
  const std::vector<int> rb = qt_blocks<R>(m, S, ldS), cb = qt_blocks<R>(n, St, ldT);
  const int nrb = (int)rb.size() - 1, ncb = (int)cb.size() - 1;
  for (int bj = 0; bj < ncb; ++bj) {
    const int j0 = cb[bj], q = cb[bj + 1] - j0;
    for (int bi = nrb - 1; bi >= 0; --bi) {
      const int i0 = rb[bi], p = rb[bi + 1] - i0;
      R rhs[4];
      for (int c = 0; c < q; ++c)
        for (int r = 0; r < p; ++r) {
          const int i = i0 + r, j = j0 + c;
          R acc = Cm[i + (size_t)j * ldC];
          for (int k = rb[bi + 1]; k < m; ++k) acc -= S[i + (size_t)k * ldS] * Y[k + (size_t)j * ldY];
          for (int k = 0; k < j0; ++k) acc -= Y[i + (size_t)k * ldY] * St[k + (size_t)j * ldT];
          rhs[r + p * c] = acc;
        }
      sylv_small<R>(p, q, S + i0 + (size_t)i0 * ldS, ldS, St + j0 + (size_t)j0 * ldT, ldT, rhs, p,
                    Y + i0 + (size_t)j0 * ldY, ldY);
    }
  }
}

// Cm(mxn) -= A(mxk) * B(kxn), real sub-blocks with leading dimensions.
template <class R>
void sub_gemm_real(int m, int n, int k, const R* A, int lda, const R* B, int ldb, R* Cm, int ldc) {
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < k; ++l) {
      const R b = B[l + (size_t)j * ldb];
      for (int i = 0; i < m; ++i) Cm[i + (size_t)j * ldc] -= A[i + (size_t)l * lda] * b;
    }
}

// Split point of a quasi-triangular dimension m for Alg. 1: floor(m/2),
// moved one index down when it would separate the two rows of a 2x2 diagonal
// block (s(h, h-1) != 0), so that no 2x2 block is cut.  Returns m when no
// split is possible (a single 2x2 block).
template <class R> int qsplit(int m, const R* S, int ld) {
  int h = m / 2;
  if (h > 0 && h < m && S[h + (size_t)(h - 1) * ld] != R(0)) ++h;
  return h;
}

// Alg. 1 for quasi-upper-triangular S and St: the recursion of rtrsyl above
// with the split points of qsplit; Cm is overwritten with Y.
template <class R>
void rtrsyl_quasi(int m, int n, const R* S, int ldS, const R* St, int ldT, R* Cm, int ldC,
                  int blks) {
  if (m <= 0 || n <= 0) return;
  const int m1 = qsplit<R>(m, S, ldS), n1 = qsplit<R>(n, St, ldT);
  const bool base = (m <= blks && n <= blks);
  const bool rows = !base && 2 * n <= m && m1 < m;
  const bool cols = !base && !rows && 2 * m <= n && n1 < n;
  const bool both = !base && !rows && !cols && 2 * n > m && 2 * m > n && m1 < m && n1 < n;
  if (!rows && !cols && !both) {
    std::vector<R> y((size_t)m * n);
    trsyl_quasi<R>(m, n, S, ldS, St, ldT, Cm, ldC, y.data(), m);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < m; ++i) Cm[i + (size_t)j * ldC] = y[i + (size_t)j * m];
    return;
  }
  if (rows) {
    const int m2 = m - m1;
    const R* S12 = S + (size_t)m1 * ldS;
    const R* S22 = S + m1 + (size_t)m1 * ldS;
    R* C2 = Cm + m1;
    rtrsyl_quasi<R>(m2, n, S22, ldS, St, ldT, C2, ldC, blks);
    sub_gemm_real<R>(m1, n, m2, S12, ldS, C2, ldC, Cm, ldC);
    rtrsyl_quasi<R>(m1, n, S, ldS, St, ldT, Cm, ldC, blks);
    return;
  }
  if (cols) {
    const int n2 = n - n1;
    const R* T12 = St + (size_t)n1 * ldT;
    const R* T22 = St + n1 + (size_t)n1 * ldT;
    R* C2 = Cm + (size_t)n1 * ldC;
    rtrsyl_quasi<R>(m, n1, S, ldS, St, ldT, Cm, ldC, blks);
    sub_gemm_real<R>(m, n2, n1, Cm, ldC, T12, ldT, C2, ldC);
    rtrsyl_quasi<R>(m, n2, S, ldS, T22, ldT, C2, ldC, blks);
    return;
  }
  const int m2 = m - m1, n2 = n - n1;
  const R* S12 = S + (size_t)m1 * ldS;
  const R* S22 = S + m1 + (size_t)m1 * ldS;
  const R* T12 = St + (size_t)n1 * ldT;
  const R* T22 = St + n1 + (size_t)n1 * ldT;
  R* C11 = Cm;
  R* C21 = Cm + m1;
  R* C12 = Cm + (size_t)n1 * ldC;
  R* C22 = Cm + m1 + (size_t)n1 * ldC;
  rtrsyl_quasi<R>(m2, n1, S22, ldS, St, ldT, C21, ldC, blks);   // Y21
  sub_gemm_real<R>(m1, n1, m2, S12, ldS, C21, ldC, C11, ldC);    // C11 -= S12 Y21
  sub_gemm_real<R>(m2, n2, n1, C21, ldC, T12, ldT, C22, ldC);    // C22 -= Y21 St12
  rtrsyl_quasi<R>(m1, n1, S, ldS, St, ldT, C11, ldC, blks);     // Y11
  rtrsyl_quasi<R>(m2, n2, S22, ldS, T22, ldT, C22, ldC, blks);  // Y22
  sub_gemm_real<R>(m1, n2, m2, S12, ldS, C22, ldC, C12, ldC);    // C12 -= S12 Y22
  sub_gemm_real<R>(m1, n2, n1, C11, ldC, T12, ldT, C12, ldC);    // C12 -= Y11 St12
  rtrsyl_quasi<R>(m1, n2, S, ldS, T22, ldT, C12, ldC, blks);    // Y12
}

// ---------------------------------------------------------------------------
// Matrix cube roots (Sec. 4, p = 3).

// Principal cube root of z (z not on the closed negative real axis):
// |z|^{1/3} e^{i arg(z)/3} with arg in (-pi, pi).
template <class R> C<R> ccbrt_principal(C<R> z) {
  if (z.real() == R(0) && z.imag() == R(0)) return C<R>(0, 0);
  const R r = std::cbrt(std::abs(z));
  const R th = std::atan2(z.imag(), z.real()) / R(3);
  return C<R>(r * std::cos(th), r * std::sin(th));
}

// Cube root of an upper triangular matrix: U with U^3 = T, principal cube
// roots on the diagonal.  With V = U^2, entry (i, j), i < j, of U^3 = U V
// and of V = U U give
//   v_ij = (u_ii + u_jj) u_ij + a_ij,            a_ij = sum_{i<k<j} u_ik u_kj,
//   (u_ii^2 + u_ii u_jj + u_jj^2) u_ij = t_ij - u_ii a_ij - b_ij,
//                                                 b_ij = sum_{i<k<j} u_ik v_kj,
// solved column by column (j ascending, i descending), the Schur method for
// p-th roots specialised to p = 3.  Returns 2 if a diagonal entry of T lies
// on the closed negative real axis.
template <class R> int trroot3(int n, const C<R>* t, C<R>* u) {
  std::vector<C<R>> v((size_t)n * n, C<R>(0, 0));
  for (size_t k = 0; k < (size_t)n * n; ++k) u[k] = 0;
  for (int i = 0; i < n; ++i) {
    C<R> d = t[i + (size_t)i * n];
    if (d.imag() == R(0) && d.real() <= R(0)) return 2;
    u[i + (size_t)i * n] = ccbrt_principal<R>(d);
    v[i + (size_t)i * n] = u[i + (size_t)i * n] * u[i + (size_t)i * n];
  }
  for (int j = 1; j < n; ++j) {
    for (int i = j - 1; i >= 0; --i) {
      C<R> a = 0, b = 0;
      for (int k = i + 1; k <= j - 1; ++k) {
        a += u[i + (size_t)k * n] * u[k + (size_t)j * n];
        b += u[i + (size_t)k * n] * v[k + (size_t)j * n];
      }
      const C<R> ui = u[i + (size_t)i * n], uj = u[j + (size_t)j * n];
      const C<R> x = (t[i + (size_t)j * n] - ui * a - b) / (ui * ui + ui * uj + uj * uj);
      u[i + (size_t)j * n] = x;
      v[i + (size_t)j * n] = (ui + uj) * x + a;
    }
  }
  return 0;
}

// Cm(mxn) -= A(mxk) * B(kxn) * Cr(nxp)... helpers for the generalized
// equation use plain products into temporaries.
template <class R>
void mat_mul(int m, int n, int k, const C<R>* A, int lda, const C<R>* B, int ldb, C<R>* D,
             int ldd) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) D[i + (size_t)j * ldd] = 0;
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < k; ++l) {
      const C<R> b = B[l + (size_t)j * ldb];
      for (int i = 0; i < m; ++i) D[i + (size_t)j * ldd] += A[i + (size_t)l * lda] * b;
    }
}

// Base case of the p = 3 equation S^2 Y + S Y St + Y St^2 = Cm (S m x m, St
// n x n upper triangular): Bartels-Stewart-type substitution, columns left
// to right and rows bottom to top.  The coefficient of y_ij is
// s_ii^2 + s_ii st_jj + st_jj^2; every other term involves entries of Y
// already known, with U = Y St accumulated column by column.
template <class R>
void trsyl3(int m, int n, const C<R>* S, int ldS, const C<R>* St, int ldT, const C<R>* Cm, int ldC,
            C<R>* Y, int ldY) {
  std::vector<C<R>> S2((size_t)m * m), T2((size_t)n * n), U((size_t)m * n, C<R>(0, 0));
  mat_mul<R>(m, m, m, S, ldS, S, ldS, S2.data(), m);
  mat_mul<R>(n, n, n, St, ldT, St, ldT, T2.data(), n);
  for (int j = 0; j < n; ++j) {
    for (int i = m - 1; i >= 0; --i) {
      C<R> acc = Cm[i + (size_t)j * ldC];
      // (S^2 Y)_ij without the diagonal term
      for (int k = i + 1; k < m; ++k) acc -= S2[i + (size_t)k * m] * Y[k + (size_t)j * ldY];
      // (S Y St)_ij = sum_{k >= i} s_ik (Y St)_kj: rows k > i are complete in U
      for (int k = i + 1; k < m; ++k) acc -= S[i + (size_t)k * ldS] * U[k + (size_t)j * m];
      //   k = i: s_ii sum_{l < j} y_il st_lj (the l = j term is on the left)
      C<R> yst = 0;
      for (int l = 0; l < j; ++l) yst += Y[i + (size_t)l * ldY] * St[l + (size_t)j * ldT];
      acc -= S[i + (size_t)i * ldS] * yst;
      // (Y St^2)_ij without the diagonal term
      for (int l = 0; l < j; ++l) acc -= Y[i + (size_t)l * ldY] * T2[l + (size_t)j * n];
      const C<R> si = S[i + (size_t)i * ldS], tj = St[j + (size_t)j * ldT];
      const C<R> y = acc / (si * si + si * tj + tj * tj);
      Y[i + (size_t)j * ldY] = y;
      U[i + (size_t)j * m] = yst + y * tj;
    }
  }
}

// Cm(mxn) -= A(mxk) B(kxn).
template <class R>
void sub_prod(int m, int n, int k, const C<R>* A, int lda, const C<R>* B, int ldb, C<R>* Cm,
              int ldc) {
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < k; ++l) {
      const C<R> b = B[l + (size_t)j * ldb];
      for (int i = 0; i < m; ++i) Cm[i + (size_t)j * ldc] -= A[i + (size_t)l * lda] * b;
    }
}

// Cm(mxn) -= A(mxk) B(kxl) D(lxn) (B, D may be rectangular blocks).
template <class R>
void sub_prod3(int m, int n, int k, int l, const C<R>* A, int lda, const C<R>* B, int ldb,
               const C<R>* D, int ldd, C<R>* Cm, int ldc) {
  std::vector<C<R>> tmp((size_t)k * n);
  mat_mul<R>(k, n, l, B, ldb, D, ldd, tmp.data(), k);
  sub_prod<R>(m, n, k, A, lda, tmp.data(), k, Cm, ldc);
}

// (X Y + Z W) for blocks: D = A11 A12 + A12 A22 with A = [A11 A12; 0 A22],
// the (1,2) block of A^2 (A11 is m1 x m1, A22 m2 x m2).
template <class R>
std::vector<C<R>> square_12(int m1, int m2, const C<R>* A, int lda) {
  std::vector<C<R>> d((size_t)m1 * m2), t((size_t)m1 * m2);
  const C<R>* A11 = A;
  const C<R>* A12 = A + (size_t)m1 * lda;
  const C<R>* A22 = A + m1 + (size_t)m1 * lda;
  mat_mul<R>(m1, m2, m1, A11, lda, A12, lda, d.data(), m1);
  mat_mul<R>(m1, m2, m2, A12, lda, A22, lda, t.data(), m1);
  for (size_t x = 0; x < d.size(); ++x) d[x] += t[x];
  return d;
}

// Block recursion for S^2 Y + S Y St + Y St^2 = Cm (Sec. 4, p = 3), the
// analogue of Alg. 1: the diagonal blocks are split at floor(m/2) (floor(n/2))
// and the four block equations of Sec. 4 are solved in the order
// Y21, Y11, Y22, Y12; when only one side is large, only that side is split
// (the same block algebra with one block row or column).  Cm is overwritten
// by Y.
template <class R>
void rtrsyl3(int m, int n, const C<R>* S, int ldS, const C<R>* St, int ldT, C<R>* Cm, int ldC,
             int blks) {
  if (m <= 0 || n <= 0) return;
  if (m <= blks && n <= blks) {
    std::vector<C<R>> y((size_t)m * n, C<R>(0, 0));
    trsyl3<R>(m, n, S, ldS, St, ldT, Cm, ldC, y.data(), m);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < m; ++i) Cm[i + (size_t)j * ldC] = y[i + (size_t)j * m];
    return;
  }
  if (2 * n <= m) {
    // rows only: S = [S11 S12; 0 S22], Y = [Y1; Y2]
    const int m1 = m / 2, m2 = m - m1;
    const C<R>* S11 = S;
    const C<R>* S12 = S + (size_t)m1 * ldS;
    const C<R>* S22 = S + m1 + (size_t)m1 * ldS;
    C<R>* C1 = Cm;
    C<R>* C2 = Cm + m1;
    rtrsyl3<R>(m2, n, S22, ldS, St, ldT, C2, ldC, blks);                  // Y2
    std::vector<C<R>> s2_12 = square_12<R>(m1, m2, S, ldS);
    sub_prod<R>(m1, n, m2, s2_12.data(), m1, C2, ldC, C1, ldC);           // -(S^2)_12 Y2
    sub_prod3<R>(m1, n, m2, n, S12, ldS, C2, ldC, St, ldT, C1, ldC);      // -S12 Y2 St
    rtrsyl3<R>(m1, n, S11, ldS, St, ldT, C1, ldC, blks);                  // Y1
    return;
  }
  if (2 * m <= n) {
    // columns only: St = [T11 T12; 0 T22], Y = [Y1 Y2]
    const int n1 = n / 2, n2 = n - n1;
    const C<R>* T11 = St;
    const C<R>* T12 = St + (size_t)n1 * ldT;
    const C<R>* T22 = St + n1 + (size_t)n1 * ldT;
    C<R>* C1 = Cm;
    C<R>* C2 = Cm + (size_t)n1 * ldC;
    rtrsyl3<R>(m, n1, S, ldS, T11, ldT, C1, ldC, blks);                   // Y1
    sub_prod3<R>(m, n2, m, n1, S, ldS, C1, ldC, T12, ldT, C2, ldC);       // -S Y1 T12
    std::vector<C<R>> t2_12 = square_12<R>(n1, n2, St, ldT);
    sub_prod<R>(m, n2, n1, C1, ldC, t2_12.data(), n1, C2, ldC);           // -Y1 (St^2)_12
    rtrsyl3<R>(m, n2, S, ldS, T22, ldT, C2, ldC, blks);                   // Y2
    return;
  }
  const int m1 = m / 2, m2 = m - m1, n1 = n / 2, n2 = n - n1;
  const C<R>* S11 = S;
  const C<R>* S12 = S + (size_t)m1 * ldS;
  const C<R>* S22 = S + m1 + (size_t)m1 * ldS;
  const C<R>* T11 = St;
  const C<R>* T12 = St + (size_t)n1 * ldT;
  const C<R>* T22 = St + n1 + (size_t)n1 * ldT;
  C<R>* C11 = Cm;
  C<R>* C21 = Cm + m1;
  C<R>* C12 = Cm + (size_t)n1 * ldC;
  C<R>* C22 = Cm + m1 + (size_t)n1 * ldC;
  const std::vector<C<R>> s2_12 = square_12<R>(m1, m2, S, ldS);   // S11 S12 + S12 S22
  const std::vector<C<R>> t2_12 = square_12<R>(n1, n2, St, ldT);  // T11 T12 + T12 T22
  // Y21: S22^2 Y21 + S22 Y21 T11 + Y21 T11^2 = C21
  rtrsyl3<R>(m2, n1, S22, ldS, T11, ldT, C21, ldC, blks);
  // Y11: ... = C11 - (S11 S12 + S12 S22) Y21 - S12 Y21 T11
  sub_prod<R>(m1, n1, m2, s2_12.data(), m1, C21, ldC, C11, ldC);
  sub_prod3<R>(m1, n1, m2, n1, S12, ldS, C21, ldC, T11, ldT, C11, ldC);
  rtrsyl3<R>(m1, n1, S11, ldS, T11, ldT, C11, ldC, blks);
  // Y22: ... = C22 - Y21 (T11 T12 + T12 T22) - S22 Y21 T12
  sub_prod<R>(m2, n2, n1, C21, ldC, t2_12.data(), n1, C22, ldC);
  sub_prod3<R>(m2, n2, m2, n1, S22, ldS, C21, ldC, T12, ldT, C22, ldC);
  rtrsyl3<R>(m2, n2, S22, ldS, T22, ldT, C22, ldC, blks);
  // Y12: ... = C12 - (S11 S12 + S12 S22) Y22 - S12 Y22 T22
  //            - Y11 (T11 T12 + T12 T22) - (S11 Y11 + S12 Y21) T12
  sub_prod<R>(m1, n2, m2, s2_12.data(), m1, C22, ldC, C12, ldC);
  sub_prod3<R>(m1, n2, m2, n2, S12, ldS, C22, ldC, T22, ldT, C12, ldC);
  sub_prod<R>(m1, n2, n1, C11, ldC, t2_12.data(), n1, C12, ldC);
  {
    std::vector<C<R>> w((size_t)m1 * n1), t((size_t)m1 * n1);
    mat_mul<R>(m1, n1, m1, S11, ldS, C11, ldC, w.data(), m1);
    mat_mul<R>(m1, n1, m2, S12, ldS, C21, ldC, t.data(), m1);
    for (size_t x = 0; x < w.size(); ++x) w[x] += t[x];
    sub_prod<R>(m1, n2, n1, w.data(), m1, T12, ldT, C12, ldC);
  }
  rtrsyl3<R>(m1, n2, S11, ldS, T22, ldT, C12, ldC, blks);
}

// ---------------------------------------------------------------------------
// Real symmetric eigendecomposition A = Q diag(lam) Q^T: Householder
// tridiagonalisation with explicit accumulation of Q, then the implicit
// symmetric QR iteration with Wilkinson shifts (Golub & Van Loan, Sec. 8.3),
// each step a chase of a bulge by Givens rotations that are also applied to Q.
// Eigenvalues are returned in ascending order with matching columns of Q.
// Returns 0, or 1 if the iteration did not converge within 30 n sweeps.
template <class R> int syev(int n, const R* ain, R* lam, R* q) {
  std::vector<R> a(ain, ain + (size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) q[i + (size_t)j * n] = (i == j) ? R(1) : R(0);
  auto A = [&](int i, int j) -> R& { return a[i + (size_t)j * n]; };
  std::vector<R> u(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    int len = n - k - 1;
    R nx2 = 0;
    for (int i = 0; i < len; ++i) nx2 += A(k + 1 + i, k) * A(k + 1 + i, k);
    R x0 = A(k + 1, k);
    if (nx2 - x0 * x0 <= R(0)) continue;
    R nx = std::sqrt(nx2);
    for (int i = 0; i < len; ++i) u[i] = A(k + 1 + i, k);
    u[0] += (x0 >= R(0) ? nx : -nx);
    R un2 = 0;
    for (int i = 0; i < len; ++i) un2 += u[i] * u[i];
    R f = R(2) / un2;
    // Two-sided update of the trailing block B = A(k+1:, k+1:) and of the
    // column/row k: A <- P A P with P = I - f u u^T.
    // p = f B u ; K = f/2 u^T p ; w = p - K u ; B <- B - u w^T - w u^T.
#pragma omp parallel for schedule(static)
    for (int i0 = 0; i0 < len; i0 += kChunk) {  // rows independent
      const int i1 = std::min(len, i0 + kChunk);
      for (int i = i0; i < i1; ++i) p[i] = 0;
      for (int j = 0; j < len; ++j)
        for (int i = i0; i < i1; ++i) p[i] += A(k + 1 + i, k + 1 + j) * u[j];
    }
    for (int i = 0; i < len; ++i) p[i] *= f;
    R K = 0;
    for (int i = 0; i < len; ++i) K += u[i] * p[i];
    K *= f / R(2);
    for (int i = 0; i < len; ++i) w[i] = p[i] - K * u[i];
#pragma omp parallel for schedule(static)
    for (int j = 0; j < len; ++j)
      for (int i = 0; i < len; ++i) A(k + 1 + i, k + 1 + j) -= u[i] * w[j] + w[i] * u[j];
    R newv = (x0 >= R(0) ? -nx : nx);
    A(k + 1, k) = newv;
    A(k, k + 1) = newv;
    for (int i = 1; i < len; ++i) { A(k + 1 + i, k) = 0; A(k, k + 1 + i) = 0; }
    // Q <- Q P:  r = Q u, then Q -= f r u^T.
    std::vector<R> r(n, R(0));
#pragma omp parallel for schedule(static)
    for (int i0 = 0; i0 < n; i0 += kChunk) {  // rows independent
      const int i1 = std::min(n, i0 + kChunk);
      for (int j = 0; j < len; ++j)
        for (int i = i0; i < i1; ++i) r[i] += q[i + (size_t)(k + 1 + j) * n] * u[j];
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < len; ++j)
      for (int i = 0; i < n; ++i) q[i + (size_t)(k + 1 + j) * n] -= f * r[i] * u[j];
  }
  std::vector<R> d(n), e(n, R(0));
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);
  const R eps = std::numeric_limits<R>::epsilon() / 2;
  // The rotations touch d, e and two columns of Q.  Rows of Q are
  // independent, so the rotations can be logged and applied later, in order,
  // to blocks of rows in parallel (same operations per entry).
  struct QRot { int k; R c, s; };
  std::vector<QRot> qlog;
  auto rotate_q = [&](int k, R c, R s, int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      R qa = q[i + (size_t)k * n], qb = q[i + (size_t)(k + 1) * n];
      q[i + (size_t)k * n] = c * qa + s * qb;
      q[i + (size_t)(k + 1) * n] = -s * qa + c * qb;
    }
  };
  auto flush_q = [&]() {
    const int nl = (int)qlog.size();
#pragma omp parallel for schedule(static)
    for (int i0 = 0; i0 < n; i0 += 16) {
      const int i1 = std::min(n, i0 + 16);
      for (int t = 0; t < nl; ++t) rotate_q(qlog[t].k, qlog[t].c, qlog[t].s, i0, i1);
    }
    qlog.clear();
  };
  int hi = n - 1, total = 0;
  while (hi > 0) {
    int lo = hi;
    while (lo > 0) {
      if (std::fabs(e[lo - 1]) <= eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) {
        e[lo - 1] = 0;
        break;
      }
      --lo;
    }
    if (lo == hi) { --hi; continue; }
    if (++total > 30 * n) { flush_q(); return 1; }
    // Wilkinson shift from the trailing 2x2 block.
    R dd = (d[hi - 1] - d[hi]) / R(2);
    R b2 = e[hi - 1] * e[hi - 1];
    R den = dd + (dd >= R(0) ? R(1) : R(-1)) * std::sqrt(dd * dd + b2);
    R mu = (den == R(0)) ? d[hi] : d[hi] - b2 / den;
    R x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      // Rotation in the (k, k+1) plane that annihilates z against x.
      R r = std::hypot(x, z);
      R c = (r == R(0)) ? R(1) : x / r;
      R s = (r == R(0)) ? R(0) : z / r;
      if (k > lo) e[k - 1] = r;
      // Apply G^T T G on the tridiagonal entries touched by the rotation.
      R dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk + R(2) * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk - R(2) * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
      if (k + 1 < hi) {
        x = e[k];
        z = s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      if (g_deferred) {
        qlog.push_back({k, c, s});
      } else {
        rotate_q(k, c, s, 0, n);
      }
    }
    if (qlog.size() >= ((size_t)1 << 20)) flush_q();
  }
  flush_q();
  // Sort ascending (selection sort keeps it obviously correct).
  for (int i = 0; i < n; ++i) {
    int m = i;
    for (int j = i + 1; j < n; ++j)
      if (d[j] < d[m]) m = j;
    if (m != i) {
      std::swap(d[i], d[m]);
      for (int r = 0; r < n; ++r) std::swap(q[r + (size_t)i * n], q[r + (size_t)m * n]);
    }
  }
  for (int i = 0; i < n; ++i) lam[i] = d[i];
  return 0;
}

}  // namespace orc

using orc::C;

extern "C" {

// Number of OpenMP threads (0 keeps the runtime's default) and the rotation
// mode (1: deferred, parallel; 0: immediate, serial order); see g_deferred.
void orc_set_threads(int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
}
int orc_get_threads(void) { return omp_get_max_threads(); }
void orc_set_deferred(int on) { orc::g_deferred = on ? 1 : 0; }

// Status codes shared by the oracle entry points.
enum { ORC_OK = 0, ORC_NOCONV = 1, ORC_NO_PRINCIPAL = 2 };

// Real quasi-triangular route: square root of a quasi-upper-triangular T,
// the block back-substitution and Alg. 1 with the no-cut split rule.
int orc_trsqrt_quasi_d(int n, const double* t, double* u) { return orc::trsqrt_quasi<double>(n, t, u); }
int orc_trsqrt_quasi_s(int n, const float* t, float* u) { return orc::trsqrt_quasi<float>(n, t, u); }
void orc_trsyl_quasi_d(int m, int n, const double* s, const double* st, const double* cm, double* y) {
  orc::trsyl_quasi<double>(m, n, s, m, st, n, cm, m, y, m);
}
void orc_rtrsyl_quasi_d(int m, int n, const double* s, const double* st, double* cm, int blks) {
  orc::rtrsyl_quasi<double>(m, n, s, m, st, n, cm, m, blks);
}
void orc_rtrsyl_quasi_s(int m, int n, const float* s, const float* st, float* cm, int blks) {
  orc::rtrsyl_quasi<float>(m, n, s, m, st, n, cm, m, blks);
}
int orc_sqrt_2x2_d(const double* b, double* x) { return orc::sqrt_2x2<double>(b, 2, x, 2) ? 0 : 2; }

// Complex Schur decomposition A = Q T Q^H (complex128).  a: in A, out T.
int orc_schur_z(int n, double* a, double* q) {
  return orc::schur<double>(n, reinterpret_cast<C<double>*>(a), reinterpret_cast<C<double>*>(q));
}
int orc_schur_c(int n, float* a, float* q) {
  return orc::schur<float>(n, reinterpret_cast<C<float>*>(a), reinterpret_cast<C<float>*>(q));
}

int orc_trsqrt_z(int n, const double* t, double* s) {
  return orc::trsqrt<double>(n, reinterpret_cast<const C<double>*>(t), reinterpret_cast<C<double>*>(s));
}
int orc_trsqrt_c(int n, const float* t, float* s) {
  return orc::trsqrt<float>(n, reinterpret_cast<const C<float>*>(t), reinterpret_cast<C<float>*>(s));
}

// Principal square root by the Schur method: A = Q T Q^H, S = T^{1/2},
// X = Q S Q^H.  complex128 in/out.  Optionally returns Q, T, S.
int orc_sqrtm_z(int n, const double* a_in, double* x_out, double* q_out, double* t_out,
                double* s_out) {
  using Z = C<double>;
  std::vector<Z> a(reinterpret_cast<const Z*>(a_in), reinterpret_cast<const Z*>(a_in) + (size_t)n * n);
  std::vector<Z> q((size_t)n * n), s((size_t)n * n), tmp((size_t)n * n), x((size_t)n * n);
  int st = orc::schur<double>(n, a.data(), q.data());
  if (st) return st;
  st = orc::trsqrt<double>(n, a.data(), s.data());
  if (st) return st;
  // X = Q S Q^H
  orc::cgemm<double>(n, q.data(), s.data(), tmp.data());
  std::vector<Z> qh((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) qh[i + (size_t)j * n] = std::conj(q[j + (size_t)i * n]);
  orc::cgemm<double>(n, tmp.data(), qh.data(), x.data());
  std::memcpy(x_out, x.data(), sizeof(Z) * (size_t)n * n);
  if (q_out) std::memcpy(q_out, q.data(), sizeof(Z) * (size_t)n * n);
  if (t_out) std::memcpy(t_out, a.data(), sizeof(Z) * (size_t)n * n);
  if (s_out) std::memcpy(s_out, s.data(), sizeof(Z) * (size_t)n * n);
  return 0;
}

// Triangular cube root (complex128 / complex64).
int orc_trroot3_z(int n, const double* t, double* u) {
  return orc::trroot3<double>(n, reinterpret_cast<const C<double>*>(t), reinterpret_cast<C<double>*>(u));
}
int orc_trroot3_c(int n, const float* t, float* u) {
  return orc::trroot3<float>(n, reinterpret_cast<const C<float>*>(t), reinterpret_cast<C<float>*>(u));
}

// p = 3 generalized triangular Sylvester equation: unblocked substitution
// (y = solution) and the block recursion (cm overwritten by Y).
void orc_trsyl3_z(int m, int n, const double* s, const double* st, const double* cm, double* y) {
  using Z = C<double>;
  std::vector<Z> yy((size_t)m * n, Z(0, 0));
  orc::trsyl3<double>(m, n, reinterpret_cast<const Z*>(s), m, reinterpret_cast<const Z*>(st), n,
                      reinterpret_cast<const Z*>(cm), m, yy.data(), m);
  std::memcpy(y, yy.data(), sizeof(Z) * (size_t)m * n);
}
void orc_rtrsyl3_z(int m, int n, const double* s, const double* st, double* cm, int blks) {
  using Z = C<double>;
  orc::rtrsyl3<double>(m, n, reinterpret_cast<const Z*>(s), m, reinterpret_cast<const Z*>(st), n,
                       reinterpret_cast<Z*>(cm), m, blks);
}
void orc_rtrsyl3_c(int m, int n, const float* s, const float* st, float* cm, int blks) {
  using Z = C<float>;
  orc::rtrsyl3<float>(m, n, reinterpret_cast<const Z*>(s), m, reinterpret_cast<const Z*>(st), n,
                      reinterpret_cast<Z*>(cm), m, blks);
}

// Principal cube root by the Schur method: A = Q T Q^H, U = T^{1/3},
// X = Q U Q^H (complex128).  Optionally returns Q, T, U.
int orc_rootm3_z(int n, const double* a_in, double* x_out, double* q_out, double* t_out,
                 double* u_out) {
  using Z = C<double>;
  std::vector<Z> a(reinterpret_cast<const Z*>(a_in), reinterpret_cast<const Z*>(a_in) + (size_t)n * n);
  std::vector<Z> q((size_t)n * n), u((size_t)n * n), tmp((size_t)n * n), x((size_t)n * n),
      qh((size_t)n * n);
  int st = orc::schur<double>(n, a.data(), q.data());
  if (st) return st;
  st = orc::trroot3<double>(n, a.data(), u.data());
  if (st) return st;
  orc::cgemm<double>(n, q.data(), u.data(), tmp.data());
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) qh[i + (size_t)j * n] = std::conj(q[j + (size_t)i * n]);
  orc::cgemm<double>(n, tmp.data(), qh.data(), x.data());
  std::memcpy(x_out, x.data(), sizeof(Z) * (size_t)n * n);
  if (q_out) std::memcpy(q_out, q.data(), sizeof(Z) * (size_t)n * n);
  if (t_out) std::memcpy(t_out, a.data(), sizeof(Z) * (size_t)n * n);
  if (u_out) std::memcpy(u_out, u.data(), sizeof(Z) * (size_t)n * n);
  return 0;
}

// Symmetric eigendecomposition (float64 / float32).
int orc_syev_d(int n, const double* a, double* lam, double* q) { return orc::syev<double>(n, a, lam, q); }
int orc_syev_s(int n, const float* a, float* lam, float* q) { return orc::syev<float>(n, a, lam, q); }

// Triangular Sylvester S Y + Y St = Cm (complex128), unblocked.
void orc_trsyl_z(int m, int n, const double* s, const double* st, const double* cm, double* y) {
  using Z = C<double>;
  orc::trsyl<double>(m, n, reinterpret_cast<const Z*>(s), m, reinterpret_cast<const Z*>(st), n,
                     reinterpret_cast<const Z*>(cm), m, reinterpret_cast<Z*>(y), m);
}
void orc_trsyl_c(int m, int n, const float* s, const float* st, const float* cm, float* y) {
  using Z = C<float>;
  orc::trsyl<float>(m, n, reinterpret_cast<const Z*>(s), m, reinterpret_cast<const Z*>(st), n,
                    reinterpret_cast<const Z*>(cm), m, reinterpret_cast<Z*>(y), m);
}

// Alg. 1 block recursion; cm is overwritten by Y.
void orc_rtrsyl_z(int m, int n, const double* s, const double* st, double* cm, int blks) {
  using Z = C<double>;
  orc::rtrsyl<double>(m, n, reinterpret_cast<const Z*>(s), m, reinterpret_cast<const Z*>(st), n,
                      reinterpret_cast<Z*>(cm), m, blks);
}
void orc_rtrsyl_c(int m, int n, const float* s, const float* st, float* cm, int blks) {
  using Z = C<float>;
  orc::rtrsyl<float>(m, n, reinterpret_cast<const Z*>(s), m, reinterpret_cast<const Z*>(st), n,
                     reinterpret_cast<Z*>(cm), m, blks);
}

// Adjoint of the Frechet derivative of the square root: solve
// X^H G + G X^H = Gbar (complex128) through the Schur form X = U S U^H.
// With H = U^H G U and K = H^H the equation becomes S K + K S = (U^H Gbar U)^H,
// an upper triangular Sylvester equation solved by back-substitution.
int orc_adjoint_z(int n, const double* x_in, const double* gb_in, double* g_out) {
  using Z = C<double>;
  std::vector<Z> s(reinterpret_cast<const Z*>(x_in), reinterpret_cast<const Z*>(x_in) + (size_t)n * n);
  std::vector<Z> u((size_t)n * n), uh((size_t)n * n), t1((size_t)n * n), t2((size_t)n * n),
      k((size_t)n * n);
  int st = orc::schur<double>(n, s.data(), u.data());
  if (st) return st;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) uh[i + (size_t)j * n] = std::conj(u[j + (size_t)i * n]);
  const Z* gb = reinterpret_cast<const Z*>(gb_in);
  orc::cgemm<double>(n, uh.data(), gb, t1.data());
  orc::cgemm<double>(n, t1.data(), u.data(), t2.data());   // U^H Gbar U
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) t1[i + (size_t)j * n] = std::conj(t2[j + (size_t)i * n]);
  orc::trsyl<double>(n, n, s.data(), n, s.data(), n, t1.data(), n, k.data(), n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) t2[i + (size_t)j * n] = std::conj(k[j + (size_t)i * n]);  // H
  orc::cgemm<double>(n, u.data(), t2.data(), t1.data());
  orc::cgemm<double>(n, t1.data(), uh.data(), t2.data());
  std::memcpy(g_out, t2.data(), sizeof(Z) * (size_t)n * n);
  return 0;
}

}  // extern "C"
