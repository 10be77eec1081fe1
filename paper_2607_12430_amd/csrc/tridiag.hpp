// Symmetric spectral decomposition on the GPU: Householder tridiagonalisation,
// divide-and-conquer tridiagonal eigensolver, back-transformation.
#pragma once

#include "factor.hpp"

namespace msqrt {

struct SytrdWork {
  DevBuf VW, WV, ypart, sp, vp, bar;
  int nbar = 0;  // batch entries of the last reduction (error flags)
};

struct StedcWork {
  DevBuf dd, ee, lam, Z2, M, meta, rot, roots, zhat, scal;
};

struct OrmtrWork {
  DevBuf gram, VT, Wpart, W;
};

// Half-bandwidth of the two-stage reduction: a panel of 4096 rows fits the
// registers of one workgroup (16 float or 8 double columns).
template <typename T>
struct BandWidth {
  static constexpr int B = sizeof(T) == 4 ? 16 : 8;
};

struct Sy2trWork {
  DevBuf AB, V1, tau1, VW, WV, VT, X, Xp, Yp, Tg, V2, tau2, ctl;
  int n = 0, nsw = 0, kmax = 0;
};

// A (n x n, ld n, full symmetric) is overwritten: column j holds the explicit
// reflector v_j (rows j+1..n-1, v_j(j+1) = 1, zeros above) for rows >= its
// panel start.  d (n), e (n-1), tau (n-1) in the factor precision.
template <typename T>
void sytrd(hipStream_t st, int n, T* A, T* d, T* e, T* tau, SytrdWork& w);
// The same for `batch` matrices A + b sA; entry b's d, e, tau start at
// d + b sD, e + b sD, tau + b sD.  As many entries as fit co-resident share
// one cooperative launch per panel (each with its own grid barrier), and
// the trailing updates are one batched GEMM.
template <typename T>
void sytrd_batched(hipStream_t st, int n, int batch, T* A, int64_t sA, T* d, T* e, T* tau,
                   int64_t sD, SytrdWork& w);
// True if a grid barrier of the last reduction timed out (synchronous).
bool sytrd_failed(SytrdWork& w);

// Eigen-decomposition of the symmetric tridiagonal (d, e): lam ascending
// (float64) and eigenvectors Z (n x n, ld n, precision T).
template <typename T>
void stedc(hipStream_t st, int n, const T* d, const T* e, double* lam, T* Z, StedcWork& w);

// stedc for `batch` tridiagonal matrices of order n (d + m sD, e + m sD),
// solved together as one block-diagonal matrix: every launch of a recursion
// level covers all entries.  lam is n x batch (contiguous), Z is n x n per
// entry (stride n * n).
template <typename T>
void stedc_batched(hipStream_t st, int n, int batch, const T* d, const T* e, int64_t sD,
                   double* lam, T* Z, StedcWork& w);

// Z <- H_0 H_1 ... H_{n-2} Z with the reflectors left in V (= A after sytrd)
// and tau.
template <typename T>
void ormtr(hipStream_t st, int n, const T* V, const T* tau, T* Z, OrmtrWork& w);

// ormtr for `batch` matrices (V + m sV, tau + m sTau, Z + m sZ); batches of
// more than one apply every reflector block to all entries with batched
// GEMMs.
template <typename T>
void ormtr_batched(hipStream_t st, int n, int batch, const T* V, int64_t sV, const T* tau,
                   int64_t sTau, T* Z, int64_t sZ, OrmtrWork& w);

// Z <- H_0 ... H_{nref-1} Z for explicit reflector columns V(:, j) (n x nref,
// ld n) that vanish above row j + off and are 1 there.
template <typename T>
void ormtr_blocks(hipStream_t st, int n, int nref, int off, const T* V, const T* tau, T* Z,
                  OrmtrWork& w);

// Two-stage reduction A = Q1 Q2 T Q2^T Q1^T (A, n x n full symmetric storage,
// is destroyed): d (n), e (n-1) of T; the reflectors of both stages stay in w
// for sy2tr_back.  n <= sy2tr_max_n().
template <typename T>
void sy2tr(hipStream_t st, int n, T* A, T* d, T* e, Sy2trWork& w);
// Z <- Q1 Q2 Z (Z n x n, ld n) with the reflectors of the last sy2tr call.
template <typename T>
void sy2tr_back(hipStream_t st, int n, T* Z, Sy2trWork& w, OrmtrWork& ow);
// Reads the bulge-chasing error flag (a dependency wait that timed out);
// synchronous.
bool sy2tr_failed(Sy2trWork& w);
int sy2tr_max_n();
// Largest n the one-stage tridiagonal reduction handles.
int sytrd_max_n();

}  // namespace msqrt
