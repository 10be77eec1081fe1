// Symmetric spectral decomposition on the GPU: Householder tridiagonalisation,
// divide-and-conquer tridiagonal eigensolver, back-transformation.
#pragma once

#include "factor.hpp"

namespace msqrt {

struct SytrdWork {
  DevBuf VW, WV, ypart, sp, vp, bar;
};

struct StedcWork {
  DevBuf dd, ee, lam, Z2, M, meta, rot, roots, zhat, scal;
};

struct OrmtrWork {
  DevBuf gram, VT, Wpart, W;
};

// A (n x n, ld n, full symmetric) is overwritten: column j holds the explicit
// reflector v_j (rows j+1..n-1, v_j(j+1) = 1, zeros above) for rows >= its
// panel start.  d (n), e (n-1), tau (n-1) in the factor precision.
template <typename T>
void sytrd(hipStream_t st, int n, T* A, T* d, T* e, T* tau, SytrdWork& w);

// Eigen-decomposition of the symmetric tridiagonal (d, e): lam ascending
// (float64) and eigenvectors Z (n x n, ld n, precision T).
template <typename T>
void stedc(hipStream_t st, int n, const T* d, const T* e, double* lam, T* Z, StedcWork& w);

// Z <- H_0 H_1 ... H_{n-2} Z with the reflectors left in V (= A after sytrd)
// and tau.
template <typename T>
void ormtr(hipStream_t st, int n, const T* V, const T* tau, T* Z, OrmtrWork& w);

}  // namespace msqrt
