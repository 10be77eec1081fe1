// Complex Schur decomposition and triangular solvers of the general path
// (Alg. 2): Hessenberg reduction, shifted QR, triangular square root and the
// triangular Sylvester solver.  All matrices are planar complex in the
// stacked layout (real rows 0..n-1, imaginary rows n..2n-1, ld = 2n).
#pragma once

#include "complex.hpp"
#include "factor.hpp"

namespace msqrt {

struct GehrdWork {
  DevBuf V, Tall, Y, W, W2, part, VT;
};

// H (stacked, n x n) is reduced in place to upper Hessenberg form
// H <- Q1^* H Q1 (entries below the subdiagonal are set to zero) and
// Q1 is formed explicitly in Z (stacked, n x n).
template <typename T>
void gehrd(hipStream_t st, int n, T* H, T* Z, GehrdWork& w);

// Real version for the real Schur route: H (n x n, ld n) <- Q1^T H Q1,
// Q1 formed in Z (n x n, ld n).
template <typename T>
void gehrd_real(hipStream_t st, int n, T* H, T* Z, GehrdWork& w);

struct HseqrWork {
  DevBuf U, shifts, flag, scratch;
};

// Complex Schur form by the shifted QR algorithm: H (upper Hessenberg,
// stacked) becomes upper triangular, Z <- Z U.  hnorm = ||H||_F (sets the
// norm-wise deflation floor).  Returns false if the iteration did not
// converge.
template <typename T>
bool hseqr(hipStream_t st, int n, T* H, T* Z, HseqrWork& w, T hnorm);

// Real Schur form by the Francis double-shift QR algorithm (real input on
// the general path): H (real upper Hessenberg, n x n, ld n) becomes
// quasi-upper-triangular with standardised 2x2 blocks, Z (n x n, ld n)
// <- Z U.  hnorm = ||H||_F.  Returns false if the iteration did not converge.
template <typename T>
bool rhseqr(hipStream_t st, int n, T* H, T* Z, HseqrWork& w, T hnorm);

// Tile boundaries (nt + 1 entries, first 0, last n) of a quasi-upper-
// triangular matrix of order n for the real tile solvers: every 32 rows, one
// row earlier where a boundary would separate the two rows of a 2x2 block.
// sub[i] != 0 marks a nonzero entry (i + 1, i).
std::vector<int> quasi_partition(int n, const unsigned char* sub);

// U = T^{1/2} (principal) for quasi-upper-triangular T (n x n, ld n), on the
// tiles of the device partition part (nt tiles); U may not alias T.  A
// diagonal block with an eigenvalue on or next to R<=0 sets the tile
// solvers' nonprincipal flag.
template <typename T>
void trsqrt_quasi(hipStream_t st, int n, const T* Tm, T* U, const int* part, int nt,
                  TrsylvWork& w);

// Solve S Y + Y S2 = C for quasi-upper-triangular S (m x m) and S2 (p x p)
// with their device tile partitions; C (m x p) is overwritten by Y.
template <typename T>
void trsyl_quasi(hipStream_t st, int m, int p, const T* S, int64_t lds, const int* rpart, int mt,
                 const T* S2, int64_t lds2, const int* cpart, int pt, T* C, int64_t ldc,
                 TrsylvWork& w);

// Error state of the tile solvers (sticky until trsylv_reset):
// timed_out = a dataflow wait timed out, nonprincipal = a diagonal entry of T
// on or next to R<=0.
void trsylv_reset(hipStream_t st, TrsylvWork& w);
void trsylv_errors(hipStream_t st, TrsylvWork& w, int* timed_out, int* nonprincipal);

// S = T^{1/2} (principal) for upper triangular T (stacked, n x n); S may not
// alias T.  Returns false if a diagonal entry of T lies on R<=0.
template <typename T>
void trsqrt(hipStream_t st, int n, const T* Tm, T* S, TrsylvWork& w, int* bad);

// U = T^{1/3} (principal) for upper triangular T (stacked, n x n), with
// workspaces UT (U^T) and V (U^2) of the same shape; *bad (device) becomes
// nonzero if a diagonal entry of T lies on R<=0.  U may not alias T.
template <typename T>
void trcbrt(hipStream_t st, int n, const T* Tm, T* U, T* UT, T* V, int* bad);

// Solve S Y + Y S2 = C (S m x m, S2 p x p upper triangular; C m x p,
// overwritten by Y); all stacked with their own leading dimensions.
template <typename T>
void trsyl(hipStream_t st, int m, int p, const T* S, int64_t lds, const T* S2, int64_t lds2, T* C,
           int64_t ldc, TrsylvWork& w);

}  // namespace msqrt
