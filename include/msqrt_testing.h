/*
 * msqrt test hooks: entry points that run one stage of the on-device
 * spectral decomposition in isolation, for the test suite.  Not part of the
 * solver API in msqrt.h.  Host buffers in, host buffers out; the call
 * allocates its own device memory and synchronises the device before
 * returning.  prec is MSQRT_PREC_FP32 (float buffers) or MSQRT_PREC_FP64
 * (double buffers).  Errors as in msqrt.h.
 */
#ifndef MSQRT_TESTING_H
#define MSQRT_TESTING_H

#include "msqrt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Householder tridiagonalisation of the symmetric n x n column-major A:
 * writes the diagonal d (n) and off-diagonal e (n-1), and tau (n-1). */
msqrt_status msqrt_test_sytrd(msqrt_prec prec, int64_t n, const void* A, void* d, void* e,
                              void* tau);

/* Two-stage tridiagonalisation A = Q T Q^T (dense -> band -> tridiagonal) of
 * the symmetric n x n column-major A (n <= 4104): the diagonal d (n) and
 * off-diagonal e (n-1) of T, and Q (n x n column-major) formed by the
 * back-transformation applied to the identity.  Errors: INVALID_ARG,
 * UNSUPPORTED (n too large), DEVICE (a dependency wait timed out). */
msqrt_status msqrt_test_sy2tr(msqrt_prec prec, int64_t n, const void* A, void* d, void* e,
                              void* Q);

/* Divide-and-conquer eigensolver of the tridiagonal (d, e): lam (n, double,
 * ascending) and the eigenvector matrix Z (n x n column-major, prec). */
msqrt_status msqrt_test_stedc(msqrt_prec prec, int64_t n, const void* d, const void* e,
                              double* lam, void* Z);

/* The stages of the general path (Alg. 2) work on complex matrices; their
 * hooks take and return interleaved complex128 (double re, im pairs),
 * column-major with ld = n, and run the stage in complex64 (FP32) or
 * complex128 (FP64) arithmetic. */

/* Householder reduction to upper Hessenberg form: A = Q H Q^*, H with exact
 * zeros below the subdiagonal (first line of Alg. 2, the start of the Schur
 * decomposition). */
msqrt_status msqrt_test_gehrd(msqrt_prec prec, int64_t n, const double* A, double* H, double* Q);

/* Complex Schur decomposition A = Q T Q^* (Hessenberg reduction followed by
 * the shifted QR algorithm); T upper triangular. */
msqrt_status msqrt_test_schur(msqrt_prec prec, int64_t n, const double* A, double* T, double* Q);

/* Principal square root S of the upper triangular T (Eq. (subst), blocked);
 * NO_PRINCIPAL if a diagonal entry lies on or next to R<=0. */
msqrt_status msqrt_test_trsqrt(msqrt_prec prec, int64_t n, const double* T, double* S);

/* Principal cube root U of the upper triangular T (U^3 = T, Sec. 4 with
 * p = 3), interleaved complex host buffers, computed on the device in the
 * precision `prec`; NO_PRINCIPAL if a diagonal entry lies on R<=0. */
msqrt_status msqrt_test_trcbrt(msqrt_prec prec, int64_t n, const double* T, double* U);

/* Triangular Sylvester equation S Y + Y S2 = C (Eq. (triangsylv), Alg. 1):
 * S m x m and S2 p x p upper triangular, C and Y m x p. */
msqrt_status msqrt_test_trsyl(msqrt_prec prec, int64_t m, int64_t p, const double* S,
                              const double* S2, const double* C, double* Y);

/* The float GEMM of the Schur-basis transforms: C = op(A) op(B), M x N,
 * inner dimension K, column-major float buffers (op = transpose when ta/tb is
 * set; A is M x K or K x M, B is K x N or N x K, ld = rows as stored).
 * split = 0: float MFMA products; split = 1: BF16-split products
 * (hi*hi + hi*lo + lo*hi with float accumulation, the BF16SPLIT precision). */
msqrt_status msqrt_test_gemm_f32(int split, int ta, int tb, int64_t M, int64_t N, int64_t K,
                                 const float* A, const float* B, float* C);

/* The symmetric-output GEMM of the refinement (lower-triangle tiles, each
 * element mirrored by the epilogue): C = A A^T for A n x k column-major in
 * float (prec FP32) or double (prec FP64); C is n x n.  Large triangles take
 * the 192 x 192-tile kernels. */
msqrt_status msqrt_test_syrk(msqrt_prec prec, int64_t n, int64_t k, const void* A, void* C);

#ifdef __cplusplus
}
#endif

#endif /* MSQRT_TESTING_H */
