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

/* Divide-and-conquer eigensolver of the tridiagonal (d, e): lam (n, double,
 * ascending) and the eigenvector matrix Z (n x n column-major, prec). */
msqrt_status msqrt_test_stedc(msqrt_prec prec, int64_t n, const void* d, const void* e,
                              double* lam, void* Z);

#ifdef __cplusplus
}
#endif

#endif /* MSQRT_TESTING_H */
