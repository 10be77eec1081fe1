/*
 * msqrt learned precision selector: matrix features, the small network that
 * predicts the refinement step count per factor precision, its training
 * kernels, and the installed selector used by MSQRT_PREC_AUTO.
 *
 * The paper observes that the number of corrections grows with the
 * conditioning of A and that the iteration diverges when the low precision
 * is too low for it (Sec. 5, the Hilbert experiments; Sec. 3.2, the rate
 * estimates); the selector learns this relation from the method's own
 * outcomes.  A wrong prediction costs time only: msqrt_sqrtm still judges
 * every answer with the float64 residual and escalates on failure.
 *
 * Network: 16 -> 64 (ReLU) -> 64 (ReLU) -> 3 (linear), float32, 5443
 * parameters in one vector: W1 (64 x 16, row-major), b1 (64), W2 (64 x 64),
 * b2 (64), W3 (3 x 64), b3 (3).  Outputs: log(1 + y) for the predicted
 * corrections y with a BF16SPLIT, FP32, FP64 factor (a failed run is
 * labelled y = maxit + 10); the runtime decodes with expm1.
 *
 * All pointers named d* are device pointers; work is ordered on `stream`.
 */
#ifndef MSQRT_SELECTOR_H
#define MSQRT_SELECTOR_H

#include "msqrt.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MSQRT_SEL_NFEAT 16
#define MSQRT_SEL_NPARAM 5443
#define MSQRT_SEL_NCOST 42

/* The 16 O(n^2) features of A (layout and dtype as in msqrt_sqrtm) into
 * dF[16] (float): log2 n / 10; exact symmetry flag; log10 departure from
 * symmetry; log10 of the largest and smallest |a_ii| relative to the rms
 * entry; fraction of Re a_ii <= 0; the smallest Gershgorin margin
 * (Re a_ii - r_i) / rms as g / (1 + |g|); fraction of Gershgorin discs
 * reaching Re <= 0; log10 of the row and column 2-norm ranges; log10 of
 * ||A||_1 / ||A||_F and ||A||_inf / ||A||_F; log10(1 + n ||A||_F^2 /
 * |tr A|^2); Re tr(A^2) / ||A||_F^2; Re tr A / (sqrt(n) ||A||_F); log10 of
 * the diagonal magnitude range.  Errors: INVALID_ARG. */
msqrt_status msqrt_features(msqrt_dtype dtype, int64_t n, const void* dA, int64_t lda, float* dF,
                            hipStream_t stream);

/* Network outputs dOut[batch x 3] for inputs dX[batch x 16] (row-major). */
msqrt_status msqrt_mlp_forward(int64_t batch, const float* dX, const float* dP, float* dOut,
                               hipStream_t stream);

/* Mean squared error over the batch and the 3 outputs against dY[batch x 3]
 * into dLoss[0], and its gradient with respect to the parameters into
 * dGrad[5443] (fixed summation order: reproducible). */
msqrt_status msqrt_mlp_grad(int64_t batch, const float* dX, const float* dY, const float* dP,
                            float* dGrad, float* dLoss, hipStream_t stream);

/* One Adam step (bias-corrected, step >= 1) on dP with moments dM, dV. */
msqrt_status msqrt_mlp_adam(const float* dGrad, float* dP, float* dM, float* dV, int step,
                            float lr, float beta1, float beta2, float eps, hipStream_t stream);

/* Installs the selector used by MSQRT_PREC_AUTO (host arrays, copied):
 * params[5443]; the feature normalisation x = (f - mean) / scale; and the
 * cost model cost[42]: for structure s (0 = HPD, 1 = general) and quantity
 * q (0..2 factorisation with BF16SPLIT / FP32 / FP64, 3..5 one correction
 * with each, 6 one residual) the milliseconds c3 n^3 + c2 n^2 + c0 at
 * cost[(7 s + q) * 3 + {0, 1, 2}].  The choice is the precision p that
 * minimises fac_p + (y_p + 1) res + y_p sweep_p for the predicted y_p;
 * msqrt_info.predicted_steps holds the decoded y_p. */
msqrt_status msqrt_selector_set(const float* params, const float* feat_mean,
                                const float* feat_scale, const double* cost, int ncost);

/* Reads a selector file written by the training driver: the 8 bytes
 * "MSQSEL01", int32 nparam, nfeat, ncost, then float32 params, mean, scale
 * and float64 cost (little-endian).  Errors: INVALID_ARG (missing or
 * malformed file). */
msqrt_status msqrt_selector_load(const char* path);

/* Removes the installed selector (AUTO then means FP32). */
void msqrt_selector_clear(void);

/* 1 if a selector is installed. */
int msqrt_selector_installed(void);

#ifdef __cplusplus
}
#endif

#endif /* MSQRT_SELECTOR_H */
