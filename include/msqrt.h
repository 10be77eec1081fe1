/*
 * msqrt -- mixed-precision principal matrix square root on AMD MI355X (gfx950).
 *
 * Problem (Sec. 1 of Gao, Kressner, Shao): for A in C^{n x n} (or R^{n x n})
 * with no eigenvalue on the closed negative real axis, compute the principal
 * square root X = A^{1/2}: the unique X with X^2 = A whose eigenvalues lie in
 * the open right half-plane.
 *
 * Method (Sec. 2, Alg. 2 and Alg. 3): a low-precision Schur factorisation
 * A ~ Q T Q^*, S = T^{1/2}, X_0 = Q S Q^*, then approximate-Newton refinement:
 * every sweep forms the working-precision residual R = A - X_k^2, stops when
 * ||R||_F <= tol ||A||_F, otherwise transforms R to the Schur basis
 * (Q^* R Q, low precision), solves S Y + Y S = Q^* R Q (Eq. (triangsylv); for
 * symmetric positive definite A the equation is diagonal,
 * y_ij = r_ij / (s_i + s_j)), and adds X_{k+1} = X_k + Q Y Q^* in working
 * precision.
 *
 * Conventions shared by every entry point:
 *  - Matrices are column-major device buffers; element (i, j) of matrix b of a
 *    batch is at ptr[b * stride + i + j * ld], ld >= n.  Because the square
 *    root of A^T is the transpose of the square root of A (and the adjoint
 *    equation transposes the same way), a row-major buffer may be passed
 *    unchanged: the result is then row-major too.
 *  - MSQRT_REAL64 buffers hold double; MSQRT_COMPLEX128 buffers hold
 *    interleaved (re, im) double pairs.
 *  - The caller owns every buffer it passes.  Input buffers are never
 *    modified.  Buffers must stay valid until the call returns.
 *  - All work is ordered on `stream` (a hipStream_t; NULL = the default
 *    stream).  Calls are blocking: the convergence test reads back one scalar
 *    per sweep.  A factor handle must not be used from two threads at once.
 *  - Every call returns a status and never aborts.  On NOT_CONVERGED or
 *    DIVERGED the output holds the iterate with the smallest residual seen and
 *    `info` holds the residual history.
 */
#ifndef MSQRT_H
#define MSQRT_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msqrt_factor_s* msqrt_factor_t; /* opaque, library-owned */

typedef enum {
  MSQRT_OK = 0,
  MSQRT_ERR_INVALID_ARG = 1,   /* bad size, pointer, stride or option */
  MSQRT_ERR_NONFINITE = 2,     /* A (or Gbar) holds Inf or NaN */
  MSQRT_ERR_NO_PRINCIPAL = 3,  /* an eigenvalue lies on or next to R<=0 even in FP64 */
  MSQRT_ERR_NOT_CONVERGED = 4, /* maxit reached or the residual stagnated */
  MSQRT_ERR_DIVERGED = 5,      /* residual grew; output = best iterate */
  MSQRT_ERR_DEVICE = 6,        /* a HIP runtime call failed */
  MSQRT_ERR_OUT_OF_MEMORY = 7,
  MSQRT_ERR_UNSUPPORTED = 8    /* combination not implemented (see message) */
} msqrt_status;

typedef enum { MSQRT_REAL64 = 0, MSQRT_COMPLEX128 = 1 } msqrt_dtype; /* working precision */

/* Precision of the Schur factorisation and of the Schur-basis transforms.
 * BF16SPLIT: transforms as two-term bfloat16 splits with float32 accumulation
 * (factorisation in FP32).  AUTO: the learned selector picks per input. */
typedef enum {
  MSQRT_PREC_AUTO = 0,
  MSQRT_PREC_BF16SPLIT = 1,
  MSQRT_PREC_FP32 = 2,
  MSQRT_PREC_FP64 = 3
} msqrt_prec;

/* AUTO tests for exact symmetry (Hermitian symmetry for complex input) and then
 * uses Alg. 3; a non-positive low-precision eigenvalue escalates the
 * precision, and one that FP64 also sees means the symmetric input has no
 * principal root (MSQRT_ERR_NO_PRINCIPAL).  Complex Hermitian input is solved
 * through its real representation [[Re A, -Im A], [Im A, Re A]] (symmetric,
 * positive definite exactly when A is; the representation maps sqrt(A) to
 * the root of that matrix), so the factor of a complex HPD input is the real
 * HPD factor of order 2n.  The symmetric route's tridiagonal reduction
 * handles order <= 4225 (real n <= 4225, complex n <= 2112): a larger
 * single input takes the general path under AUTO, and HPD (or a batch)
 * beyond that size returns MSQRT_ERR_UNSUPPORTED. */
typedef enum { MSQRT_STRUCT_AUTO = 0, MSQRT_STRUCT_GENERAL = 1, MSQRT_STRUCT_HPD = 2 } msqrt_struct;

typedef struct {
  msqrt_prec prec;        /* default MSQRT_PREC_FP32 */
  msqrt_struct structure; /* default MSQRT_STRUCT_AUTO */
  int maxit;              /* maximum number of corrections, default 30 */
  double tol;             /* stop when ||A - X^2||_F <= tol ||A||_F, default 1e-13;
                             tol < 0 nullifies the stopping test (see msqrt_refine) */
  int blks;               /* minimal block size of the triangular solvers, default 32 */
  int fallback;           /* 1: escalate BF16SPLIT -> FP32 -> FP64 on failure (default) */
  int64_t batch;          /* number of matrices, default 1 */
  int real_schur;         /* real input on the general path: 1 = real Schur form
                             A = Q T Q^T with quasi-triangular T (1x1 and 2x2 diagonal
                             blocks, remark on real input in Sec. 2.2.1), default;
                             0 = complex Schur form (Alg. 2 as printed) */
} msqrt_options;

typedef struct {
  int steps;                 /* corrections applied (max over the batch) */
  double relres;             /* final ||A - X^2||_F / ||A||_F (max over the batch) */
  double relres_hist[64];    /* residual after 0, 1, ... corrections (first matrix) */
  int nhist;                 /* entries of relres_hist in use */
  msqrt_prec prec_used;      /* precision of the factor that produced X */
  msqrt_struct struct_used;  /* HPD or GENERAL */
  int fallbacks;             /* number of precision escalations */
  int scale_exp;             /* k of the exact scaling A / 4^k */
  float predicted_steps[3];  /* selector prediction for BF16SPLIT, FP32, FP64 (AUTO only) */
  float t_ms[12];            /* phase timers, see MSQRT_T_* */
} msqrt_info;

enum {
  MSQRT_T_VALIDATE = 0, /* finiteness, symmetry, norm, scaling */
  MSQRT_T_SELECT = 1,   /* selector features + inference */
  MSQRT_T_REDUCE = 2,   /* tridiagonal / Hessenberg reduction */
  MSQRT_T_EIG = 3,      /* tridiagonal eigensolver / Schur QR */
  MSQRT_T_BACK = 4,     /* back-transformation of the Schur vectors */
  MSQRT_T_X0 = 5,       /* triangular root and X_0 */
  MSQRT_T_RESIDUAL = 6, /* all residual evaluations */
  MSQRT_T_TRANSFORM = 7,/* Q^* R Q, including the SPD diagonal solve */
  MSQRT_T_SOLVE = 8,    /* triangular Sylvester solves (general path) */
  MSQRT_T_UPDATE = 9,   /* Q Y Q^* and the working-precision update */
  MSQRT_T_TOTAL = 10
};

/* Fills *opt with the defaults listed in msqrt_options. */
void msqrt_default_options(msqrt_options* opt);

/* Low-precision Schur factorisation of A (the factorisation steps of Alg. 2 and Alg. 3):
 * HPD input -> spectral decomposition A/4^k ~ Q diag(s^2) Q^*;
 * general input -> complex Schur form A/4^k ~ Q T Q^*, S = T^{1/2}; real general input
 * with opt->real_schur (default) -> real Schur form A/4^k ~ Q T Q^T, T quasi-upper-
 * triangular with standardised 2x2 blocks for complex conjugate pairs, S = T^{1/2}
 * quasi-upper-triangular (remark on real input in Sec. 2.2.1), and the refinement's
 * Sylvester solves run on tiles that never cut a 2x2 block.
 * The precision is opt->prec (AUTO picks one).  On success *out owns Q, S, the
 * scale exponent k and workspaces; release it with msqrt_factor_destroy.
 * Errors: INVALID_ARG (n < 0, ld < n, NULL pointer with n > 0), NONFINITE,
 * NO_PRINCIPAL (eigenvalue on R<=0 in this precision), OUT_OF_MEMORY, DEVICE. */
msqrt_status msqrt_factor(const msqrt_options* opt, msqrt_dtype dtype, int64_t n, const void* dA,
                          int64_t lda, int64_t strideA, hipStream_t stream, msqrt_factor_t* out);

/* Approximate-Newton refinement with a frozen factor (Alg. 2/3 loop, Sec. 2.1):
 * X <- X + Q Y Q^*, S Y + Y S = Q^* (A - X^2) Q, until the relative residual is
 * <= tol or maxit corrections were applied.  With init_from_factor != 0, X is
 * first overwritten by X_0 = Q S Q^*; otherwise the caller's X is the start
 * (it may be the root of a nearby matrix).  Never escalates the precision.
 * dA/dX layout as above; A must be the matrix the factor was built from or a
 * nearby one of the same size and structure.  With an HPD factor, A and a
 * caller-supplied X must be exactly symmetric (the residual is formed as
 * A - X X^T from one triangle): otherwise MSQRT_ERR_INVALID_ARG, with X
 * untouched.  Inf or NaN in A (or in the caller-supplied X of an HPD
 * factor): MSQRT_ERR_NONFINITE.  tol < 0 nullifies the stopping test, as in
 * the paper's accuracy experiments (Sec. 5.1): exactly maxit corrections are
 * applied, every residual is recorded in info, X is the last iterate and the
 * status is MSQRT_OK (a non-finite residual still ends the loop as
 * MSQRT_ERR_DIVERGED).  tol = NaN: MSQRT_ERR_INVALID_ARG. */
msqrt_status msqrt_refine(msqrt_factor_t f, const void* dA, int64_t lda, int64_t strideA,
                          void* dX, int64_t ldx, int64_t strideX, int init_from_factor, int maxit,
                          double tol, hipStream_t stream, msqrt_info* info);

/* msqrt_refine for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as msqrt_refine, for HPD factors
 * (other factors: MSQRT_ERR_UNSUPPORTED).  Every device buffer the call needs
 * beyond A, X and the factor lives in one static 64 MiB device array per GPU
 * (held until the process ends); the call performs no hipMalloc / hipFree.
 * It needs batch * n^2 * (2 * e + 8) bytes plus a few KiB, e = 4 (FP32 or
 * BF16SPLIT factor) or 8 (FP64 factor): about n <= 2040 (FP32) or n <= 1670
 * (FP64) for one matrix; larger sizes return MSQRT_ERR_INVALID_ARG before
 * any device work.  All calls on one GPU share that array, so calls that
 * overlap in time on one GPU (other threads, other streams) race and must
 * not be issued.  Phase timers are not recorded (info->t_ms stays zero). */
msqrt_status msqrt_refine_noalloc(msqrt_factor_t f, const void* dA, int64_t lda, int64_t strideA,
                                  void* dX, int64_t ldx, int64_t strideX, int init_from_factor,
                                  int maxit, double tol, hipStream_t stream, msqrt_info* info);

/* Complete solve: factor, X_0, refinement, with precision escalation when
 * opt->fallback is set: a BF16SPLIT run that does not converge repeats the
 * refinement with float transforms on the same (float) factor; a float run
 * that fails, or a float factorisation without a principal root, is redone
 * with an FP64 factor.  If keep != NULL the factor is returned for reuse
 * (e.g. by msqrt_sqrtm_backward); otherwise it is freed. */
msqrt_status msqrt_sqrtm(const msqrt_options* opt, msqrt_dtype dtype, int64_t n, const void* dA,
                         int64_t lda, int64_t strideA, void* dX, int64_t ldx, int64_t strideX,
                         hipStream_t stream, msqrt_info* info, msqrt_factor_t* keep);

/* Principal matrix p-th root (Sec. 4): the unique X with X^p = A whose
 * eigenvalues lie in |arg z| < pi/p, for A with no eigenvalue on R<=0.
 * p = 2 is msqrt_sqrtm for one matrix.  p = 3 runs the Sec. 4 framework on
 * the general path: low-precision complex Schur form of A/8^k, U = T^{1/3}
 * (the Schur method for p-th roots), X_0 = Q U Q^*, then corrections from
 * S^2 Y + S Y S + Y S^2 = Q^* fl_l(A - X^3) Q (S = U) with the residual and
 * update in working precision, X <- 2^k X on exit; real input returns the
 * real root.  opt->prec FP64 selects a float64 factor, anything else float32
 * (escalated to FP64 when opt->fallback is set and the float run fails);
 * opt->batch must be 1; maxit, tol (tol < 0: nullified stop) as for
 * msqrt_sqrtm.  Other p: MSQRT_ERR_UNSUPPORTED.  Buffers, streams and errors
 * as above (ld in elements). */
msqrt_status msqrt_rootm(const msqrt_options* opt, int p, msqrt_dtype dtype, int64_t n,
                         const void* dA, int64_t lda, void* dX, int64_t ldx, hipStream_t stream,
                         msqrt_info* info);

/* Reverse-mode derivative of X = sqrtm(A): given Gbar = dL/dX, returns
 * G = dL/dA, the solution of X^* G + G X^* = Gbar (adjoint of the Frechet
 * derivative; for HPD input X G + G X = Gbar).  Solved in the factor's Schur
 * basis in low precision and refined with working-precision residuals, the
 * same framework as the forward solve.  dX must be the root returned for the
 * factor's matrix; all three buffers use `stride` between batch entries. */
msqrt_status msqrt_sqrtm_backward(msqrt_factor_t f, const void* dX, int64_t ldx,
                                  const void* dGbar, int64_t ldgb, void* dG, int64_t ldg,
                                  int64_t stride, int maxit, double tol, hipStream_t stream,
                                  msqrt_info* info);

/* Releases a factor and its device memory.  NULL is ignored. */
void msqrt_factor_destroy(msqrt_factor_t f);

/* Human-readable name of a status code (static storage). */
const char* msqrt_status_string(msqrt_status s);

/* Last error message recorded by the calling thread (static storage). */
const char* msqrt_last_error(void);

/* Frees what the library caches between calls: the pool of device
 * allocations released by finished calls and destroyed factors, the timing
 * events of msqrt_profile_*, and the selector's device copy.  Call it when no
 * library call is in flight (later calls allocate again); it gives an ordered
 * shutdown while the HIP runtime is still up (the Python binding calls it at
 * interpreter exit).  Live factors keep their memory. */
void msqrt_release_cached(void);

/* Kernel-class timing for measurement tools.  msqrt_profile_enable(1) clears
 * the counters and starts recording a pair of hipEvents on the launch stream
 * around every launch of an instrumented kernel class ("gemm_f32",
 * "gemm_f64", "sytrd_panel_f32", "sytrd_panel_f64", ...), together with the
 * launch's algorithmic flop and byte counts; 0 stops recording.
 * msqrt_profile_query returns 0 and the accumulated launches, time (ms),
 * flops and bytes of one class (1 if the class was never launched).
 * msqrt_profile_list writes the comma-separated class names into buf and
 * returns the full length.  Querying waits for the recorded events. */
void msqrt_profile_enable(int on);
int msqrt_profile_query(const char* kernel_class, int64_t* launches, double* total_ms,
                        double* flops, double* bytes);
int msqrt_profile_list(char* buf, int buflen);

/* Test hook: builds a factor from caller-provided Q (n x n) and S (length n for
 * HPD, n x n upper triangular for GENERAL), column-major, in the precision
 * `prec` (FP32 buffers hold float / complex64, FP64 buffers double /
 * complex128).  on_device selects device or host pointers.  batch = 1. */
msqrt_status msqrt_factor_wrap(msqrt_prec prec, msqrt_struct structure, msqrt_dtype dtype,
                               int64_t n, const void* Q, const void* S, int on_device,
                               msqrt_factor_t* out);

/* Test hook: reads the factor's Q and S back to host buffers in the factor's
 * own precision (layout as in msqrt_factor_wrap; for a real-Schur general
 * factor Q and S are both real n x n, column-major); the scale exponent goes
 * to *scale_exp.  Either pointer may be NULL. */
msqrt_status msqrt_factor_export(msqrt_factor_t f, void* Q, void* S, int* scale_exp);

#ifdef __cplusplus
}
#endif

#endif /* MSQRT_H */
