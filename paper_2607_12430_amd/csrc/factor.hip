// Factorisation driver: validation, scaling, structure detection and the
// low-precision Schur / spectral decomposition of Alg. 2 / Alg. 3.
#include <cmath>

#include "factor.hpp"
#include "kernels.hpp"

namespace msqrt {

msqrt_status build_factor(Factor* f, const msqrt_options& o, const double* A, int64_t lda,
                          int64_t sA, hipStream_t st, PhaseTimer* tm) {
  (void)o; (void)A; (void)lda; (void)sA; (void)st; (void)tm; (void)f;
  throw Error{MSQRT_ERR_UNSUPPORTED, "on-device factorisation is not available in this build"};
}

msqrt_prec select_precision(const msqrt_options& o, msqrt_dtype dtype, int64_t n, const void* A,
                            int64_t lda, int64_t sA, hipStream_t st, msqrt_info* info,
                            PhaseTimer& tm) {
  (void)o; (void)dtype; (void)n; (void)A; (void)lda; (void)sA; (void)st; (void)info; (void)tm;
  return MSQRT_PREC_FP32;
}

msqrt_status backward(Factor* f, const double* X, int64_t ldx, const double* Gbar, int64_t ldgb,
                      double* G, int64_t ldg, int64_t stride, int maxit, double tol,
                      hipStream_t st, msqrt_info* info, PhaseTimer& tm) {
  (void)f; (void)X; (void)ldx; (void)Gbar; (void)ldgb; (void)G; (void)ldg; (void)stride;
  (void)maxit; (void)tol; (void)st; (void)info; (void)tm;
  throw Error{MSQRT_ERR_UNSUPPORTED, "backward is not available in this build"};
}

}  // namespace msqrt
