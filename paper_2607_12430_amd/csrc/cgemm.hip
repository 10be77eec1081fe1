// Complex products over planar storage: four real MFMA GEMMs (float or
// double), accumulated through the epilogue's beta.
#include "complex.hpp"
#include "kernels.hpp"

namespace msqrt {

namespace {
template <typename T>
void rgemm(hipStream_t st, bool ta, bool tb, int M, int N, int K, const T* A, int64_t lda,
           const T* B, int64_t ldb, T* C, int64_t ldc, T alpha, T beta) {
  if (std::is_same<T, float>::value)
    gemm_store_f32(st, ta, tb, M, N, K, (const float*)A, lda, 0, (const float*)B, ldb, 0,
                   (float*)C, ldc, 0, (float)alpha, (float)beta, 1, false);
  else
    gemm_store_f64(st, ta, tb, M, N, K, (const double*)A, lda, 0, (const double*)B, ldb, 0,
                   (double*)C, ldc, 0, (double)alpha, (double)beta, 1, false);
}
}  // namespace

template <typename T>
void cgemm(hipStream_t st, char opA, char opB, int M, int N, int K, CMat<T> A, CMat<T> B,
           T alpha, T beta, CMat<T> C) {
  if (M <= 0 || N <= 0) return;
  const bool ta = opA != 'N', tb = opB != 'N';
  const T sa = opA == 'C' ? T(-1) : T(1), sb = opB == 'C' ? T(-1) : T(1);
  if (K <= 0) {
    rgemm<T>(st, false, false, M, N, 0, A.re, A.ld, B.re, B.ld, C.re, C.ld, T(0), beta);
    if (C.im) rgemm<T>(st, false, false, M, N, 0, A.re, A.ld, B.re, B.ld, C.im, C.ld, T(0), beta);
    return;
  }
  // Re C = alpha (Ar Br - sa sb Ai Bi) + beta Re C
  rgemm<T>(st, ta, tb, M, N, K, A.re, A.ld, B.re, B.ld, C.re, C.ld, alpha, beta);
  if (A.im && B.im)
    rgemm<T>(st, ta, tb, M, N, K, A.im, A.ld, B.im, B.ld, C.re, C.ld, -alpha * sa * sb, T(1));
  if (!C.im) return;
  // Im C = alpha (sb Ar Bi + sa Ai Br) + beta Im C
  bool first = true;
  if (B.im) {
    rgemm<T>(st, ta, tb, M, N, K, A.re, A.ld, B.im, B.ld, C.im, C.ld, alpha * sb, beta);
    first = false;
  }
  if (A.im) {
    rgemm<T>(st, ta, tb, M, N, K, A.im, A.ld, B.re, B.ld, C.im, C.ld, alpha * sa,
             first ? beta : T(1));
    first = false;
  }
  if (first) rgemm<T>(st, false, false, M, N, 0, A.re, A.ld, B.re, B.ld, C.im, C.ld, T(0), beta);
}

template void cgemm<float>(hipStream_t, char, char, int, int, int, CMat<float>, CMat<float>, float,
                           float, CMat<float>);
template void cgemm<double>(hipStream_t, char, char, int, int, int, CMat<double>, CMat<double>,
                            double, double, CMat<double>);

}  // namespace msqrt
