// Instantiations of the MFMA GEMM for the products of the refinement loop.
#include "gemm.hpp"
#include "kernels.hpp"

namespace msqrt {

void gemm_store_f32(hipStream_t st, bool ta, bool tb, int M, int N, int K, const float* A,
                    int64_t lda, int64_t sA, const float* B, int64_t ldb, int64_t sB, float* C,
                    int64_t ldc, int64_t sC, float alpha, float beta, int batch, bool tri,
                    bool split) {
  GemmShape s = make_shape(M, N, K, lda, ldb, sA, sB, tri);
  EpiStore<float> e{C, ldc, sC, alpha, beta};
  launch_gemm<float>(st, ta, tb, s, A, B, e, nullptr, batch, split);
}

void gemm_store_f64(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A,
                    int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double* C,
                    int64_t ldc, int64_t sC, double alpha, double beta, int batch, bool tri) {
  GemmShape s = make_shape(M, N, K, lda, ldb, sA, sB, tri);
  EpiStore<double> e{C, ldc, sC, alpha, beta};
  launch_gemm<double>(st, ta, tb, s, A, B, e, nullptr, batch);
}

template <typename T>
void gemm_store_splitk(hipStream_t st, bool ta, bool tb, int M, int N, int K, int K_last,
                       const T* A, int64_t lda, int64_t sA, const T* B, int64_t ldb, int64_t sB,
                       T* C, int64_t ldc, int64_t sC, int splits) {
  GemmShape s = make_shape(M, N, K, lda, ldb, sA, sB, false);
  s.K_last = K_last;
  EpiStore<T> e{C, ldc, sC, T(1), T(0)};
  launch_gemm<T>(st, ta, tb, s, A, B, e, nullptr, splits);
}
template void gemm_store_splitk<float>(hipStream_t, bool, bool, int, int, int, int, const float*,
                                       int64_t, int64_t, const float*, int64_t, int64_t, float*,
                                       int64_t, int64_t, int);
template void gemm_store_splitk<double>(hipStream_t, bool, bool, int, int, int, int, const double*,
                                        int64_t, int64_t, const double*, int64_t, int64_t, double*,
                                        int64_t, int64_t, int);

int gemm_residual(hipStream_t st, int n, const double* X, int64_t ldx, int64_t sX,
                  const double* A, int64_t lda, int64_t sA, const double* ascale, float* Rl,
                  double* R64, int64_t ldr, int64_t sR, double* partials, int batch, bool sym) {
  // For symmetric X, X X = X X^T and only the lower triangle of tiles is
  // computed (the epilogue mirrors it), halving the float64 flops.
  GemmShape s = make_shape(n, n, n, ldx, ldx, sX, sX, sym);
  if (Rl) {
    EpiResidual e{A, lda, sA, ascale, Rl, ldr, sR};
    return launch_gemm<double>(st, false, sym, s, X, X, e, partials, batch);
  }
  EpiResidual64 e{A, lda, sA, ascale, R64, ldr, sR};
  return launch_gemm<double>(st, false, sym, s, X, X, e, partials, batch);
}

int gemm_residual_general(hipStream_t st, int n, const double* Xa, int64_t lda_, int64_t sXa,
                          const double* Xb, int64_t ldb_, int64_t sXb, const double* C,
                          int64_t ldc, int64_t sC, float* Rl, double* R64, int64_t ldr, int64_t sR,
                          double* partials, int batch) {
  GemmShape s = make_shape(n, n, n, lda_, ldb_, sXa, sXb, false);
  if (Rl) {
    EpiResidual e{C, ldc, sC, nullptr, Rl, ldr, sR};
    return launch_gemm<double>(st, false, false, s, Xa, Xb, e, partials, batch);
  }
  EpiResidual64 e{C, ldc, sC, nullptr, R64, ldr, sR};
  return launch_gemm<double>(st, false, false, s, Xa, Xb, e, partials, batch);
}

int gemm_residual_ex(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A,
                     int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
                     const double* C, int64_t ldc, int64_t sC, const double* cscale, float* Rl,
                     double* R64, int64_t ldr, int64_t sR, double* partials, int batch) {
  GemmShape s = make_shape(M, N, K, lda, ldb, sA, sB, false);
  if (Rl) {
    EpiResidual e{C, ldc, sC, cscale, Rl, ldr, sR};
    return launch_gemm<double>(st, ta, tb, s, A, B, e, partials, batch);
  }
  EpiResidual64 e{C, ldc, sC, cscale, R64, ldr, sR};
  return launch_gemm<double>(st, ta, tb, s, A, B, e, partials, batch);
}

template <typename T>
void gemm_diagsylv(hipStream_t st, bool ta, bool tb, int n, const T* A, int64_t lda, int64_t sA,
                   const T* B, int64_t ldb, int64_t sB, const T* s, int64_t sS, T* Y, int64_t ldy,
                   int64_t sY, int batch, bool tri, bool split) {
  GemmShape sh = make_shape(n, n, n, lda, ldb, sA, sB, tri);
  EpiDiagSylv<T> e{s, sS, Y, ldy, sY};
  launch_gemm<T>(st, ta, tb, sh, A, B, e, nullptr, batch, split);
}

template <typename T>
void gemm_update(hipStream_t st, bool ta, bool tb, int n, int K, const T* A, int64_t lda,
                 int64_t sA, const T* B, int64_t ldb, int64_t sB, double* X, int64_t ldx,
                 int64_t sX, const int* active, int batch, bool tri, bool split) {
  GemmShape sh = make_shape(n, n, K, lda, ldb, sA, sB, tri);
  EpiUpdate<T> e{X, ldx, sX, active};
  launch_gemm<T>(st, ta, tb, sh, A, B, e, nullptr, batch, split);
}

template <typename T>
void gemm_set_f64(hipStream_t st, bool ta, bool tb, int n, int K, const T* A, int64_t lda,
                  int64_t sA, const T* B, int64_t ldb, int64_t sB, double* X, int64_t ldx,
                  int64_t sX, int batch, bool tri, bool split) {
  GemmShape sh = make_shape(n, n, K, lda, ldb, sA, sB, tri);
  EpiSetF64<T> e{X, ldx, sX};
  launch_gemm<T>(st, ta, tb, sh, A, B, e, nullptr, batch, split);
}

#define MSQRT_INST(T)                                                                          \
  template void gemm_diagsylv<T>(hipStream_t, bool, bool, int, const T*, int64_t, int64_t,     \
                                 const T*, int64_t, int64_t, const T*, int64_t, T*, int64_t,   \
                                 int64_t, int, bool, bool);                                    \
  template void gemm_update<T>(hipStream_t, bool, bool, int, int, const T*, int64_t, int64_t,  \
                               const T*, int64_t, int64_t, double*, int64_t, int64_t,          \
                               const int*, int, bool, bool);                                   \
  template void gemm_set_f64<T>(hipStream_t, bool, bool, int, int, const T*, int64_t, int64_t, \
                                const T*, int64_t, int64_t, double*, int64_t, int64_t, int,    \
                                bool, bool);
MSQRT_INST(float)
MSQRT_INST(double)
#undef MSQRT_INST

}  // namespace msqrt
