// Host-side launchers of the msqrt HIP kernels.  All launchers are
// asynchronous on the given stream and throw msqrt::Error on launch failure.
#pragma once

#include "common.hpp"

namespace msqrt {

// ---- elementwise / reductions (elementwise.hip) ---------------------------

// Per batch entry b: flags[b] bit0 = non-finite element, bit1 = not exactly
// symmetric; partials[b * nblk + blk] = sum of squares.  Returns nblk.
int launch_validate(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA, int batch,
                    int check_sym, int* flags, double* partials);
// Real representation E = [[Re A, -Im A], [Im A, Re A]] (2n x 2n, ld 2n,
// batch stride sE) of interleaved complex A (ld lda in complex elements).
void launch_embed_complex(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA,
                          double* E, int64_t sE, int batch);
// Inverse of launch_embed_complex, averaging the two copies of each part.
void launch_extract_complex(hipStream_t st, int n, const double* E, int64_t sE, double* X,
                            int64_t ldx, int64_t sX, int batch);
// p[i] = v for i < count.
void launch_fill_i32(hipStream_t st, int* p, int count, int v);
// out[b] = sqrt(sum_{t < count} partials[b * count + t]) (fixed summation order).
void launch_reduce_sqrt(hipStream_t st, const double* partials, int count, int batch, double* out);
// B = scale[b] * A (double source, float or double destination).
void launch_cast_scale_f64_f32(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA,
                               const double* scale, float* B, int64_t ldb, int64_t sB, int batch);
void launch_cast_scale_f64_f64(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA,
                               const double* scale, double* B, int64_t ldb, int64_t sB, int batch);
// W(:, j) = Q(:, j) * s[j]   (T = float or double)
template <typename T>
void launch_scale_cols(hipStream_t st, int n, const T* Q, int64_t ldq, int64_t sQ, const T* s,
                       int64_t sS, T* W, int64_t ldw, int64_t sW, int batch);
// X *= scale[b] (double, in place)
void launch_scale_inplace(hipStream_t st, int n, double* X, int64_t ldx, int64_t sX,
                          const double* scale, int batch);
// Copies / casts between matrices with leading dimensions.
void launch_copy_f64(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA, double* B,
                     int64_t ldb, int64_t sB, int batch);

// ---- GEMMs (gemm.hip) -----------------------------------------------------

// C = alpha op(A) op(B)   (+ beta C)
// split = true: BF16-split products (hi*hi + hi*lo + lo*hi, float accumulation)
void gemm_store_f32(hipStream_t st, bool ta, bool tb, int M, int N, int K, const float* A,
                    int64_t lda, int64_t sA, const float* B, int64_t ldb, int64_t sB, float* C,
                    int64_t ldc, int64_t sC, float alpha, float beta, int batch, bool tri,
                    bool split = false);
void gemm_store_f64(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A,
                    int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double* C,
                    int64_t ldc, int64_t sC, double alpha, double beta, int batch, bool tri);
// Split-K partial products: C_b = op(A_b) op(B_b) with A_b = A + b*sA,
// B_b = B + b*sB, C_b = C + b*sC, K for every entry but the last (K_last).
template <typename T>
void gemm_store_splitk(hipStream_t st, bool ta, bool tb, int M, int N, int K, int K_last,
                       const T* A, int64_t lda, int64_t sA, const T* B, int64_t ldb, int64_t sB,
                       T* C, int64_t ldc, int64_t sC, int splits);
// Residual R = ascale * A - X X (float64); writes R as float (Rl) or double
// (R64), partials[b * ntiles + tile] = sum of R^2.  Returns ntiles.
int gemm_residual(hipStream_t st, int n, const double* X, int64_t ldx, int64_t sX,
                  const double* A, int64_t lda, int64_t sA, const double* ascale, float* Rl,
                  double* R64, int64_t ldr, int64_t sR, double* partials, int batch, bool sym);
// R = C - Xa Xb (general product, float64); R as float (Rl) or double (R64),
// partials[b * ntiles + tile] = sum of R^2.  Returns ntiles.
int gemm_residual_general(hipStream_t st, int n, const double* Xa, int64_t lda, int64_t sXa,
                          const double* Xb, int64_t ldb, int64_t sXb, const double* C,
                          int64_t ldc, int64_t sC, float* Rl, double* R64, int64_t ldr, int64_t sR,
                          double* partials, int batch);
// R_b = cscale[b] C_b - op(A_b) op(B_b) (float64, M x N, inner K); R as float
// (Rl) or double (R64); partials[b * ntiles + tile] = sum of R^2.  Returns
// ntiles.
int gemm_residual_ex(hipStream_t st, bool ta, bool tb, int M, int N, int K, const double* A,
                     int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
                     const double* C, int64_t ldc, int64_t sC, const double* cscale, float* Rl,
                     double* R64, int64_t ldr, int64_t sR, double* partials, int batch);
// Y = (op(A) op(B)) ./ (s_i + s_j)
template <typename T>
void gemm_diagsylv(hipStream_t st, bool ta, bool tb, int n, const T* A, int64_t lda, int64_t sA,
                   const T* B, int64_t ldb, int64_t sB, const T* s, int64_t sS, T* Y, int64_t ldy,
                   int64_t sY, int batch, bool tri, bool split = false);
// X += fl64(op(A) op(B))
template <typename T>
void gemm_update(hipStream_t st, bool ta, bool tb, int n, int K, const T* A, int64_t lda,
                 int64_t sA, const T* B, int64_t ldb, int64_t sB, double* X, int64_t ldx,
                 int64_t sX, const int* active, int batch, bool tri, bool split = false);
// X = fl64(op(A) op(B))
template <typename T>
void gemm_set_f64(hipStream_t st, bool ta, bool tb, int n, int K, const T* A, int64_t lda,
                  int64_t sA, const T* B, int64_t ldb, int64_t sB, double* X, int64_t ldx,
                  int64_t sX, int batch, bool tri, bool split = false);

}  // namespace msqrt
