// Planar complex arithmetic for the general (complex Schur) path.
//
// Complex matrices live as two real planes.  Two layouts are used:
//   stacked: the real plane in rows 0..m-1 and the imaginary plane in rows
//            m..2m-1 of one column-major array with ld >= 2m, so that
//            [Re; Im] is itself a real 2m x n matrix;
//   wide:    the imaginary plane follows the real plane (Im = Re + ld * n),
//            so that [Re | Im] is a real m x 2n matrix.
// A complex product then becomes real MFMA GEMMs over the planes.
#pragma once

#include "common.hpp"

namespace msqrt {

template <typename T>
struct cx {
  T r, i;
};

template <typename T>
__host__ __device__ inline cx<T> cmk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ inline cx<T> cadd(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__host__ __device__ inline cx<T> csub(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
// conj(a) * b
template <typename T>
__host__ __device__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
template <typename T>
__host__ __device__ inline cx<T> cconj(cx<T> a) { return {a.r, -a.i}; }
template <typename T>
__host__ __device__ inline cx<T> cscale(cx<T> a, T s) { return {a.r * s, a.i * s}; }
template <typename T>
__host__ __device__ inline T cabs2(cx<T> a) { return a.r * a.r + a.i * a.i; }
template <typename T>
__device__ inline T cabs(cx<T> a) { return hypot(a.r, a.i); }
// a / b with scaling against overflow (Smith's algorithm).
template <typename T>
__device__ inline cx<T> cdiv(cx<T> a, cx<T> b) {
  if (fabs(b.r) >= fabs(b.i)) {
    const T q = b.i / b.r, d = b.r + b.i * q;
    return {(a.r + a.i * q) / d, (a.i - a.r * q) / d};
  }
  const T q = b.r / b.i, d = b.i + b.r * q;
  return {(a.r * q + a.i) / d, (a.i * q - a.r) / d};
}
// Principal square root by the half-angle formula: for z = x + iy,
// t = sqrt((|x| + |z|) / 2); x >= 0 -> (t, y / 2t), else (|y| / 2t, sign(y) t).
template <typename T>
__device__ inline cx<T> csqrt_principal(cx<T> z) {
  if (z.r == T(0) && z.i == T(0)) return {T(0), T(0)};
  const T t = sqrt((fabs(z.r) + hypot(z.r, z.i)) * T(0.5));
  if (z.r >= T(0)) return {t, z.i / (T(2) * t)};
  return {fabs(z.i) / (T(2) * t), copysign(t, z.i)};
}

// A complex matrix as two real planes with a common leading dimension.
template <typename T>
struct CMat {
  T* re;
  T* im;
  int64_t ld;
};
template <typename T>
inline CMat<T> stacked(T* base, int64_t m, int64_t ld) { return {base, base + m, ld}; }
template <typename T>
inline CMat<T> sub(CMat<T> a, int64_t i, int64_t j) {
  return {a.re + i + j * a.ld, a.im ? a.im + i + j * a.ld : nullptr, a.ld};
}

// C = alpha op(A) op(B) + beta C  (op: 'N', 'T' transpose, 'C' conjugate
// transpose); four real GEMMs over the planes.  A.im or B.im may be NULL for
// real operands.
template <typename T>
void cgemm(hipStream_t st, char opA, char opB, int M, int N, int K, CMat<T> A, CMat<T> B,
           T alpha, T beta, CMat<T> C);

// Elementwise helpers (general.hip).
template <typename T>
void launch_cset_identity(hipStream_t st, int n, CMat<T> A);

}  // namespace msqrt
