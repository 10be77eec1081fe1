// Test hooks of the general-path stages (include/msqrt_testing.h): host
// interleaved complex128 in, stage run on the device in complex64 or
// complex128, host interleaved complex128 out.
#include <cmath>
#include <algorithm>
#include <vector>

#include "../../include/msqrt_testing.h"
#include "kernels.hpp"
#include "schur.hpp"

using namespace msqrt;

namespace {

// interleaved (ld = rows) -> stacked (ld = 2 * rows) in precision T
template <typename T>
std::vector<T> to_stacked_host(int64_t rows, int64_t cols, const double* A) {
  std::vector<T> s(2 * rows * cols);
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i) {
      s[i + j * 2 * rows] = (T)A[2 * (i + j * rows)];
      s[rows + i + j * 2 * rows] = (T)A[2 * (i + j * rows) + 1];
    }
  return s;
}
template <typename T>
void from_stacked_host(int64_t rows, int64_t cols, const std::vector<T>& s, double* A) {
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i) {
      A[2 * (i + j * rows)] = (double)s[i + j * 2 * rows];
      A[2 * (i + j * rows) + 1] = (double)s[rows + i + j * 2 * rows];
    }
}
template <typename T>
T* upload(DevBuf& b, const std::vector<T>& h) {
  T* d = b.ensure<T>((int64_t)h.size());
  MSQRT_HIP(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return d;
}
template <typename T>
std::vector<T> download(const T* d, size_t cnt) {
  std::vector<T> h(cnt);
  MSQRT_HIP(hipMemcpy(h.data(), d, sizeof(T) * cnt, hipMemcpyDeviceToHost));
  return h;
}

template <typename T>
msqrt_status gehrd_impl(int n, const double* A, double* H, double* Q, bool schur) {
  DevBuf hb, qb;
  T* dH = upload(hb, to_stacked_host<T>(n, n, A));
  T* dQ = qb.ensure<T>(2 * (int64_t)n * n);
  GehrdWork gw;
  gehrd<T>(nullptr, n, dH, dQ, gw);
  if (schur) {
    HseqrWork hw;
    double fro = 0.0;
    for (size_t k = 0; k < 2 * (size_t)n * n; ++k) fro += A[k] * A[k];
    if (!hseqr<T>(nullptr, n, dH, dQ, hw, (T)std::sqrt(fro))) {
      set_last_error("complex Schur QR did not converge");
      return MSQRT_ERR_NOT_CONVERGED;
    }
  }
  MSQRT_HIP(hipDeviceSynchronize());
  from_stacked_host<T>(n, n, download(dH, 2 * (size_t)n * n), H);
  from_stacked_host<T>(n, n, download(dQ, 2 * (size_t)n * n), Q);
  return MSQRT_OK;
}

template <typename T>
msqrt_status trcbrt_impl(int n, const double* Tm, double* U) {
  DevBuf tb, ub, utb, vb, fb;
  T* dT = upload(tb, to_stacked_host<T>(n, n, Tm));
  T* dU = ub.ensure<T>(2 * (int64_t)n * n);
  T* dUT = utb.ensure<T>(2 * (int64_t)n * n);
  T* dV = vb.ensure<T>(2 * (int64_t)n * n);
  int* bad = fb.ensure<int>(1);
  trcbrt<T>(nullptr, n, dT, dU, dUT, dV, bad);
  MSQRT_HIP(hipDeviceSynchronize());
  int hbad = 0;
  MSQRT_HIP(hipMemcpy(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost));
  if (hbad) {
    set_last_error("a diagonal entry lies on the closed negative real axis");
    return MSQRT_ERR_NO_PRINCIPAL;
  }
  from_stacked_host<T>(n, n, download(dU, 2 * (size_t)n * n), U);
  return MSQRT_OK;
}

template <typename T>
msqrt_status trsqrt_impl(int n, const double* Tm, double* S) {
  DevBuf tb, sb;
  T* dT = upload(tb, to_stacked_host<T>(n, n, Tm));
  T* dS = sb.ensure<T>(2 * (int64_t)n * n);
  TrsylvWork tw;
  trsylv_reset(nullptr, tw);
  trsqrt<T>(nullptr, n, dT, dS, tw, nullptr);
  int to = 0, np = 0;
  trsylv_errors(nullptr, tw, &to, &np);
  if (to) throw Error{MSQRT_ERR_DEVICE, "dataflow wait timed out"};
  from_stacked_host<T>(n, n, download(dS, 2 * (size_t)n * n), S);
  if (np) {
    set_last_error("an eigenvalue lies on or next to the closed negative real axis");
    return MSQRT_ERR_NO_PRINCIPAL;
  }
  return MSQRT_OK;
}

template <typename T>
msqrt_status trsyl_impl(int m, int p, const double* S, const double* S2, const double* C,
                        double* Y) {
  DevBuf sb, s2b, cb;
  T* dS = upload(sb, to_stacked_host<T>(m, m, S));
  T* dS2 = upload(s2b, to_stacked_host<T>(p, p, S2));
  T* dC = upload(cb, to_stacked_host<T>(m, p, C));
  TrsylvWork tw;
  trsylv_reset(nullptr, tw);
  trsyl<T>(nullptr, m, p, dS, 2 * (int64_t)m, dS2, 2 * (int64_t)p, dC, 2 * (int64_t)m, tw);
  int to = 0;
  trsylv_errors(nullptr, tw, &to, nullptr);
  if (to) throw Error{MSQRT_ERR_DEVICE, "dataflow wait timed out"};
  from_stacked_host<T>(m, p, download(dC, 2 * (size_t)m * p), Y);
  return MSQRT_OK;
}

template <class F>
msqrt_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return (msqrt_status)e.status;
  } catch (...) {
    set_last_error("unknown error");
    return MSQRT_ERR_DEVICE;
  }
}

}  // namespace

extern "C" msqrt_status msqrt_test_gehrd(msqrt_prec prec, int64_t n, const double* A, double* H,
                                         double* Q) {
  if (n < 1 || !A || !H || !Q || n > 16384) return MSQRT_ERR_INVALID_ARG;
  return guarded([&] {
    if (prec == MSQRT_PREC_FP64) return gehrd_impl<double>((int)n, A, H, Q, false);
    if (prec == MSQRT_PREC_FP32) return gehrd_impl<float>((int)n, A, H, Q, false);
    return MSQRT_ERR_INVALID_ARG;
  });
}

extern "C" msqrt_status msqrt_test_schur(msqrt_prec prec, int64_t n, const double* A, double* T,
                                         double* Q) {
  if (n < 1 || !A || !T || !Q || n > 16384) return MSQRT_ERR_INVALID_ARG;
  return guarded([&] {
    if (prec == MSQRT_PREC_FP64) return gehrd_impl<double>((int)n, A, T, Q, true);
    if (prec == MSQRT_PREC_FP32) return gehrd_impl<float>((int)n, A, T, Q, true);
    return MSQRT_ERR_INVALID_ARG;
  });
}

extern "C" msqrt_status msqrt_test_trsqrt(msqrt_prec prec, int64_t n, const double* Tm, double* S) {
  if (n < 1 || !Tm || !S || n > 16384) return MSQRT_ERR_INVALID_ARG;
  return guarded([&] {
    if (prec == MSQRT_PREC_FP64) return trsqrt_impl<double>((int)n, Tm, S);
    if (prec == MSQRT_PREC_FP32) return trsqrt_impl<float>((int)n, Tm, S);
    return MSQRT_ERR_INVALID_ARG;
  });
}

extern "C" msqrt_status msqrt_test_trcbrt(msqrt_prec prec, int64_t n, const double* Tm, double* U) {
  if (n < 1 || !Tm || !U || n > 16384) return MSQRT_ERR_INVALID_ARG;
  return guarded([&] {
    if (prec == MSQRT_PREC_FP64) return trcbrt_impl<double>((int)n, Tm, U);
    if (prec == MSQRT_PREC_FP32) return trcbrt_impl<float>((int)n, Tm, U);
    return MSQRT_ERR_INVALID_ARG;
  });
}

extern "C" msqrt_status msqrt_test_trsyl(msqrt_prec prec, int64_t m, int64_t p, const double* S,
                                         const double* S2, const double* C, double* Y) {
  if (m < 1 || p < 1 || !S || !S2 || !C || !Y || m > 16384 || p > 16384)
    return MSQRT_ERR_INVALID_ARG;
  return guarded([&] {
    if (prec == MSQRT_PREC_FP64) return trsyl_impl<double>((int)m, (int)p, S, S2, C, Y);
    if (prec == MSQRT_PREC_FP32) return trsyl_impl<float>((int)m, (int)p, S, S2, C, Y);
    return MSQRT_ERR_INVALID_ARG;
  });
}

extern "C" msqrt_status msqrt_test_gemm_f32(int split, int ta, int tb, int64_t M, int64_t N,
                                            int64_t K, const float* A, const float* B, float* C) {
  if (M < 1 || N < 1 || K < 0 || !A || !B || !C || M > 65536 || N > 65536 || K > 65536)
    return MSQRT_ERR_INVALID_ARG;
  return guarded([&] {
    DevBuf ab, bb, cb;
    const size_t na = (size_t)M * K, nb = (size_t)K * N, nc = (size_t)M * N;
    float* dA = ab.ensure<float>((int64_t)na + 1);
    float* dB = bb.ensure<float>((int64_t)nb + 1);
    float* dC = cb.ensure<float>((int64_t)nc);
    MSQRT_HIP(hipMemcpy(dA, A, sizeof(float) * na, hipMemcpyHostToDevice));
    MSQRT_HIP(hipMemcpy(dB, B, sizeof(float) * nb, hipMemcpyHostToDevice));
    const int64_t lda = ta ? K : M, ldb = tb ? N : K;
    gemm_store_f32(nullptr, ta != 0, tb != 0, (int)M, (int)N, (int)K, dA, std::max<int64_t>(lda, 1),
                   0, dB, std::max<int64_t>(ldb, 1), 0, dC, M, 0, 1.f, 0.f, 1, false, split != 0);
    MSQRT_HIP(hipDeviceSynchronize());
    MSQRT_HIP(hipMemcpy(C, dC, sizeof(float) * nc, hipMemcpyDeviceToHost));
    return MSQRT_OK;
  });
}

extern "C" msqrt_status msqrt_test_syrk(msqrt_prec prec, int64_t n, int64_t k, const void* A,
                                        void* C) {
  if (n < 1 || k < 0 || !A || !C || n > 65536 || k > 65536 ||
      (prec != MSQRT_PREC_FP32 && prec != MSQRT_PREC_FP64))
    return MSQRT_ERR_INVALID_ARG;
  return guarded([&] {
    const size_t es = prec == MSQRT_PREC_FP64 ? 8 : 4;
    const size_t na = (size_t)n * k, nc = (size_t)n * n;
    DevBuf ab, cb;
    void* dA = ab.ensure<unsigned char>((int64_t)(es * na + 8));
    void* dC = cb.ensure<unsigned char>((int64_t)(es * nc));
    MSQRT_HIP(hipMemcpy(dA, A, es * na, hipMemcpyHostToDevice));
    const int64_t ld = std::max<int64_t>(n, 1);
    // lower-triangle tiles only, the epilogue mirrors each element
    if (prec == MSQRT_PREC_FP64)
      gemm_store_f64(nullptr, false, true, (int)n, (int)n, (int)k, (const double*)dA, ld, 0,
                     (const double*)dA, ld, 0, (double*)dC, n, 0, 1.0, 0.0, 1, true);
    else
      gemm_store_f32(nullptr, false, true, (int)n, (int)n, (int)k, (const float*)dA, ld, 0,
                     (const float*)dA, ld, 0, (float*)dC, n, 0, 1.f, 0.f, 1, true, false);
    MSQRT_HIP(hipDeviceSynchronize());
    MSQRT_HIP(hipMemcpy(C, dC, es * nc, hipMemcpyDeviceToHost));
    return MSQRT_OK;
  });
}
