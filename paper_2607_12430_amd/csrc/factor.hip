// Factorisation driver: validation, scaling, structure detection and the
// low-precision Schur / spectral decomposition of Alg. 2 / Alg. 3.
#include <cmath>
#include <vector>

#include "factor.hpp"
#include "kernels.hpp"
#include "tridiag.hpp"
#include "../../include/msqrt_testing.h"

namespace msqrt {

namespace {

// s_i = sqrt(lam_i) in the factor precision and min lam (float64), for
// batch entry blockIdx.x (lam, s: n per entry).
template <typename T>
__global__ __launch_bounds__(256) void finish_hpd_kernel(int n, const double* lam, T* s,
                                                         double* minlam) {
  lam += (int64_t)blockIdx.x * n;
  s += (int64_t)blockIdx.x * n;
  minlam += blockIdx.x;
  __shared__ double red[4];
  double mn = INFINITY;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double l = lam[i];
    mn = fmin(mn, l);
    s[i] = (T)sqrt(fmax(l, 0.0));
  }
  mn = -block_max(-mn, red);
  if (threadIdx.x == 0) *minlam = mn;
}

// The two-stage reduction replaces one grid synchronisation per column by
// MFMA panel updates and a pipelined bulge chase.  It is selected from this
// size on (above every supported size: the one-stage kernel is currently the
// faster one at all sizes; the two-stage route is reached through its test
// hook).
constexpr int kTwoStageMinN = 1 << 30;
inline bool use_two_stage(int n) { return n >= kTwoStageMinN && n <= sy2tr_max_n(); }

template <typename T>
void factor_hpd(Factor* f, const double* A, int64_t lda, int64_t sA, hipStream_t st,
                PhaseTimer* tm, std::vector<double>& minlam) {
  const int n = (int)f->n, batch = (int)f->batch;
  const int64_t nn = (int64_t)n * n;
  T* Q = f->Q.ensure<T>(nn * batch);
  T* S = f->S.ensure<T>((int64_t)n * batch);
  // all batch entries are cast, tridiagonalised, diagonalised and
  // back-transformed together (the two-stage route runs entry by entry)
  const int64_t sD = 3 * (int64_t)n + 8;
  T* Aw = f->fw1.ensure<T>(nn * batch);
  T* d = f->fw2.ensure<T>(sD * batch);
  double* lam = f->fw3.ensure<double>((int64_t)n * batch + 8);
  double* mins = f->fw4.ensure<double>(batch);
  SytrdWork sw;
  Sy2trWork tw;
  StedcWork ew;
  OrmtrWork ow;
  const bool two = use_two_stage(n);
  if (tm) tm->begin(MSQRT_T_REDUCE);
  if (std::is_same<T, float>::value)
    launch_cast_scale_f64_f32(st, n, A, lda, sA, f->ascale_dev(), (float*)Aw, n, nn, batch);
  else
    launch_cast_scale_f64_f64(st, n, A, lda, sA, f->ascale_dev(), (double*)Aw, n, nn, batch);
  if (two) {
    for (int b = 0; b < batch; ++b) {
      T* db = d + b * sD;
      if (tm) tm->begin(MSQRT_T_REDUCE);
      sy2tr<T>(st, n, Aw + b * nn, db, db + n, tw);
      if (tm) tm->begin(MSQRT_T_EIG);
      stedc<T>(st, n, db, db + n, lam + (int64_t)b * n, Q + b * nn, ew);
      if (tm) tm->begin(MSQRT_T_BACK);
      sy2tr_back<T>(st, n, Q + b * nn, tw, ow);
    }
  } else {
    sytrd_batched<T>(st, n, batch, Aw, nn, d, d + n, d + 2 * n, sD, sw);
    if (tm) tm->begin(MSQRT_T_EIG);
    stedc_batched<T>(st, n, batch, d, d + n, sD, lam, Q, ew);
  }
  hipLaunchKernelGGL(finish_hpd_kernel<T>, dim3(batch), dim3(256), 0, st, n, (const double*)lam, S,
                     mins);
  MSQRT_LAUNCH_CHECK();
  if (!two) {
    if (tm) tm->begin(MSQRT_T_BACK);
    ormtr_batched<T>(st, n, batch, Aw, nn, d + 2 * n, sD, Q, nn, ow);
  }
  if (tm) tm->end();
  minlam.resize(batch);
  MSQRT_HIP(hipMemcpyAsync(minlam.data(), mins, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipStreamSynchronize(st));
  if (tm) tm->collect();
  if (two && sy2tr_failed(tw))
    throw Error{MSQRT_ERR_DEVICE, "band reduction: a bulge-chasing dependency wait timed out"};
  if (sytrd_failed(sw))
    throw Error{MSQRT_ERR_DEVICE, "tridiagonal reduction: grid barrier timed out"};
}

}  // namespace

msqrt_status build_factor(Factor* f, const msqrt_options& o, const double* A, int64_t lda,
                          int64_t sA, hipStream_t st, PhaseTimer* tm) {
  if (o.prec != MSQRT_PREC_FP32 && o.prec != MSQRT_PREC_FP64 && o.prec != MSQRT_PREC_BF16SPLIT) {
    set_last_error("invalid precision");
    return MSQRT_ERR_INVALID_ARG;
  }
  const bool cplx = f->dtype == MSQRT_COMPLEX128;
  f->real_schur = false;
  if (cplx && o.structure == MSQRT_STRUCT_HPD) {
    set_last_error("complex Hermitian input runs on the general path (structure AUTO or GENERAL)");
    return MSQRT_ERR_UNSUPPORTED;
  }
  if (tm) tm->begin(MSQRT_T_VALIDATE);
  int flags;
  if (cplx) {
    if (f->batch != 1) {
      set_last_error("the general path takes one matrix per call (batch = 1)");
      return MSQRT_ERR_UNSUPPORTED;
    }
    flags = analyse_input_general(f, A, lda, 1, st) | 2;
  } else {
    const bool want_sym_check = o.structure != MSQRT_STRUCT_GENERAL;
    flags = analyse_input(f, A, lda, sA, want_sym_check, st);
    if (!want_sym_check) flags |= 2;
  }
  if (tm) tm->end();
  if (flags & 1) {
    set_last_error("input contains Inf or NaN");
    return MSQRT_ERR_NONFINITE;
  }
  msqrt_struct sc = o.structure;
  if (sc == MSQRT_STRUCT_AUTO) sc = (flags & 2) ? MSQRT_STRUCT_GENERAL : MSQRT_STRUCT_HPD;
  if (sc == MSQRT_STRUCT_HPD && (flags & 2)) {
    set_last_error("structure HPD requested but the input is not exactly symmetric");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (sc == MSQRT_STRUCT_HPD && f->n > sytrd_max_n()) {
    // Beyond the tridiagonal reduction's size limit a symmetric input takes
    // the general path when the caller left the structure open.
    if (o.structure != MSQRT_STRUCT_AUTO || f->batch != 1) {
      set_last_error("the symmetric route supports n <= " + std::to_string(sytrd_max_n()) +
                     " (larger single inputs run on the general path with structure AUTO)");
      return MSQRT_ERR_UNSUPPORTED;
    }
    sc = MSQRT_STRUCT_GENERAL;
  }
  f->structure = sc;
  // BF16SPLIT keeps the float factorisation; only the refinement's
  // Schur-basis products differ
  f->prec = o.prec;
  if (sc == MSQRT_STRUCT_GENERAL) {
    if (f->batch != 1) {
      set_last_error("the general path takes one matrix per call (batch = 1)");
      return MSQRT_ERR_UNSUPPORTED;
    }
    if (!cplx && o.real_schur) {
      if (f->prec == MSQRT_PREC_FP64) return factor_real<double>(f, A, lda, st, tm);
      return factor_real<float>(f, A, lda, st, tm);
    }
    f->real_schur = false;
    if (f->prec == MSQRT_PREC_FP64) return factor_general<double>(f, A, lda, cplx ? 1 : 0, st, tm);
    return factor_general<float>(f, A, lda, cplx ? 1 : 0, st, tm);
  }
  std::vector<double> minlam;
  if (f->prec == MSQRT_PREC_FP64) factor_hpd<double>(f, A, lda, sA, st, tm, minlam);
  else factor_hpd<float>(f, A, lda, sA, st, tm, minlam);
  for (double l : minlam)
    if (!(l > 0.0)) {
      set_last_error("a computed eigenvalue is not positive in this precision");
      return MSQRT_ERR_NO_PRINCIPAL;
    }
  return MSQRT_OK;
}

}  // namespace msqrt

// ---------------------------------------------------------------------------
// Test hooks (include/msqrt_testing.h).

using namespace msqrt;

namespace {
template <typename T>
void test_sytrd_impl(int n, const void* A, void* d, void* e, void* tau) {
  DevBuf a, dd;
  T* da = a.ensure<T>((int64_t)n * n);
  T* dv = dd.ensure<T>(3 * (int64_t)n + 8);
  MSQRT_HIP(hipMemcpy(da, A, sizeof(T) * n * n, hipMemcpyHostToDevice));
  SytrdWork sw;
  sytrd<T>(nullptr, n, da, dv, dv + n, dv + 2 * n, sw);
  MSQRT_HIP(hipDeviceSynchronize());
  MSQRT_HIP(hipMemcpy(d, dv, sizeof(T) * n, hipMemcpyDeviceToHost));
  if (n > 1) {
    MSQRT_HIP(hipMemcpy(e, dv + n, sizeof(T) * (n - 1), hipMemcpyDeviceToHost));
    MSQRT_HIP(hipMemcpy(tau, dv + 2 * n, sizeof(T) * (n - 1), hipMemcpyDeviceToHost));
  }
  if (sytrd_failed(sw)) throw Error{MSQRT_ERR_DEVICE, "grid barrier timed out"};
}
template <typename T>
void test_sy2tr_impl(int n, const void* A, void* d, void* e, void* Q) {
  if (n > sy2tr_max_n()) throw Error{MSQRT_ERR_UNSUPPORTED, "n too large for the two-stage reduction"};
  DevBuf a, dd, q;
  T* da = a.ensure<T>((int64_t)n * n);
  T* dv = dd.ensure<T>(2 * (int64_t)n + 8);
  T* dq = q.ensure<T>((int64_t)n * n);
  MSQRT_HIP(hipMemcpy(da, A, sizeof(T) * n * n, hipMemcpyHostToDevice));
  std::vector<T> eye((size_t)n * n, T(0));
  for (int i = 0; i < n; ++i) eye[(size_t)i * n + i] = T(1);
  MSQRT_HIP(hipMemcpy(dq, eye.data(), sizeof(T) * n * n, hipMemcpyHostToDevice));
  Sy2trWork tw;
  OrmtrWork ow;
  sy2tr<T>(nullptr, n, da, dv, dv + n, tw);
  sy2tr_back<T>(nullptr, n, dq, tw, ow);
  MSQRT_HIP(hipDeviceSynchronize());
  if (sy2tr_failed(tw)) throw Error{MSQRT_ERR_DEVICE, "bulge-chasing dependency wait timed out"};
  MSQRT_HIP(hipMemcpy(d, dv, sizeof(T) * n, hipMemcpyDeviceToHost));
  if (n > 1) MSQRT_HIP(hipMemcpy(e, dv + n, sizeof(T) * (n - 1), hipMemcpyDeviceToHost));
  MSQRT_HIP(hipMemcpy(Q, dq, sizeof(T) * n * n, hipMemcpyDeviceToHost));
}
template <typename T>
void test_stedc_impl(int n, const void* d, const void* e, double* lam, void* Z) {
  DevBuf dd, z, l;
  T* dv = dd.ensure<T>(2 * (int64_t)n + 8);
  T* dz = z.ensure<T>((int64_t)n * n);
  double* dl = l.ensure<double>(n);
  MSQRT_HIP(hipMemcpy(dv, d, sizeof(T) * n, hipMemcpyHostToDevice));
  if (n > 1) MSQRT_HIP(hipMemcpy(dv + n, e, sizeof(T) * (n - 1), hipMemcpyHostToDevice));
  StedcWork ew;
  stedc<T>(nullptr, n, dv, dv + n, dl, dz, ew);
  MSQRT_HIP(hipDeviceSynchronize());
  MSQRT_HIP(hipMemcpy(lam, dl, sizeof(double) * n, hipMemcpyDeviceToHost));
  MSQRT_HIP(hipMemcpy(Z, dz, sizeof(T) * n * n, hipMemcpyDeviceToHost));
}
}  // namespace

extern "C" msqrt_status msqrt_test_sytrd(msqrt_prec prec, int64_t n, const void* A, void* d,
                                         void* e, void* tau) {
  try {
    if (n < 1 || !A || !d || !e || !tau) return MSQRT_ERR_INVALID_ARG;
    if (prec == MSQRT_PREC_FP64) test_sytrd_impl<double>((int)n, A, d, e, tau);
    else if (prec == MSQRT_PREC_FP32) test_sytrd_impl<float>((int)n, A, d, e, tau);
    else return MSQRT_ERR_INVALID_ARG;
    return MSQRT_OK;
  } catch (const Error& err) {
    set_last_error(err.msg);
    return (msqrt_status)err.status;
  }
}

extern "C" msqrt_status msqrt_test_sy2tr(msqrt_prec prec, int64_t n, const void* A, void* d,
                                         void* e, void* Q) {
  try {
    if (n < 1 || !A || !d || !e || !Q) return MSQRT_ERR_INVALID_ARG;
    if (prec == MSQRT_PREC_FP64) test_sy2tr_impl<double>((int)n, A, d, e, Q);
    else if (prec == MSQRT_PREC_FP32) test_sy2tr_impl<float>((int)n, A, d, e, Q);
    else return MSQRT_ERR_INVALID_ARG;
    return MSQRT_OK;
  } catch (const Error& err) {
    set_last_error(err.msg);
    return (msqrt_status)err.status;
  }
}

extern "C" msqrt_status msqrt_test_stedc(msqrt_prec prec, int64_t n, const void* d, const void* e,
                                         double* lam, void* Z) {
  try {
    if (n < 1 || !d || !lam || !Z) return MSQRT_ERR_INVALID_ARG;
    if (prec == MSQRT_PREC_FP64) test_stedc_impl<double>((int)n, d, e, lam, Z);
    else if (prec == MSQRT_PREC_FP32) test_stedc_impl<float>((int)n, d, e, lam, Z);
    else return MSQRT_ERR_INVALID_ARG;
    return MSQRT_OK;
  } catch (const Error& err) {
    set_last_error(err.msg);
    return (msqrt_status)err.status;
  }
}
