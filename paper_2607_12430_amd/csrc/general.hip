// General path (Alg. 2): complex Schur factorisation A/4^k ~ Q T Q^*, the
// triangular root S = T^{1/2}, X_0 = Q S Q^*, and the refinement
//   R = A - X^2 (float64),  Y = rtrsyl(S, S, Q^* fl(R) Q),  X += Q Y Q^*,
// plus the adjoint solve of the backward pass.  Real nonsymmetric input runs
// through the same complex route and returns Re X.
//
// Every complex product of the refinement is one batched real MFMA GEMM with
// an inner dimension of 2n: with the planes of Q stored in the four layouts
//   QSa = [-Qi; Qr; Qi], QSb = [Qi; Qr; -Qi]   (3n x n, stacked)
//   QWa = [Qi | Qr | -Qi], QWb = [-Qi | Qr | Qi] (n x 3n, wide)
// each product's real and imaginary parts are batch entries 0 and 1, e.g.
//   Re(R Q) = [Rr | Ri] [Qr; -Qi],  Im(R Q) = [Rr | Ri] [Qi; Qr].
// The float64 iterate is kept wide (X = [Xr | Xi], n x 2n) and the residual
// product X X uses XS = [Xi; Xr; -Xi].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "factor.hpp"
#include "kernels.hpp"
#include "schur.hpp"

namespace msqrt {

namespace {

constexpr int kRedBlocks = 256;

// Finiteness and sum of squares of a complex (interleaved) or real matrix.
__global__ __launch_bounds__(256) void cvalidate_kernel(int n, const double* A, int64_t lda, int cplx,
                                                        int* flags, double* part) {
  __shared__ double red[4];
  const int64_t cnt = (int64_t)n * n;
  double s = 0.0;
  int bad = 0;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < cnt;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x % n, j = x / n;
    if (cplx) {
      const double re = A[2 * (i + j * lda)], im = A[2 * (i + j * lda) + 1];
      if (!isfinite(re) || !isfinite(im)) bad = 1;
      s += re * re + im * im;
    } else {
      const double re = A[i + j * lda];
      if (!isfinite(re)) bad = 1;
      s += re * re;
    }
  }
  if (bad) atomicOr(flags, 1);
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// H (stacked, ld 2n) = scale * A in precision T.
template <typename T>
__global__ void to_stacked_kernel(int n, const double* A, int64_t lda, int cplx,
                                  const double* scale, T* H) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (int64_t)n * n) return;
  const int64_t i = x % n, j = x / n;
  const double s = *scale;
  double re, im = 0.0;
  if (cplx) { re = A[2 * (i + j * lda)]; im = A[2 * (i + j * lda) + 1]; }
  else re = A[i + j * lda];
  H[i + j * 2 * n] = (T)(re * s);
  H[n + i + j * 2 * n] = (T)(im * s);
}

template <typename T>
__global__ void q_variants_kernel(int n, const T* Q, T* QSa, T* QSb, T* QWa, T* QWb) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (x >= nn) return;
  const int64_t i = x % n, j = x / n;
  const T qr = Q[i + j * 2 * n], qi = Q[n + i + j * 2 * n];
  const int64_t l3 = 3 * (int64_t)n;
  QSa[i + j * l3] = -qi;
  QSa[n + i + j * l3] = qr;
  QSa[2 * n + i + j * l3] = qi;
  QSb[i + j * l3] = qi;
  QSb[n + i + j * l3] = qr;
  QSb[2 * n + i + j * l3] = -qi;
  QWa[i + j * n] = qi;
  QWa[nn + i + j * n] = qr;
  QWa[2 * nn + i + j * n] = -qi;
  QWb[i + j * n] = -qi;
  QWb[nn + i + j * n] = qr;
  QWb[2 * nn + i + j * n] = qi;
}

// XS = [Xi; Xr; -Xi] (ld 3n) from the wide X.
__global__ void x_stack_kernel(int n, const double* Xw, double* XS) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (x >= nn) return;
  const int64_t i = x % n, j = x / n;
  const double xr = Xw[i + j * n], xi = Xw[nn + i + j * n];
  const int64_t l3 = 3 * (int64_t)n;
  XS[i + j * l3] = xi;
  XS[n + i + j * l3] = xr;
  XS[2 * n + i + j * l3] = -xi;
}

// Wide float64 W = scale * op(X_user); op = identity or conjugate transpose.
__global__ void x_in_kernel(int n, const double* X, int64_t ldx, int cplx, int ctrans,
                            const double* scale, double* Xw) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (x >= nn) return;
  const int64_t i = x % n, j = x / n;
  const int64_t si = ctrans ? j : i, sj = ctrans ? i : j;
  const double s = scale ? *scale : 1.0;
  double re, im = 0.0;
  if (cplx) { re = X[2 * (si + sj * ldx)]; im = X[2 * (si + sj * ldx) + 1]; }
  else re = X[si + sj * ldx];
  if (ctrans) im = -im;
  Xw[i + j * n] = re * s;
  Xw[nn + i + j * n] = im * s;
}

// X_user = scale * op(Xw) (complex: interleaved; real: the real part) and
// partial sums of |X|^2 and |Im X|^2.
__global__ __launch_bounds__(256) void x_out_kernel(int n, const double* Xw, int cplx, int ctrans,
                                                    const double* scale, double* X, int64_t ldx,
                                                    double* part) {
  __shared__ double red[4];
  const int64_t nn = (int64_t)n * n;
  const double s = scale ? *scale : 1.0;
  double a2 = 0.0, i2 = 0.0;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nn;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x % n, j = x / n;
    const int64_t di = ctrans ? j : i, dj = ctrans ? i : j;
    const double re = Xw[i + j * n] * s;
    double im = Xw[nn + i + j * n] * s;
    if (ctrans) im = -im;
    a2 += re * re + im * im;
    i2 += im * im;
    if (cplx) {
      X[2 * (di + dj * ldx)] = re;
      X[2 * (di + dj * ldx) + 1] = im;
    } else {
      X[di + dj * ldx] = re;
    }
  }
  a2 = block_sum(a2, red);
  i2 = block_sum(i2, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a2;
    part[kRedBlocks + blockIdx.x] = i2;
  }
}

inline unsigned blocks_for(int64_t cnt) { return (unsigned)std::max<int64_t>(1, ceil_div(cnt, 256)); }

// ---- triangular cube root U = T^{1/3} (stacked, ld 2n), by superdiagonals.
// With V = U^2, entry (i, j), i < j, of U^3 = U V and V = U U give
//   (u_ii^2 + u_ii u_jj + u_jj^2) u_ij = t_ij - u_ii a_ij - b_ij,
//   v_ij = (u_ii + u_jj) u_ij + a_ij,
// a_ij = sum_{i<k<j} u_ik u_kj, b_ij = sum_{i<k<j} u_ik v_kj: every entry of
// superdiagonal d needs only superdiagonals < d, so a launch per superdiagonal
// computes all its entries at once (one wave per entry; UT = U^T holds the
// rows of U as contiguous columns).

template <typename T>
__device__ inline cx<T> sload(const T* M, int n, int i, int j) {
  const int64_t ld = 2 * (int64_t)n;
  return {M[i + j * ld], M[n + i + j * ld]};
}
template <typename T>
__device__ inline void sstore(T* M, int n, int i, int j, cx<T> v) {
  const int64_t ld = 2 * (int64_t)n;
  M[i + j * ld] = v.r;
  M[n + i + j * ld] = v.i;
}

template <typename T>
__global__ void trcbrt_diag_kernel(int n, const T* Tm, T* U, T* UT, T* V, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cx<T> t = sload(Tm, n, i, i);
  if (t.i == T(0) && t.r <= T(0)) atomicOr(bad, 1);
  // principal cube root |t|^{1/3} e^{i arg(t) / 3}
  const T r = cbrt(hypot(t.r, t.i));
  const T th = atan2(t.i, t.r) / T(3);
  const cx<T> u = {r * cos(th), r * sin(th)};
  sstore(U, n, i, i, u);
  sstore(UT, n, i, i, u);
  sstore(V, n, i, i, cmul(u, u));
}

template <typename T>
__global__ __launch_bounds__(256) void trcbrt_band_kernel(int n, int d, const T* Tm, T* U, T* UT,
                                                          T* V) {
  const int i = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x % kWave;
  const int j = i + d;
  if (j >= n) return;  // uniform over the wave
  cx<T> a = {T(0), T(0)}, b = {T(0), T(0)};
  for (int k = i + 1 + lane; k < j; k += kWave) {
    const cx<T> uik = sload(UT, n, k, i);
    a = cadd(a, cmul(uik, sload(U, n, k, j)));
    b = cadd(b, cmul(uik, sload(V, n, k, j)));
  }
  a.r = wave_sum(a.r);
  a.i = wave_sum(a.i);
  b.r = wave_sum(b.r);
  b.i = wave_sum(b.i);
  if (lane == 0) {
    const cx<T> ui = sload(U, n, i, i), uj = sload(U, n, j, j);
    const cx<T> den = cadd(cadd(cmul(ui, ui), cmul(ui, uj)), cmul(uj, uj));
    const cx<T> x = cdiv(csub(csub(sload(Tm, n, i, j), cmul(ui, a)), b), den);
    sstore(U, n, i, j, x);
    sstore(UT, n, j, i, x);
    sstore(V, n, i, j, cadd(cmul(cadd(ui, uj), x), a));
  }
}

// S2 = c S for the complex scalar c (stacked, n x n).
template <typename T>
__global__ void cscale_stacked_kernel(int n, const T* S, T cr, T ci, T* S2) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (int64_t)n * n) return;
  const int i = (int)(x % n), j = (int)(x / n);
  sstore(S2, n, i, j, cmul(sload(S, n, i, j), cx<T>{cr, ci}));
}

template <typename T>
void gstore_b(hipStream_t st, bool ta, bool tb, int n, int K, const T* A, int64_t lda, int64_t sA,
              const T* B, int64_t ldb, int64_t sB, T* C, int64_t ldc, int64_t sC,
              bool split = false) {
  if (std::is_same<T, float>::value)
    gemm_store_f32(st, ta, tb, n, n, K, (const float*)A, lda, sA, (const float*)B, ldb, sB,
                   (float*)C, ldc, sC, 1.f, 0.f, 2, false, split);
  else
    gemm_store_f64(st, ta, tb, n, n, K, (const double*)A, lda, sA, (const double*)B, ldb, sB,
                   (double*)C, ldc, sC, 1.0, 0.0, 2, false);
}

// Device views of the factor used by the refinement products.
template <typename T>
struct GView {
  int n;
  int64_t nn;
  const T *QSa, *QSb, *QWa, *QWb, *S;
};

template <typename T>
GView<T> prepare_view(Factor* f, hipStream_t st) {
  const int n = (int)f->n;
  const int64_t nn = (int64_t)n * n;
  T* qv = f->gq.ensure<T>(12 * nn);
  if (!f->gq_ready) {
    hipLaunchKernelGGL(q_variants_kernel<T>, dim3(blocks_for(nn)), dim3(256), 0, st, n,
                       (const T*)f->Q.as<T>(), qv, qv + 3 * nn, qv + 6 * nn, qv + 9 * nn);
    MSQRT_LAUNCH_CHECK();
    f->gq_ready = true;
  }
  return GView<T>{n, nn, qv, qv + 3 * nn, qv + 6 * nn, qv + 9 * nn, f->S.as<T>()};
}

// M (wide, low precision, n x 2n) -> Y = rtrsyl(S, S, Q^* M Q) (stacked, in
// Rt) -> V = Q Y (wide, overwrites M) -> X (+)= fl64(V Q^*).
// With S2a = -w S and S2b = -w^2 S (w = e^{2 pi i / 3}) the p = 3 equation
// S^2 Y + S Y S + Y S^2 = C is solved instead: its operator is
// L^2 + L R + R^2 with the commuting L(Y) = S Y, R(Y) = Y S, and
// a^2 + ab + b^2 = (a - w b)(a - w^2 b), so Y follows from the two triangular
// Sylvester equations S Z + Z S2a = C and S Y + Y S2b = Z.
template <typename T>
void correction(hipStream_t st, const GView<T>& g, T* M, T* Wst, T* Rt, double* Xw, bool set,
                TrsylvWork& tw, PhaseTimer& tm, bool split, const T* S2a = nullptr,
                const T* S2b = nullptr) {
  const int n = g.n;
  const int64_t nn = g.nn, n2 = 2 * (int64_t)n, n3 = 3 * (int64_t)n;
  tm.begin(MSQRT_T_TRANSFORM);
  // W = M Q (stacked): Re = [Mr | Mi][Qr; -Qi], Im = [Mr | Mi][Qi; Qr]
  gstore_b<T>(st, false, false, n, 2 * n, M, n, 0, g.QSb + n, n3, -(int64_t)n, Wst, n2, n, split);
  // Rt = Q^* W (stacked): Re = [Qr; Qi]^T W, Im = [-Qi; Qr]^T W
  gstore_b<T>(st, true, false, n, 2 * n, g.QSa + n, n3, -(int64_t)n, Wst, n2, 0, Rt, n2, n, split);
  tm.begin(MSQRT_T_SOLVE);
  if (S2a) {
    trsyl<T>(st, n, n, g.S, n2, S2a, n2, Rt, n2, tw);
    trsyl<T>(st, n, n, g.S, n2, S2b, n2, Rt, n2, tw);
  } else {
    trsyl<T>(st, n, n, g.S, n2, g.S, n2, Rt, n2, tw);
  }
  tm.begin(MSQRT_T_UPDATE);
  // V = Q Y (wide): Re = [Qr | -Qi][Yr; Yi], Im = [Qi | Qr][Yr; Yi]
  gstore_b<T>(st, false, false, n, 2 * n, g.QWa + nn, n, -nn, Rt, n2, 0, M, n, nn, split);
  // X (+)= V Q^*: Re = [Vr | Vi][Qr | Qi]^T, Im = [Vr | Vi][-Qi | Qr]^T
  if (set)
    gemm_set_f64<T>(st, false, true, n, 2 * n, M, n, 0, g.QWb + nn, n, -nn, Xw, n, nn, 2, false,
                    split);
  else
    gemm_update<T>(st, false, true, n, 2 * n, M, n, 0, g.QWb + nn, n, -nn, Xw, n, nn, nullptr, 2,
                   false, split);
  tm.end();
}

// ---- real route helpers

// sub[i] = 1 where t(i+1, i) != 0 (2x2 diagonal blocks of a quasi-
// triangular T); 2 where that entry is not finite.
template <typename T>
__global__ void quasi_sub_kernel(int n, const T* Tm, unsigned char* sub) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const T v = Tm[(i + 1) + (int64_t)i * n];
  sub[i] = !isfinite(v) ? 2 : (v != T(0) ? 1 : 0);
}

// C = op(A) op(B), all n x n real in precision T (batch 1).
template <typename T>
void gstore1(hipStream_t st, bool ta, bool tb, int n, const T* A, const T* B, T* C,
             bool split = false) {
  if (std::is_same<T, float>::value)
    gemm_store_f32(st, ta, tb, n, n, n, (const float*)A, n, 0, (const float*)B, n, 0, (float*)C,
                   n, 0, 1.f, 0.f, 1, false, split);
  else
    gemm_store_f64(st, ta, tb, n, n, n, (const double*)A, n, 0, (const double*)B, n, 0,
                   (double*)C, n, 0, 1.0, 0.0, 1, false);
}

// M (low precision, n x n) -> Y = rtrsyl(U, U, Q^T M Q) (in Rt) -> V = Q Y (in
// M) -> X (+)= fl64(V Q^T), with the quasi-triangular U and its partition.
template <typename T>
void correction_real(hipStream_t st, Factor* f, T* M, T* Wm, T* Rt, double* Xw, bool set,
                     PhaseTimer& tm) {
  const int n = (int)f->n;
  const T* Q = f->Q.as<T>();
  const T* U = f->S.as<T>();
  const bool split = f->prec == MSQRT_PREC_BF16SPLIT;
  tm.begin(MSQRT_T_TRANSFORM);
  gstore1<T>(st, false, false, n, M, Q, Wm, split);
  gstore1<T>(st, true, false, n, Q, Wm, Rt, split);
  tm.begin(MSQRT_T_SOLVE);
  const int* dp = f->qpart.as<int>();
  trsyl_quasi<T>(st, n, n, U, n, dp, f->qnt, U, n, dp, f->qnt, Rt, n, f->tw);
  tm.begin(MSQRT_T_UPDATE);
  gstore1<T>(st, false, false, n, Q, Rt, M, split);
  if (set)
    gemm_set_f64<T>(st, false, true, n, n, M, n, 0, Q, n, 0, Xw, n, 0, 1, false, split);
  else
    gemm_update<T>(st, false, true, n, n, M, n, 0, Q, n, 0, Xw, n, 0, nullptr, 1, false, split);
  tm.end();
}

double sum_host(const std::vector<double>& v, int off, int cnt) {
  double s = 0.0;
  for (int i = 0; i < cnt; ++i) s += v[off + i];
  return s;
}

}  // namespace

// ||A||_F, finiteness and the scale exponent for complex or real input
// without a symmetry test.  Returns the flags (bit0 = non-finite).
int analyse_input_general(Factor* f, const double* A, int64_t lda, int cplx, hipStream_t st) {
  const int n = (int)f->n;
  int* flags = f->active.ensure<int>(1);
  double* part = f->part.ensure<double>(kRedBlocks + 64);
  MSQRT_HIP(hipMemsetAsync(flags, 0, sizeof(int), st));
  hipLaunchKernelGGL(cvalidate_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, A, lda, cplx, flags,
                     part);
  MSQRT_LAUNCH_CHECK();
  std::vector<double> hp(kRedBlocks);
  int hf = 0;
  MSQRT_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * kRedBlocks, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipStreamSynchronize(st));
  const double nrm = std::sqrt(sum_host(hp, 0, kRedBlocks));
  f->kexp.assign(1, 0);
  f->anorm.assign(1, nrm);
  if (nrm > 0 && std::isfinite(nrm))
    f->kexp[0] = (int)std::lround(std::log(nrm / std::sqrt((double)n)) /
                                  std::log(std::ldexp(1.0, f->root)));
  f->upload_scales(st);
  return hf;
}

template <typename T>
msqrt_status factor_general(Factor* f, const double* A, int64_t lda, int cplx, hipStream_t st,
                            PhaseTimer* tm) {
  const int n = (int)f->n;
  const int64_t sz = 2 * (int64_t)n * n;
  T* Q = f->Q.ensure<T>(sz);
  T* S = f->S.ensure<T>(sz);
  T* H = f->fw1.ensure<T>(sz);
  f->gq_ready = false;
  if (tm) tm->begin(MSQRT_T_REDUCE);
  hipLaunchKernelGGL(to_stacked_kernel<T>, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, st, n, A,
                     lda, cplx, f->ascale_dev(), H);
  MSQRT_LAUNCH_CHECK();
  GehrdWork gw;
  gehrd<T>(st, n, H, Q, gw);
  if (tm) tm->begin(MSQRT_T_EIG);
  HseqrWork hw;
  // ||H||_F = ||A||_F / 4^k (unitary similarity)
  const bool ok = hseqr<T>(st, n, H, Q, hw, (T)f->anorm_scaled[0]);
  if (!ok) {
    if (tm) tm->end();
    set_last_error("complex Schur QR did not converge");
    return MSQRT_ERR_NOT_CONVERGED;
  }
  if (tm) tm->begin(MSQRT_T_X0);
  trsylv_reset(st, f->tw);
  trsqrt<T>(st, n, H, S, f->tw, nullptr);
  if (tm) tm->end();
  int timed_out = 0, nonprincipal = 0;
  trsylv_errors(st, f->tw, &timed_out, &nonprincipal);
  if (tm) tm->collect();
  if (timed_out) throw Error{MSQRT_ERR_DEVICE, "triangular square root: dataflow wait timed out"};
  if (nonprincipal) {
    set_last_error("an eigenvalue lies on or next to the closed negative real axis");
    return MSQRT_ERR_NO_PRINCIPAL;
  }
  return MSQRT_OK;
}

template <typename T>
msqrt_status refine_general(Factor* f, const double* A, int64_t lda, double* X, int64_t ldx,
                            int init, int maxit, double tol, hipStream_t st, msqrt_info* info,
                            PhaseTimer& tm) {
  const int n = (int)f->n;
  const int64_t nn = (int64_t)n * n;
  const int cplx = f->dtype == MSQRT_COMPLEX128;
  const GView<T> g = prepare_view<T>(f, st);
  double* Xw = f->gx.ensure<double>(7 * nn);
  double* XS = Xw + 2 * nn;
  double* Aw = Xw + 5 * nn;  // A in the wide layout [Ar | Ai]
  T* M = f->ws1.ensure<T>(2 * nn);
  T* Wst = f->ws2.ensure<T>(2 * nn);
  T* Rt = f->gt.ensure<T>(2 * nn);
  const int ntiles = (int)(ceil_div(n, 128) * ceil_div(n, 128));
  double* part = f->part.ensure<double>(2 * (int64_t)ntiles + 2 * kRedBlocks + 64);
  double* rn = f->rnorm.ensure<double>(2);
  double* sc2 = f->gsc.ensure<double>(2);
  {
    const double a = std::ldexp(1.0, -2 * f->kexp[0]);
    const double h[2] = {a, a};
    MSQRT_HIP(hipMemcpyAsync(sc2, h, sizeof(h), hipMemcpyHostToDevice, st));
  }
  hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, A, lda, cplx, 0,
                     (const double*)nullptr, Aw);
  MSQRT_LAUNCH_CHECK();
  trsylv_reset(st, f->tw);
  if (init) {
    tm.begin(MSQRT_T_X0);
    // V = Q S (wide), X_0 = fl64(V Q^*)
    gstore_b<T>(st, false, false, n, 2 * n, g.QWa + nn, n, -nn, g.S, 2 * (int64_t)n, 0, M, n, nn);
    gemm_set_f64<T>(st, false, true, n, 2 * n, M, n, 0, g.QWb + nn, n, -nn, Xw, n, nn, 2, false);
  } else {
    tm.begin(MSQRT_T_VALIDATE);
    hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, (const double*)X,
                       ldx, cplx, 0, f->rscale_dev(), Xw);
    MSQRT_LAUNCH_CHECK();
  }
  std::vector<double> hist, hp(2 * ntiles);
  double best_r = INFINITY;
  double* best = nullptr;
  Verdict verdict = Verdict::Continue;
  int steps = 0;
  for (int it = 0;; ++it) {
    tm.begin(MSQRT_T_RESIDUAL);
    hipLaunchKernelGGL(x_stack_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, (const double*)Xw,
                       XS);
    MSQRT_LAUNCH_CHECK();
    // R = A - X X: Re = Ar - [Xr | Xi][Xr; -Xi], Im = Ai - [Xr | Xi][Xi; Xr]
    const int nt = gemm_residual_ex(st, false, false, n, n, 2 * n, Xw, n, 0, XS + n, 3 * (int64_t)n,
                                    -(int64_t)n, Aw, n, nn, sc2,
                                    std::is_same<T, float>::value ? (float*)M : nullptr,
                                    std::is_same<T, float>::value ? nullptr : (double*)M, n, nn,
                                    part, 2);
    launch_reduce_sqrt(st, part, 2 * nt, 1, rn);
    double hrn = 0.0;
    MSQRT_HIP(hipMemcpyAsync(&hrn, rn, sizeof(double), hipMemcpyDeviceToHost, st));
    tm.end();
    MSQRT_HIP(hipStreamSynchronize(st));
    tm.collect();
    hist.push_back(hrn / f->anorm_scaled[0]);
    Verdict v = judge_step(hist, tol, it, maxit);
    if (v != Verdict::Continue) {
      verdict = v;
      break;
    }
    if (hist.back() < best_r) {
      best_r = hist.back();
      if (!best) best = f->best.ensure<double>(2 * nn);
      MSQRT_HIP(hipMemcpyAsync(best, Xw, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
    }
    correction<T>(st, g, M, Wst, Rt, Xw, false, f->tw, tm, f->prec == MSQRT_PREC_BF16SPLIT);
    ++steps;
  }
  msqrt_status status = MSQRT_OK;
  double final_r = hist.back();
  if (verdict != Verdict::Converged) {
    if (best && !(final_r <= best_r)) {  // also when final_r is NaN
      MSQRT_HIP(hipMemcpyAsync(Xw, best, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
      final_r = best_r;
    }
    status = verdict == Verdict::Diverged ? MSQRT_ERR_DIVERGED : MSQRT_ERR_NOT_CONVERGED;
    set_last_error(verdict == Verdict::Diverged ? "refinement diverged"
                                                 : "refinement did not converge");
  }
  // X = 2^k X_s in the caller's layout
  tm.begin(MSQRT_T_VALIDATE);
  hipLaunchKernelGGL(x_out_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, (const double*)Xw, cplx, 0,
                     f->uscale_dev(), X, ldx, part);
  MSQRT_LAUNCH_CHECK();
  std::vector<double> hx(2 * kRedBlocks);
  MSQRT_HIP(hipMemcpyAsync(hx.data(), part, sizeof(double) * 2 * kRedBlocks, hipMemcpyDeviceToHost, st));
  tm.end();
  int timed_out = 0;
  trsylv_errors(st, f->tw, &timed_out, nullptr);
  tm.collect();
  if (timed_out) throw Error{MSQRT_ERR_DEVICE, "triangular Sylvester solve: dataflow wait timed out"};
  if (info) {
    info->steps = steps;
    info->relres = std::isfinite(final_r) ? final_r : INFINITY;
    info->nhist = (int)std::min<size_t>(64, hist.size());
    for (int k = 0; k < info->nhist; ++k) info->relres_hist[k] = hist[k];
  }
  if (!cplx && status == MSQRT_OK && tol >= 0) {
    // a real matrix without eigenvalues on R<=0 has a real principal root
    // (not asserted for the intermediate iterates of a nullified-stop run)
    const double xa = std::sqrt(sum_host(hx, 0, kRedBlocks));
    const double xi = std::sqrt(sum_host(hx, kRedBlocks, kRedBlocks));
    if (xi > 1e-12 * xa) {
      set_last_error("the root of the real input has a non-negligible imaginary part");
      return MSQRT_ERR_NO_PRINCIPAL;
    }
  }
  return status;
}

template <typename T>
void trcbrt(hipStream_t st, int n, const T* Tm, T* U, T* UT, T* V, int* bad) {
  const int64_t sz = 2 * (int64_t)n * n;
  MSQRT_HIP(hipMemsetAsync(U, 0, sizeof(T) * sz, st));
  MSQRT_HIP(hipMemsetAsync(UT, 0, sizeof(T) * sz, st));
  MSQRT_HIP(hipMemsetAsync(V, 0, sizeof(T) * sz, st));
  MSQRT_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
  if (n <= 0) return;
  hipLaunchKernelGGL(trcbrt_diag_kernel<T>, dim3(blocks_for(n)), dim3(256), 0, st, n, Tm, U, UT, V,
                     bad);
  MSQRT_LAUNCH_CHECK();
  for (int d = 1; d < n; ++d) {
    const int waves = n - d;
    hipLaunchKernelGGL(trcbrt_band_kernel<T>, dim3((unsigned)ceil_div(waves, 256 / kWave)),
                       dim3(256), 0, st, n, d, Tm, U, UT, V);
    MSQRT_LAUNCH_CHECK();
  }
}

template <typename T>
msqrt_status factor_root3(Factor* f, const double* A, int64_t lda, int cplx, hipStream_t st,
                          PhaseTimer* tm) {
  const int n = (int)f->n;
  const int64_t sz = 2 * (int64_t)n * n;
  T* Q = f->Q.ensure<T>(sz);
  T* U = f->S.ensure<T>(sz);
  T* H = f->fw1.ensure<T>(sz);
  T* UT = f->fw2.ensure<T>(sz);
  T* V = f->fw3.ensure<T>(sz);
  T* S2a = f->fw4.ensure<T>(sz);
  T* S2b = f->fw5.ensure<T>(sz);
  int* bad = f->active.ensure<int>(1);
  f->gq_ready = false;
  if (tm) tm->begin(MSQRT_T_REDUCE);
  hipLaunchKernelGGL(to_stacked_kernel<T>, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, st, n, A,
                     lda, cplx, f->ascale_dev(), H);
  MSQRT_LAUNCH_CHECK();
  GehrdWork gw;
  gehrd<T>(st, n, H, Q, gw);
  if (tm) tm->begin(MSQRT_T_EIG);
  HseqrWork hw;
  const bool ok = hseqr<T>(st, n, H, Q, hw, (T)f->anorm_scaled[0]);
  if (!ok) {
    if (tm) tm->end();
    set_last_error("complex Schur QR did not converge");
    return MSQRT_ERR_NOT_CONVERGED;
  }
  if (tm) tm->begin(MSQRT_T_X0);
  trcbrt<T>(st, n, H, U, UT, V, bad);
  // -w U and -w^2 U, w = e^{2 pi i / 3}: -w = (1/2, -sqrt(3)/2), -w^2 = (1/2, sqrt(3)/2)
  const T h3 = (T)0.86602540378443864676;
  hipLaunchKernelGGL(cscale_stacked_kernel<T>, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, st, n,
                     (const T*)U, T(0.5), -h3, S2a);
  MSQRT_LAUNCH_CHECK();
  hipLaunchKernelGGL(cscale_stacked_kernel<T>, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, st, n,
                     (const T*)U, T(0.5), h3, S2b);
  MSQRT_LAUNCH_CHECK();
  int hbad = 0;
  MSQRT_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  if (tm) tm->end();
  MSQRT_HIP(hipStreamSynchronize(st));
  if (tm) tm->collect();
  if (hbad) {
    set_last_error("an eigenvalue lies on or next to the closed negative real axis");
    return MSQRT_ERR_NO_PRINCIPAL;
  }
  return MSQRT_OK;
}

template <typename T>
msqrt_status refine_root3(Factor* f, const double* A, int64_t lda, double* X, int64_t ldx,
                            int init, int maxit, double tol, hipStream_t st, msqrt_info* info,
                            PhaseTimer& tm) {
  const int n = (int)f->n;
  const int64_t nn = (int64_t)n * n;
  const int cplx = f->dtype == MSQRT_COMPLEX128;
  const GView<T> g = prepare_view<T>(f, st);
  double* Xw = f->gx.ensure<double>(12 * nn);
  double* XS = Xw + 2 * nn;
  double* Aw = Xw + 5 * nn;  // A in the wide layout [Ar | Ai]
  double* Pw = Xw + 7 * nn;  // X^2, wide
  double* PS = Xw + 9 * nn;  // X^2, stacked variant
  T* M = f->ws1.ensure<T>(2 * nn);
  T* Wst = f->ws2.ensure<T>(2 * nn);
  T* Rt = f->gt.ensure<T>(2 * nn);
  const int ntiles = (int)(ceil_div(n, 128) * ceil_div(n, 128));
  double* part = f->part.ensure<double>(2 * (int64_t)ntiles + 2 * kRedBlocks + 64);
  double* rn = f->rnorm.ensure<double>(2);
  double* sc2 = f->gsc.ensure<double>(2);
  {
    const double a = std::ldexp(1.0, -3 * f->kexp[0]);
    const double h[2] = {a, a};
    MSQRT_HIP(hipMemcpyAsync(sc2, h, sizeof(h), hipMemcpyHostToDevice, st));
  }
  hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, A, lda, cplx, 0,
                     (const double*)nullptr, Aw);
  MSQRT_LAUNCH_CHECK();
  trsylv_reset(st, f->tw);
  if (init) {
    tm.begin(MSQRT_T_X0);
    // V = Q S (wide), X_0 = fl64(V Q^*)
    gstore_b<T>(st, false, false, n, 2 * n, g.QWa + nn, n, -nn, g.S, 2 * (int64_t)n, 0, M, n, nn);
    gemm_set_f64<T>(st, false, true, n, 2 * n, M, n, 0, g.QWb + nn, n, -nn, Xw, n, nn, 2, false);
  } else {
    tm.begin(MSQRT_T_VALIDATE);
    hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, (const double*)X,
                       ldx, cplx, 0, f->rscale_dev(), Xw);
    MSQRT_LAUNCH_CHECK();
  }
  std::vector<double> hist, hp(2 * ntiles);
  double best_r = INFINITY;
  double* best = nullptr;
  Verdict verdict = Verdict::Continue;
  int steps = 0;
  for (int it = 0;; ++it) {
    tm.begin(MSQRT_T_RESIDUAL);
    hipLaunchKernelGGL(x_stack_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, (const double*)Xw,
                       XS);
    MSQRT_LAUNCH_CHECK();
    // P = X X (float64, wide), then R = A - X P: the same planar products
    // as for the square root, Re = [Xr | Xi][Pr; -Pi], Im = [Xr | Xi][Pi; Pr]
    gemm_store_f64(st, false, false, n, n, 2 * n, Xw, n, 0, XS + n, 3 * (int64_t)n, -(int64_t)n,
                   Pw, n, nn, 1.0, 0.0, 2, false);
    hipLaunchKernelGGL(x_stack_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, (const double*)Pw,
                       PS);
    MSQRT_LAUNCH_CHECK();
    const int nt = gemm_residual_ex(st, false, false, n, n, 2 * n, Xw, n, 0, PS + n, 3 * (int64_t)n,
                                    -(int64_t)n, Aw, n, nn, sc2,
                                    std::is_same<T, float>::value ? (float*)M : nullptr,
                                    std::is_same<T, float>::value ? nullptr : (double*)M, n, nn,
                                    part, 2);
    launch_reduce_sqrt(st, part, 2 * nt, 1, rn);
    double hrn = 0.0;
    MSQRT_HIP(hipMemcpyAsync(&hrn, rn, sizeof(double), hipMemcpyDeviceToHost, st));
    tm.end();
    MSQRT_HIP(hipStreamSynchronize(st));
    tm.collect();
    hist.push_back(hrn / f->anorm_scaled[0]);
    Verdict v = judge_step(hist, tol, it, maxit);
    if (v != Verdict::Continue) {
      verdict = v;
      break;
    }
    if (hist.back() < best_r) {
      best_r = hist.back();
      if (!best) best = f->best.ensure<double>(2 * nn);
      MSQRT_HIP(hipMemcpyAsync(best, Xw, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
    }
    correction<T>(st, g, M, Wst, Rt, Xw, false, f->tw, tm, false, f->fw4.as<T>(),
                  f->fw5.as<T>());
    ++steps;
  }
  msqrt_status status = MSQRT_OK;
  double final_r = hist.back();
  if (verdict != Verdict::Converged) {
    if (best && !(final_r <= best_r)) {  // also when final_r is NaN
      MSQRT_HIP(hipMemcpyAsync(Xw, best, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
      final_r = best_r;
    }
    status = verdict == Verdict::Diverged ? MSQRT_ERR_DIVERGED : MSQRT_ERR_NOT_CONVERGED;
    set_last_error(verdict == Verdict::Diverged ? "refinement diverged"
                                                 : "refinement did not converge");
  }
  // X = 2^k X_s in the caller's layout
  tm.begin(MSQRT_T_VALIDATE);
  hipLaunchKernelGGL(x_out_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, (const double*)Xw, cplx, 0,
                     f->uscale_dev(), X, ldx, part);
  MSQRT_LAUNCH_CHECK();
  std::vector<double> hx(2 * kRedBlocks);
  MSQRT_HIP(hipMemcpyAsync(hx.data(), part, sizeof(double) * 2 * kRedBlocks, hipMemcpyDeviceToHost, st));
  tm.end();
  int timed_out = 0;
  trsylv_errors(st, f->tw, &timed_out, nullptr);
  tm.collect();
  if (timed_out) throw Error{MSQRT_ERR_DEVICE, "triangular Sylvester solve: dataflow wait timed out"};
  if (info) {
    info->steps = steps;
    info->relres = std::isfinite(final_r) ? final_r : INFINITY;
    info->nhist = (int)std::min<size_t>(64, hist.size());
    for (int k = 0; k < info->nhist; ++k) info->relres_hist[k] = hist[k];
  }
  if (!cplx && status == MSQRT_OK && tol >= 0) {
    // a real matrix without eigenvalues on R<=0 has a real principal root
    // (not asserted for the intermediate iterates of a nullified-stop run)
    const double xa = std::sqrt(sum_host(hx, 0, kRedBlocks));
    const double xi = std::sqrt(sum_host(hx, kRedBlocks, kRedBlocks));
    if (xi > 1e-12 * xa) {
      set_last_error("the cube root of the real input has a non-negligible imaginary part");
      return MSQRT_ERR_NO_PRINCIPAL;
    }
  }
  return status;
}

// Backward: X^* G + G X^* = Gbar.  Its conjugate transpose is
// X G~ + G~ X = Gbar^* with G~ = G^*: the forward correction equation, solved
// with the same factor (Q^* (.) Q, rtrsyl, Q (.) Q^*) and refined with
// float64 residuals.  The factor belongs to A/4^k, whose root is
// X_s = 2^-k X, so G = 2^-k G'.
template <typename T>
msqrt_status backward_general(Factor* f, const double* X, int64_t ldx, const double* Gbar,
                              int64_t ldgb, double* G, int64_t ldg, int maxit, double tol,
                              hipStream_t st, msqrt_info* info, PhaseTimer& tm) {
  const int n = (int)f->n;
  const int64_t nn = (int64_t)n * n, n3 = 3 * (int64_t)n;
  const int cplx = f->dtype == MSQRT_COMPLEX128;
  const GView<T> g = prepare_view<T>(f, st);
  double* Xw = f->gx.ensure<double>(5 * nn);  // X_s (wide)
  double* XS = Xw + 2 * nn;                   // [X_s i; X_s r; -X_s i]
  double* Cw = f->best.ensure<double>(6 * nn);  // Gbar^* (wide), T1 (wide), G~ (wide)
  double* T1 = Cw + 2 * nn;
  double* Gw = Cw + 4 * nn;
  double* GS = f->fw2.ensure<double>(3 * nn);  // [G~i; G~r; -G~i]
  T* M = f->ws1.ensure<T>(2 * nn);
  T* Wst = f->ws2.ensure<T>(2 * nn);
  T* Rt = f->gt.ensure<T>(2 * nn);
  const int ntiles = (int)(ceil_div(n, 128) * ceil_div(n, 128));
  double* part = f->part.ensure<double>(2 * (int64_t)ntiles + 2 * kRedBlocks + 64);
  double* rn = f->rnorm.ensure<double>(2);
  double* one2 = f->gsc.ensure<double>(2);
  {
    const double h[2] = {1.0, 1.0};
    MSQRT_HIP(hipMemcpyAsync(one2, h, sizeof(h), hipMemcpyHostToDevice, st));
  }
  trsylv_reset(st, f->tw);
  tm.begin(MSQRT_T_VALIDATE);
  int* flags = f->active.ensure<int>(1);
  MSQRT_HIP(hipMemsetAsync(flags, 0, sizeof(int), st));
  hipLaunchKernelGGL(cvalidate_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, Gbar, ldgb, cplx,
                     flags, part);
  MSQRT_LAUNCH_CHECK();
  std::vector<double> hp(kRedBlocks);
  int hf = 0;
  MSQRT_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * kRedBlocks, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, st));
  hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, X, ldx, cplx, 0,
                     f->rscale_dev(), Xw);
  MSQRT_LAUNCH_CHECK();
  hipLaunchKernelGGL(x_stack_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, (const double*)Xw, XS);
  MSQRT_LAUNCH_CHECK();
  hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, Gbar, ldgb, cplx, 1,
                     nullptr, Cw);
  MSQRT_LAUNCH_CHECK();
  tm.end();
  MSQRT_HIP(hipStreamSynchronize(st));
  tm.collect();
  if (hf & 1) {
    set_last_error("Gbar contains Inf or NaN");
    return MSQRT_ERR_NONFINITE;
  }
  const double gnorm = std::sqrt(sum_host(hp, 0, kRedBlocks));
  std::vector<double> hist;
  Verdict verdict = Verdict::Continue;
  int steps = 0;
  for (int it = 0;; ++it) {
    tm.begin(MSQRT_T_RESIDUAL);
    if (it == 0) {
      // G~ = 0: the residual is Gbar^* itself
      hist.push_back(gnorm > 0.0 ? 1.0 : 0.0);
      if (gnorm == 0.0) {
        verdict = Verdict::Converged;
        MSQRT_HIP(hipMemsetAsync(Gw, 0, sizeof(double) * 2 * nn, st));
        break;
      }
      // fl(Gbar^*) in the wide low-precision layout
      if (std::is_same<T, float>::value)
        launch_cast_scale_f64_f32(st, n, Cw, n, nn, nullptr, (float*)M, n, nn, 2);
      else
        launch_cast_scale_f64_f64(st, n, Cw, n, nn, nullptr, (double*)M, n, nn, 2);
    } else {
      // R = Gbar^* - X_s G~ - G~ X_s
      MSQRT_HIP(hipMemcpyAsync(T1, Cw, sizeof(double) * 2 * nn, hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(x_stack_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n,
                         (const double*)Gw, GS);
      MSQRT_LAUNCH_CHECK();
      // T1 -= X_s G~: Re -= [Xr | Xi][Gr; -Gi], Im -= [Xr | Xi][Gi; Gr]
      gemm_store_f64(st, false, false, n, n, 2 * n, Xw, n, 0, GS + n, n3, -(int64_t)n, T1, n, nn,
                     -1.0, 1.0, 2, false);
      // R = T1 - G~ X_s
      const int nt = gemm_residual_ex(st, false, false, n, n, 2 * n, Gw, n, 0, XS + n, n3,
                                      -(int64_t)n, T1, n, nn, one2,
                                      std::is_same<T, float>::value ? (float*)M : nullptr,
                                      std::is_same<T, float>::value ? nullptr : (double*)M, n, nn,
                                      part, 2);
      launch_reduce_sqrt(st, part, 2 * nt, 1, rn);
      double hrn = 0.0;
      MSQRT_HIP(hipMemcpyAsync(&hrn, rn, sizeof(double), hipMemcpyDeviceToHost, st));
      tm.end();
      MSQRT_HIP(hipStreamSynchronize(st));
      tm.collect();
      hist.push_back(hrn / gnorm);
      Verdict v = judge_step(hist, tol, it, maxit);
      if (v != Verdict::Continue) {
        verdict = v;
        break;
      }
    }
    correction<T>(st, g, M, Wst, Rt, Gw, it == 0, f->tw, tm, f->prec == MSQRT_PREC_BF16SPLIT);
    ++steps;
  }
  // G = 2^-k (G~)^*
  tm.begin(MSQRT_T_VALIDATE);
  hipLaunchKernelGGL(x_out_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, (const double*)Gw, cplx, 1,
                     f->rscale_dev(), G, ldg, part);
  MSQRT_LAUNCH_CHECK();
  tm.end();
  int timed_out = 0;
  trsylv_errors(st, f->tw, &timed_out, nullptr);
  tm.collect();
  if (timed_out) throw Error{MSQRT_ERR_DEVICE, "triangular Sylvester solve: dataflow wait timed out"};
  msqrt_status status = MSQRT_OK;
  if (verdict == Verdict::Diverged) status = MSQRT_ERR_DIVERGED;
  else if (verdict != Verdict::Converged) status = MSQRT_ERR_NOT_CONVERGED;
  if (info) {
    info->steps = steps;
    info->relres = hist.back();
    info->nhist = (int)std::min<size_t>(64, hist.size());
    for (int k = 0; k < info->nhist; ++k) info->relres_hist[k] = hist[k];
    info->prec_used = f->prec;
    info->struct_used = f->structure;
    info->scale_exp = f->kexp.empty() ? 0 : f->kexp[0];
  }
  return status;
}

// ---------------------------------------------------------------------------
// Real route: real input on the general path with the real Schur form
// A/4^k ~ Q T Q^T (remark on real input in Sec. 2.2.1): real Hessenberg
// reduction, the real double-shift QR, the tile partition that keeps 2x2
// blocks whole, and U = T^{1/2} on it.

template <typename T>
msqrt_status factor_real(Factor* f, const double* A, int64_t lda, hipStream_t st, PhaseTimer* tm) {
  const int n = (int)f->n;
  const int64_t nn = (int64_t)n * n;
  T* Q = f->Q.ensure<T>(nn);
  T* U = f->S.ensure<T>(nn);
  T* H = f->fw3.ensure<T>(nn);
  unsigned char* dsub = f->fw4.ensure<unsigned char>(n + 64);
  f->gq_ready = false;
  f->real_schur = true;
  if (tm) tm->begin(MSQRT_T_REDUCE);
  if (std::is_same<T, float>::value)
    launch_cast_scale_f64_f32(st, n, A, lda, 0, f->ascale_dev(), (float*)H, n, 0, 1);
  else
    launch_cast_scale_f64_f64(st, n, A, lda, 0, f->ascale_dev(), (double*)H, n, 0, 1);
  GehrdWork gw;
  gehrd_real<T>(st, n, H, Q, gw);
  if (tm) tm->begin(MSQRT_T_EIG);
  HseqrWork hw;
  const bool ok = rhseqr<T>(st, n, H, Q, hw, (T)f->anorm_scaled[0]);
  if (!ok) {
    if (tm) tm->end();
    set_last_error("real Schur QR did not converge");
    return MSQRT_ERR_NOT_CONVERGED;
  }
  if (tm) tm->begin(MSQRT_T_X0);
  std::vector<unsigned char> sub(std::max(n, 1), 0);
  if (n > 1) {
    hipLaunchKernelGGL(quasi_sub_kernel<T>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n,
                       (const T*)H, dsub);
    MSQRT_LAUNCH_CHECK();
    MSQRT_HIP(hipMemcpyAsync(sub.data(), dsub, n - 1, hipMemcpyDeviceToHost, st));
    MSQRT_HIP(hipStreamSynchronize(st));
  }
  for (int i = 0; i + 1 < n; ++i) {
    if (sub[i] == 2 || (sub[i] && i + 2 < n && sub[i + 1])) {
      if (tm) tm->end();
      set_last_error("real Schur QR left a non-finite or overlapping 2x2 block");
      return MSQRT_ERR_NOT_CONVERGED;
    }
  }
  f->qpart_h = quasi_partition(n, sub.data());
  f->qnt = (int)f->qpart_h.size() - 1;
  int* dp = f->qpart.ensure<int>((int64_t)f->qpart_h.size());
  MSQRT_HIP(hipMemcpyAsync(dp, f->qpart_h.data(), sizeof(int) * f->qpart_h.size(),
                           hipMemcpyHostToDevice, st));
  trsylv_reset(st, f->tw);
  trsqrt_quasi<T>(st, n, H, U, dp, f->qnt, f->tw);
  if (tm) tm->end();
  int timed_out = 0, nonprincipal = 0;
  trsylv_errors(st, f->tw, &timed_out, &nonprincipal);
  if (tm) tm->collect();
  if (timed_out) throw Error{MSQRT_ERR_DEVICE, "quasi-triangular square root: dataflow wait timed out"};
  if (nonprincipal) {
    set_last_error("an eigenvalue lies on or next to the closed negative real axis");
    return MSQRT_ERR_NO_PRINCIPAL;
  }
  return MSQRT_OK;
}

template <typename T>
msqrt_status refine_real(Factor* f, const double* A, int64_t lda, double* X, int64_t ldx, int init,
                         int maxit, double tol, hipStream_t st, msqrt_info* info, PhaseTimer& tm) {
  const int n = (int)f->n;
  const int64_t nn = (int64_t)n * n;
  const T* Q = f->Q.as<T>();
  const T* U = f->S.as<T>();
  // X (float64) with an all-zero second plane, so that the wide in/out
  // kernels of the complex route read and write it unchanged
  double* Xw = f->gx.ensure<double>(2 * nn);
  T* M = f->ws1.ensure<T>(nn);
  T* Wm = f->ws2.ensure<T>(nn);
  T* Rt = f->gt.ensure<T>(nn);
  const int ntiles = (int)(ceil_div(n, 128) * ceil_div(n, 128));
  double* part = f->part.ensure<double>((int64_t)ntiles + 2 * kRedBlocks + 64);
  double* rn = f->rnorm.ensure<double>(1);
  trsylv_reset(st, f->tw);
  if (init) {
    tm.begin(MSQRT_T_X0);
    MSQRT_HIP(hipMemsetAsync(Xw + nn, 0, sizeof(double) * nn, st));
    // V = Q U, X_0 = fl64(V Q^T)
    gstore1<T>(st, false, false, n, Q, U, M);
    gemm_set_f64<T>(st, false, true, n, n, M, n, 0, Q, n, 0, Xw, n, 0, 1, false);
  } else {
    tm.begin(MSQRT_T_VALIDATE);
    hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, (const double*)X,
                       ldx, 0, 0, f->rscale_dev(), Xw);
    MSQRT_LAUNCH_CHECK();
  }
  std::vector<double> hist;
  double best_r = INFINITY;
  double* best = nullptr;
  Verdict verdict = Verdict::Continue;
  int steps = 0;
  for (int it = 0;; ++it) {
    tm.begin(MSQRT_T_RESIDUAL);
    // R = A/4^k - X X
    const int nt = gemm_residual_ex(st, false, false, n, n, n, Xw, n, 0, Xw, n, 0, A, lda, 0,
                                    f->ascale_dev(),
                                    std::is_same<T, float>::value ? (float*)M : nullptr,
                                    std::is_same<T, float>::value ? nullptr : (double*)M, n, 0,
                                    part, 1);
    launch_reduce_sqrt(st, part, nt, 1, rn);
    double hrn = 0.0;
    MSQRT_HIP(hipMemcpyAsync(&hrn, rn, sizeof(double), hipMemcpyDeviceToHost, st));
    tm.end();
    MSQRT_HIP(hipStreamSynchronize(st));
    tm.collect();
    hist.push_back(hrn / f->anorm_scaled[0]);
    Verdict v = judge_step(hist, tol, it, maxit);
    if (v != Verdict::Continue) {
      verdict = v;
      break;
    }
    if (hist.back() < best_r) {
      best_r = hist.back();
      if (!best) best = f->best.ensure<double>(nn);
      MSQRT_HIP(hipMemcpyAsync(best, Xw, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    }
    correction_real<T>(st, f, M, Wm, Rt, Xw, false, tm);
    ++steps;
  }
  msqrt_status status = MSQRT_OK;
  double final_r = hist.back();
  if (verdict != Verdict::Converged) {
    if (best && !(final_r <= best_r)) {  // also when final_r is NaN
      MSQRT_HIP(hipMemcpyAsync(Xw, best, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
      final_r = best_r;
    }
    status = verdict == Verdict::Diverged ? MSQRT_ERR_DIVERGED : MSQRT_ERR_NOT_CONVERGED;
    set_last_error(verdict == Verdict::Diverged ? "refinement diverged"
                                                 : "refinement did not converge");
  }
  tm.begin(MSQRT_T_VALIDATE);
  hipLaunchKernelGGL(x_out_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, (const double*)Xw, 0, 0,
                     f->uscale_dev(), X, ldx, part);
  MSQRT_LAUNCH_CHECK();
  tm.end();
  int timed_out = 0;
  trsylv_errors(st, f->tw, &timed_out, nullptr);
  tm.collect();
  if (timed_out) throw Error{MSQRT_ERR_DEVICE, "quasi-triangular Sylvester solve: dataflow wait timed out"};
  if (info) {
    info->steps = steps;
    info->relres = std::isfinite(final_r) ? final_r : INFINITY;
    info->nhist = (int)std::min<size_t>(64, hist.size());
    for (int k = 0; k < info->nhist; ++k) info->relres_hist[k] = hist[k];
  }
  return status;
}

// Backward on the real route: X^T G + G X^T = Gbar, i.e. X G~ + G~ X = Gbar^T
// with G~ = G^T, solved with the factor of A/4^k (root X_s = 2^-k X) and
// refined with float64 residuals; G = 2^-k G~^T.
template <typename T>
msqrt_status backward_real(Factor* f, const double* X, int64_t ldx, const double* Gbar,
                           int64_t ldgb, double* G, int64_t ldg, int maxit, double tol,
                           hipStream_t st, msqrt_info* info, PhaseTimer& tm) {
  const int n = (int)f->n;
  const int64_t nn = (int64_t)n * n;
  double* Xw = f->gx.ensure<double>(2 * nn);   // X_s (second plane zero)
  double* Cw = f->best.ensure<double>(5 * nn);  // Gbar^T (two planes), T1, G~ (two planes)
  double* T1 = Cw + 2 * nn;
  double* Gw = Cw + 3 * nn;
  T* M = f->ws1.ensure<T>(nn);
  T* Wm = f->ws2.ensure<T>(nn);
  T* Rt = f->gt.ensure<T>(nn);
  const int ntiles = (int)(ceil_div(n, 128) * ceil_div(n, 128));
  double* part = f->part.ensure<double>((int64_t)ntiles + 2 * kRedBlocks + 64);
  double* rn = f->rnorm.ensure<double>(1);
  double* one = f->gsc.ensure<double>(1);
  {
    const double h = 1.0;
    MSQRT_HIP(hipMemcpyAsync(one, &h, sizeof(h), hipMemcpyHostToDevice, st));
  }
  trsylv_reset(st, f->tw);
  tm.begin(MSQRT_T_VALIDATE);
  int* flags = f->active.ensure<int>(1);
  MSQRT_HIP(hipMemsetAsync(flags, 0, sizeof(int), st));
  hipLaunchKernelGGL(cvalidate_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, Gbar, ldgb, 0,
                     flags, part);
  MSQRT_LAUNCH_CHECK();
  std::vector<double> hp(kRedBlocks);
  int hf = 0;
  MSQRT_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * kRedBlocks, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, st));
  hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, X, ldx, 0, 0,
                     f->rscale_dev(), Xw);
  MSQRT_LAUNCH_CHECK();
  hipLaunchKernelGGL(x_in_kernel, dim3(blocks_for(nn)), dim3(256), 0, st, n, Gbar, ldgb, 0, 1,
                     (const double*)nullptr, Cw);
  MSQRT_LAUNCH_CHECK();
  MSQRT_HIP(hipMemsetAsync(Gw + nn, 0, sizeof(double) * nn, st));
  tm.end();
  MSQRT_HIP(hipStreamSynchronize(st));
  tm.collect();
  if (hf & 1) {
    set_last_error("Gbar contains Inf or NaN");
    return MSQRT_ERR_NONFINITE;
  }
  const double gnorm = std::sqrt(sum_host(hp, 0, kRedBlocks));
  std::vector<double> hist;
  Verdict verdict = Verdict::Continue;
  int steps = 0;
  for (int it = 0;; ++it) {
    tm.begin(MSQRT_T_RESIDUAL);
    if (it == 0) {
      hist.push_back(gnorm > 0.0 ? 1.0 : 0.0);
      if (gnorm == 0.0) {
        verdict = Verdict::Converged;
        MSQRT_HIP(hipMemsetAsync(Gw, 0, sizeof(double) * nn, st));
        break;
      }
      if (std::is_same<T, float>::value)
        launch_cast_scale_f64_f32(st, n, Cw, n, 0, nullptr, (float*)M, n, 0, 1);
      else
        launch_cast_scale_f64_f64(st, n, Cw, n, 0, nullptr, (double*)M, n, 0, 1);
    } else {
      // R = Gbar^T - X_s G~ - G~ X_s
      MSQRT_HIP(hipMemcpyAsync(T1, Cw, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
      gemm_store_f64(st, false, false, n, n, n, Xw, n, 0, Gw, n, 0, T1, n, 0, -1.0, 1.0, 1, false);
      const int nt = gemm_residual_ex(st, false, false, n, n, n, Gw, n, 0, Xw, n, 0, T1, n, 0, one,
                                      std::is_same<T, float>::value ? (float*)M : nullptr,
                                      std::is_same<T, float>::value ? nullptr : (double*)M, n, 0,
                                      part, 1);
      launch_reduce_sqrt(st, part, nt, 1, rn);
      double hrn = 0.0;
      MSQRT_HIP(hipMemcpyAsync(&hrn, rn, sizeof(double), hipMemcpyDeviceToHost, st));
      tm.end();
      MSQRT_HIP(hipStreamSynchronize(st));
      tm.collect();
      hist.push_back(hrn / gnorm);
      Verdict v = judge_step(hist, tol, it, maxit);
      if (v != Verdict::Continue) {
        verdict = v;
        break;
      }
    }
    correction_real<T>(st, f, M, Wm, Rt, Gw, it == 0, tm);
    ++steps;
  }
  tm.begin(MSQRT_T_VALIDATE);
  hipLaunchKernelGGL(x_out_kernel, dim3(kRedBlocks), dim3(256), 0, st, n, (const double*)Gw, 0, 1,
                     f->rscale_dev(), G, ldg, part);
  MSQRT_LAUNCH_CHECK();
  tm.end();
  int timed_out = 0;
  trsylv_errors(st, f->tw, &timed_out, nullptr);
  tm.collect();
  if (timed_out) throw Error{MSQRT_ERR_DEVICE, "quasi-triangular Sylvester solve: dataflow wait timed out"};
  msqrt_status status = MSQRT_OK;
  if (verdict == Verdict::Diverged) status = MSQRT_ERR_DIVERGED;
  else if (verdict != Verdict::Converged) status = MSQRT_ERR_NOT_CONVERGED;
  if (info) {
    info->steps = steps;
    info->relres = hist.back();
    info->nhist = (int)std::min<size_t>(64, hist.size());
    for (int k = 0; k < info->nhist; ++k) info->relres_hist[k] = hist[k];
    info->prec_used = f->prec;
    info->struct_used = f->structure;
    info->scale_exp = f->kexp.empty() ? 0 : f->kexp[0];
  }
  return status;
}

#define MSQRT_REAL_INST(T)                                                                      \
  template msqrt_status factor_real<T>(Factor*, const double*, int64_t, hipStream_t, PhaseTimer*); \
  template msqrt_status refine_real<T>(Factor*, const double*, int64_t, double*, int64_t, int, int, \
                                       double, hipStream_t, msqrt_info*, PhaseTimer&);          \
  template msqrt_status backward_real<T>(Factor*, const double*, int64_t, const double*, int64_t, \
                                         double*, int64_t, int, double, hipStream_t, msqrt_info*, \
                                         PhaseTimer&);
MSQRT_REAL_INST(float)
MSQRT_REAL_INST(double)
#undef MSQRT_REAL_INST

template msqrt_status factor_general<float>(Factor*, const double*, int64_t, int, hipStream_t,
                                            PhaseTimer*);
template msqrt_status factor_general<double>(Factor*, const double*, int64_t, int, hipStream_t,
                                             PhaseTimer*);
template msqrt_status refine_general<float>(Factor*, const double*, int64_t, double*, int64_t, int,
                                            int, double, hipStream_t, msqrt_info*, PhaseTimer&);
template msqrt_status refine_general<double>(Factor*, const double*, int64_t, double*, int64_t,
                                             int, int, double, hipStream_t, msqrt_info*,
                                             PhaseTimer&);
template void trcbrt<float>(hipStream_t, int, const float*, float*, float*, float*, int*);
template void trcbrt<double>(hipStream_t, int, const double*, double*, double*, double*, int*);
template msqrt_status factor_root3<float>(Factor*, const double*, int64_t, int, hipStream_t,
                                          PhaseTimer*);
template msqrt_status factor_root3<double>(Factor*, const double*, int64_t, int, hipStream_t,
                                           PhaseTimer*);
template msqrt_status refine_root3<float>(Factor*, const double*, int64_t, double*, int64_t, int,
                                          int, double, hipStream_t, msqrt_info*, PhaseTimer&);
template msqrt_status refine_root3<double>(Factor*, const double*, int64_t, double*, int64_t, int,
                                           int, double, hipStream_t, msqrt_info*, PhaseTimer&);
template msqrt_status backward_general<float>(Factor*, const double*, int64_t, const double*,
                                              int64_t, double*, int64_t, int, double, hipStream_t,
                                              msqrt_info*, PhaseTimer&);
template msqrt_status backward_general<double>(Factor*, const double*, int64_t, const double*,
                                               int64_t, double*, int64_t, int, double,
                                               hipStream_t, msqrt_info*, PhaseTimer&);

}  // namespace msqrt
