// Host runtime and C-ABI of the msqrt library: factor objects, validation and
// scaling, the refinement loop of Alg. 2/3 and precision escalation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/msqrt.h"
#include "factor.hpp"
#include "kernels.hpp"
#include "profile.hpp"
#include "tridiag.hpp"

namespace msqrt {

thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// Device allocation cache.

namespace {
std::mutex g_pool_mu;
std::multimap<std::pair<int, size_t>, void*> g_pool;
}  // namespace

void* pool_alloc(size_t bytes) {
  int dev = 0;
  MSQRT_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pool.find({dev, bytes});
    if (it != g_pool.end()) {
      void* p = it->second;
      g_pool.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // release the cache and retry once
    {
      std::lock_guard<std::mutex> lk(g_pool_mu);
      for (auto& kv : g_pool) (void)hipFree(kv.second);
      g_pool.clear();
    }
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{MSQRT_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
  }
  return p;
}

// Frees every cached allocation (each on its own device).
void pool_release() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (auto& kv : g_pool) {
    if (hipSetDevice(kv.first.first) == hipSuccess) (void)hipFree(kv.second);
  }
  if (have) (void)hipSetDevice(cur);
  g_pool.clear();
}

void selector_release();

void pool_free(void* p, size_t bytes) {
  if (!p) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pool.insert({{dev, bytes}, p});
}

// ---------------------------------------------------------------------------
// Refinement for HPD (real SPD) factors: Alg. 3 loop.  T is the factor
// precision (float for FP32, double for FP64).

// Tiles of the symmetric residual GEMM (128 x 128, lower triangle): sizes
// the per-tile partial sums of ||R||_F.
static int64_t residual_tiles(int n) { return ceil_div(n, 128) * (ceil_div(n, 128) + 1) / 2; }

template <typename T>
static msqrt_status refine_hpd(Factor* f, const double* A, int64_t lda, int64_t sA, double* X,
                               int64_t ldx, int64_t sX, int init, int maxit, double tol,
                               hipStream_t st, msqrt_info* info, PhaseTimer& tm,
                               const RefineWs* ws) {
  const int n = (int)f->n, batch = (int)f->batch;
  const int64_t nn = (int64_t)n * n;
  const T* Q = f->Q.as<T>();
  const T* s = f->S.as<T>();
  T* W1 = ws ? (T*)ws->w1 : f->ws1.ensure<T>(nn * batch);
  T* W2 = ws ? (T*)ws->w2 : f->ws2.ensure<T>(nn * batch);
  double* part = ws ? ws->part : f->part.ensure<double>(residual_tiles(n) * batch + 64);
  double* rn = ws ? ws->rn : f->rnorm.ensure<double>(batch);
  int* active = ws ? ws->flags : f->active.ensure<int>(batch);
  double* best = nullptr;
  // BF16SPLIT: float factor, Schur-basis transforms as BF16-split products
  const bool split = f->prec == MSQRT_PREC_BF16SPLIT;

  if (init) {
    tm.begin(MSQRT_T_X0);
    // X_0 = (Q diag(s)) Q^T in the factor precision, stored in float64.
    launch_scale_cols<T>(st, n, Q, n, nn, s, n, W1, n, nn, batch);
    gemm_set_f64<T>(st, false, true, n, n, W1, n, nn, Q, n, nn, X, ldx, sX, batch, true);
  }

  std::vector<std::vector<double>> hist(batch);
  std::vector<int> done(batch, 0), steps(batch, 0);
  std::vector<Verdict> verdict(batch, Verdict::Continue);
  std::vector<double> host_rn(batch), best_r(batch, INFINITY);
  std::vector<int> host_active(batch, 1);
  bool need_best = false;

  for (int it = 0;; ++it) {
    tm.begin(MSQRT_T_RESIDUAL);
    int ntiles;
    if (std::is_same<T, float>::value)
      ntiles = gemm_residual(st, n, X, ldx, sX, A, lda, sA, f->ascale_dev(), (float*)W1, nullptr, n,
                             nn, part, batch, true);
    else
      ntiles = gemm_residual(st, n, X, ldx, sX, A, lda, sA, f->ascale_dev(), nullptr, (double*)W1,
                             n, nn, part, batch, true);
    launch_reduce_sqrt(st, part, ntiles, batch, rn);
    MSQRT_HIP(hipMemcpyAsync(host_rn.data(), rn, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    tm.end();
    MSQRT_HIP(hipStreamSynchronize(st));
    tm.collect();
    bool all_done = true;
    for (int b = 0; b < batch; ++b) {
      if (done[b]) continue;
      const double r = host_rn[b] / f->anorm_scaled[b];
      hist[b].push_back(r);
      Verdict v = judge_step(hist[b], tol, it, maxit);
      if (v != Verdict::Continue) {
        done[b] = 1;
        verdict[b] = v;
        host_active[b] = 0;
      } else {
        all_done = false;
      }
    }
    if (all_done) break;
    // Keep the best iterate of every entry that is still being refined, so a
    // diverging entry can return it.
    for (int b = 0; b < batch; ++b)
      if (!done[b] && hist[b].back() < best_r[b]) {
        best_r[b] = hist[b].back();
        need_best = true;
      }
    if (need_best) {
      if (!best) best = ws ? ws->best : f->best.ensure<double>(nn * batch);
      for (int b = 0; b < batch; ++b)
        if (!done[b] && hist[b].back() == best_r[b])
          launch_copy_f64(st, n, X + b * sX, ldx, 0, best + b * nn, n, 0, 1);
      need_best = false;
    }
    MSQRT_HIP(hipMemcpyAsync(active, host_active.data(), sizeof(int) * batch, hipMemcpyHostToDevice, st));
    // Schur-basis transform and diagonal solve (Alg. 3):
    //   W2 = R_l Q;  Y = (Q^T W2) ./ (s_i + s_j)  -> W1
    tm.begin(MSQRT_T_TRANSFORM);
    if (std::is_same<T, float>::value)
      gemm_store_f32(st, false, false, n, n, n, (const float*)W1, n, nn, (const float*)Q, n, nn,
                     (float*)W2, n, nn, 1.f, 0.f, batch, false, split);
    else
      gemm_store_f64(st, false, false, n, n, n, (const double*)W1, n, nn, (const double*)Q, n, nn,
                     (double*)W2, n, nn, 1.0, 0.0, batch, false);
    gemm_diagsylv<T>(st, true, false, n, Q, n, nn, W2, n, nn, s, n, W1, n, nn, batch, true, split);
    // Back-transform and working-precision update:  V = Q Y -> W2;  X += V Q^T
    tm.begin(MSQRT_T_UPDATE);
    if (std::is_same<T, float>::value)
      gemm_store_f32(st, false, false, n, n, n, (const float*)Q, n, nn, (const float*)W1, n, nn,
                     (float*)W2, n, nn, 1.f, 0.f, batch, false, split);
    else
      gemm_store_f64(st, false, false, n, n, n, (const double*)Q, n, nn, (const double*)W1, n, nn,
                     (double*)W2, n, nn, 1.0, 0.0, batch, false);
    gemm_update<T>(st, false, true, n, n, W2, n, nn, Q, n, nn, X, ldx, sX, active, batch, true,
                   split);
    tm.end();
    for (int b = 0; b < batch; ++b)
      if (!done[b]) steps[b]++;
  }

  // Restore the best iterate where the refinement failed.
  msqrt_status status = MSQRT_OK;
  int max_steps = 0;
  double max_r = 0.0;
  for (int b = 0; b < batch; ++b) {
    max_steps = std::max(max_steps, steps[b]);
    double final_r = hist[b].back();
    if (verdict[b] != Verdict::Converged) {
      if (best && !(final_r <= best_r[b])) {  // also when final_r is NaN
        launch_copy_f64(st, n, best + b * nn, n, 0, X + b * sX, ldx, 0, 1);
        final_r = best_r[b];
      }
      msqrt_status sb = verdict[b] == Verdict::Diverged ? MSQRT_ERR_DIVERGED : MSQRT_ERR_NOT_CONVERGED;
      if (status == MSQRT_OK || sb == MSQRT_ERR_DIVERGED) status = sb;
    }
    max_r = std::max(max_r, std::isfinite(final_r) ? final_r : INFINITY);
  }
  if (info) {
    info->steps = max_steps;
    info->relres = max_r;
    info->nhist = (int)std::min<size_t>(64, hist[0].size());
    for (int k = 0; k < info->nhist; ++k) info->relres_hist[k] = hist[0][k];
  }
  return status;
}

msqrt_status refine(Factor* f, const double* A, int64_t lda, int64_t sA, double* X, int64_t ldx,
                    int64_t sX, int init, int maxit, double tol, hipStream_t st, msqrt_info* info,
                    PhaseTimer& tm, const RefineWs* ws = nullptr) {
  if (f->structure == MSQRT_STRUCT_HPD) {
    if (f->prec == MSQRT_PREC_FP64)
      return refine_hpd<double>(f, A, lda, sA, X, ldx, sX, init, maxit, tol, st, info, tm, ws);
    return refine_hpd<float>(f, A, lda, sA, X, ldx, sX, init, maxit, tol, st, info, tm, ws);
  }
  if (ws) throw Error{MSQRT_ERR_UNSUPPORTED, "caller workspace: HPD factors only"};
  // general path: one matrix; X is read and written at the caller's scale
  if (f->real_schur) {
    if (f->prec == MSQRT_PREC_FP64)
      return refine_real<double>(f, A, lda, X, ldx, init, maxit, tol, st, info, tm);
    return refine_real<float>(f, A, lda, X, ldx, init, maxit, tol, st, info, tm);
  }
  if (f->prec == MSQRT_PREC_FP64)
    return refine_general<double>(f, A, lda, X, ldx, init, maxit, tol, st, info, tm);
  return refine_general<float>(f, A, lda, X, ldx, init, maxit, tol, st, info, tm);
}

// ---------------------------------------------------------------------------
// Backward: the adjoint of the Frechet derivative of the square root,
// X G + G X = Gbar (X symmetric), solved in the factor's eigenbasis in low
// precision and refined with float64 residuals -- the correction framework
// of Sec. 2 applied to this linear equation.  The factor belongs to A/4^k,
// whose root is X_s = X 2^-k; X_s G' + G' X_s = Gbar gives G = 2^-k G'.

template <typename T>
static msqrt_status backward_hpd(Factor* f, const double* X, int64_t ldx, const double* Gbar,
                                 int64_t ldgb, double* G, int64_t ldg, int64_t stride, int maxit,
                                 double tol, hipStream_t st, msqrt_info* info, PhaseTimer& tm) {
  const int n = (int)f->n, batch = (int)f->batch;
  const int64_t nn = (int64_t)n * n;
  const T* Q = f->Q.as<T>();
  const T* s = f->S.as<T>();
  double* Xs = f->best.ensure<double>(2 * nn * batch);  // scaled X, then T1
  double* T1 = Xs + nn * batch;
  T* W1 = f->ws1.ensure<T>(nn * batch);
  T* W2 = f->ws2.ensure<T>(nn * batch);
  const int ntile = (int)(ceil_div(n, 128) * ceil_div(n, 128));
  const int nt32 = (int)ceil_div(n, 32);
  double* part = f->part.ensure<double>((int64_t)std::max(ntile, nt32 * (nt32 + 1) / 2) * batch + 64);
  double* rn = f->rnorm.ensure<double>(2 * batch);
  int* flags = f->active.ensure<int>(batch);
  const bool split = f->prec == MSQRT_PREC_BF16SPLIT;
  // ||Gbar||_F per entry (and finiteness)
  tm.begin(MSQRT_T_VALIDATE);
  MSQRT_HIP(hipMemsetAsync(flags, 0, sizeof(int) * batch, st));
  const int nblk = launch_validate(st, n, Gbar, ldgb, stride, batch, 0, flags, part);
  launch_reduce_sqrt(st, part, nblk, batch, rn + batch);
  std::vector<double> gnorm(batch);
  std::vector<int> hflags(batch);
  MSQRT_HIP(hipMemcpyAsync(gnorm.data(), rn + batch, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipMemcpyAsync(hflags.data(), flags, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
  launch_cast_scale_f64_f64(st, n, X, ldx, stride, f->rscale_dev(), Xs, n, nn, batch);
  tm.end();
  MSQRT_HIP(hipStreamSynchronize(st));
  tm.collect();
  for (int b = 0; b < batch; ++b)
    if (hflags[b] & 1) {
      set_last_error("Gbar contains Inf or NaN");
      return MSQRT_ERR_NONFINITE;
    }
  std::vector<std::vector<double>> hist(batch);
  std::vector<int> done(batch, 0), steps(batch, 0);
  std::vector<Verdict> verdict(batch, Verdict::Continue);
  std::vector<double> host_rn(batch);
  for (int it = 0;; ++it) {
    if (it == 0) {
      // G = 0: the residual is Gbar itself
      tm.begin(MSQRT_T_RESIDUAL);
      if (std::is_same<T, float>::value)
        launch_cast_scale_f64_f32(st, n, Gbar, ldgb, stride, nullptr, (float*)W1, n, nn, batch);
      else
        launch_cast_scale_f64_f64(st, n, Gbar, ldgb, stride, nullptr, (double*)W1, n, nn, batch);
      for (int b = 0; b < batch; ++b) {
        hist[b].push_back(gnorm[b] > 0.0 ? 1.0 : 0.0);
        if (gnorm[b] == 0.0) { done[b] = 1; verdict[b] = Verdict::Converged; }
      }
    } else {
      // R = Gbar - X_s G - G X_s  (float64), written as the float R_l
      tm.begin(MSQRT_T_RESIDUAL);
      launch_copy_f64(st, n, Gbar, ldgb, stride, T1, n, nn, batch);
      gemm_store_f64(st, false, false, n, n, n, Xs, n, nn, G, ldg, stride, T1, n, nn, -1.0, 1.0,
                     batch, false);
      int nt;
      if (std::is_same<T, float>::value)
        nt = gemm_residual_general(st, n, G, ldg, stride, Xs, n, nn, T1, n, nn, (float*)W1, nullptr,
                                   n, nn, part, batch);
      else
        nt = gemm_residual_general(st, n, G, ldg, stride, Xs, n, nn, T1, n, nn, nullptr,
                                   (double*)W1, n, nn, part, batch);
      launch_reduce_sqrt(st, part, nt, batch, rn);
      MSQRT_HIP(hipMemcpyAsync(host_rn.data(), rn, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
      tm.end();
      MSQRT_HIP(hipStreamSynchronize(st));
      tm.collect();
      for (int b = 0; b < batch; ++b) {
        if (done[b]) continue;
        hist[b].push_back(host_rn[b] / gnorm[b]);
        Verdict v = judge_step(hist[b], tol, it, maxit);
        if (v != Verdict::Continue) { done[b] = 1; verdict[b] = v; }
      }
    }
    bool all_done = true;
    for (int b = 0; b < batch; ++b) all_done = all_done && done[b];
    if (all_done && it > 0) break;
    // correction in the eigenbasis:  G (+)= Q [(Q^T R Q) ./ (s_i + s_j)] Q^T
    tm.begin(MSQRT_T_TRANSFORM);
    if (std::is_same<T, float>::value)
      gemm_store_f32(st, false, false, n, n, n, (const float*)W1, n, nn, (const float*)Q, n, nn,
                     (float*)W2, n, nn, 1.f, 0.f, batch, false, split);
    else
      gemm_store_f64(st, false, false, n, n, n, (const double*)W1, n, nn, (const double*)Q, n, nn,
                     (double*)W2, n, nn, 1.0, 0.0, batch, false);
    gemm_diagsylv<T>(st, true, false, n, Q, n, nn, W2, n, nn, s, n, W1, n, nn, batch, false, split);
    tm.begin(MSQRT_T_UPDATE);
    if (std::is_same<T, float>::value)
      gemm_store_f32(st, false, false, n, n, n, (const float*)Q, n, nn, (const float*)W1, n, nn,
                     (float*)W2, n, nn, 1.f, 0.f, batch, false, split);
    else
      gemm_store_f64(st, false, false, n, n, n, (const double*)Q, n, nn, (const double*)W1, n, nn,
                     (double*)W2, n, nn, 1.0, 0.0, batch, false);
    if (it == 0)
      gemm_set_f64<T>(st, false, true, n, n, W2, n, nn, Q, n, nn, G, ldg, stride, batch, false,
                      split);
    else
      gemm_update<T>(st, false, true, n, n, W2, n, nn, Q, n, nn, G, ldg, stride, nullptr, batch,
                     false, split);
    tm.end();
    for (int b = 0; b < batch; ++b)
      if (!done[b]) steps[b]++;
  }
  // G = 2^-k G'
  launch_scale_inplace(st, n, G, ldg, stride, f->rscale_dev(), batch);
  MSQRT_HIP(hipStreamSynchronize(st));
  tm.collect();
  msqrt_status status = MSQRT_OK;
  int max_steps = 0;
  double max_r = 0.0;
  for (int b = 0; b < batch; ++b) {
    max_steps = std::max(max_steps, steps[b]);
    max_r = std::max(max_r, hist[b].back());
    if (verdict[b] == Verdict::Diverged) status = MSQRT_ERR_DIVERGED;
    else if (verdict[b] != Verdict::Converged && status == MSQRT_OK) status = MSQRT_ERR_NOT_CONVERGED;
  }
  if (info) {
    info->steps = max_steps;
    info->relres = max_r;
    info->nhist = (int)std::min<size_t>(64, hist[0].size());
    for (int k = 0; k < info->nhist; ++k) info->relres_hist[k] = hist[0][k];
    info->prec_used = f->prec;
    info->struct_used = f->structure;
    info->scale_exp = f->kexp.empty() ? 0 : f->kexp[0];
  }
  return status;
}

msqrt_status backward(Factor* f, const double* X, int64_t ldx, const double* Gbar, int64_t ldgb,
                      double* G, int64_t ldg, int64_t stride, int maxit, double tol,
                      hipStream_t st, msqrt_info* info, PhaseTimer& tm) {
  if (f->batch > 1 && stride < std::max(std::max(ldx, ldgb), ldg) * f->n) {
    set_last_error("msqrt_sqrtm_backward: batch stride too small");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (f->structure == MSQRT_STRUCT_HPD) {
    if (f->prec == MSQRT_PREC_FP64)
      return backward_hpd<double>(f, X, ldx, Gbar, ldgb, G, ldg, stride, maxit, tol, st, info, tm);
    return backward_hpd<float>(f, X, ldx, Gbar, ldgb, G, ldg, stride, maxit, tol, st, info, tm);
  }
  if (f->real_schur) {
    if (f->prec == MSQRT_PREC_FP64)
      return backward_real<double>(f, X, ldx, Gbar, ldgb, G, ldg, maxit, tol, st, info, tm);
    return backward_real<float>(f, X, ldx, Gbar, ldgb, G, ldg, maxit, tol, st, info, tm);
  }
  if (f->prec == MSQRT_PREC_FP64)
    return backward_general<double>(f, X, ldx, Gbar, ldgb, G, ldg, maxit, tol, st, info, tm);
  return backward_general<float>(f, X, ldx, Gbar, ldgb, G, ldg, maxit, tol, st, info, tm);
}

// Finiteness (bit 0) and exact symmetry failures (bit 1) of a batch of
// matrices, without touching the factor's scales.
int validate_flags(Factor* f, const double* M, int64_t ld, int64_t sM, hipStream_t st,
                   const RefineWs* ws) {
  const int n = (int)f->n, batch = (int)f->batch;
  const int nt = (int)ceil_div(n, 32);
  int* flags = ws ? ws->flags : f->active.ensure<int>(batch);
  double* part = ws ? ws->part : f->part.ensure<double>((int64_t)nt * (nt + 1) / 2 * batch + 64);
  launch_fill_i32(st, flags, batch, 0);
  launch_validate(st, n, M, ld, sM, batch, 1, flags, part);
  std::vector<int> hf(batch);
  MSQRT_HIP(hipMemcpyAsync(hf.data(), flags, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipStreamSynchronize(st));
  int agg = 0;
  for (int b = 0; b < batch; ++b) agg |= hf[b];
  return agg;
}

// Computes ||A_b||_F and the scale exponents k_b = round(log4(||A_b||_F / sqrt(n)))
// into the factor; also validates finiteness / symmetry.  Returns flags.
int analyse_input(Factor* f, const double* A, int64_t lda, int64_t sA, bool check_sym,
                  hipStream_t st, const RefineWs* ws) {
  const int n = (int)f->n, batch = (int)f->batch;
  const int nt = (int)ceil_div(n, 32);
  const int nblk = nt * (nt + 1) / 2;
  int* flags = ws ? ws->flags : f->active.ensure<int>(batch);
  double* part = ws ? ws->part : f->part.ensure<double>((int64_t)nblk * batch + 64);
  double* rn = ws ? ws->rn : f->rnorm.ensure<double>(batch);
  launch_fill_i32(st, flags, batch, 0);
  launch_validate(st, n, A, lda, sA, batch, check_sym ? 1 : 0, flags, part);
  launch_reduce_sqrt(st, part, nblk, batch, rn);
  std::vector<int> hf(batch);
  std::vector<double> hn(batch);
  MSQRT_HIP(hipMemcpyAsync(hf.data(), flags, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipMemcpyAsync(hn.data(), rn, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipStreamSynchronize(st));
  int agg = 0;
  f->kexp.assign(batch, 0);
  f->anorm.assign(batch, 0.0);
  for (int b = 0; b < batch; ++b) {
    agg |= hf[b];
    f->anorm[b] = hn[b];
    int k = 0;
    if (hn[b] > 0 && std::isfinite(hn[b])) k = (int)std::lround(std::log(hn[b] / std::sqrt((double)n)) / std::log(4.0));
    f->kexp[b] = k;
  }
  f->upload_scales(st);
  return agg;
}

}  // namespace msqrt

using namespace msqrt;

// ---------------------------------------------------------------------------
// C-ABI

#define MSQRT_API_BEGIN try {
#define MSQRT_API_END                                                                   \
  }                                                                                     \
  catch (const Error& e) {                                                              \
    set_last_error(e.msg);                                                              \
    return (msqrt_status)e.status;                                                      \
  }                                                                                     \
  catch (const std::bad_alloc&) {                                                       \
    set_last_error("host allocation failed");                                           \
    return MSQRT_ERR_OUT_OF_MEMORY;                                                     \
  }                                                                                     \
  catch (...) {                                                                         \
    set_last_error("unknown error");                                                    \
    return MSQRT_ERR_DEVICE;                                                            \
  }

namespace {
int embed_and_check(int64_t n, int64_t batch, const void* dA, int64_t lda, int64_t strideA,
                    double* E, hipStream_t st);
}  // namespace

extern "C" {

void msqrt_default_options(msqrt_options* o) {
  if (!o) return;
  o->prec = MSQRT_PREC_FP32;
  o->structure = MSQRT_STRUCT_AUTO;
  o->maxit = 30;
  o->tol = 1e-13;
  o->blks = 32;
  o->fallback = 1;
  o->batch = 1;
  o->real_schur = 1;
}

const char* msqrt_status_string(msqrt_status s) {
  switch (s) {
    case MSQRT_OK: return "ok";
    case MSQRT_ERR_INVALID_ARG: return "invalid argument";
    case MSQRT_ERR_NONFINITE: return "non-finite input";
    case MSQRT_ERR_NO_PRINCIPAL: return "no principal square root (eigenvalue on R<=0)";
    case MSQRT_ERR_NOT_CONVERGED: return "refinement did not converge";
    case MSQRT_ERR_DIVERGED: return "refinement diverged";
    case MSQRT_ERR_DEVICE: return "device error";
    case MSQRT_ERR_OUT_OF_MEMORY: return "out of memory";
    case MSQRT_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* msqrt_last_error(void) { return g_last_error.c_str(); }

void msqrt_release_cached(void) {
  try {
    pool_release();
    prof_release();
    selector_release();
  } catch (...) {
  }
}

void msqrt_factor_destroy(msqrt_factor_t f) { delete reinterpret_cast<Factor*>(f); }

static msqrt_status check_common(msqrt_dtype dtype, int64_t n, const void* A, int64_t lda,
                                 int64_t batch) {
  if (n < 0 || batch < 1 || (n > 0 && (A == nullptr || lda < n))) {
    set_last_error("invalid size, pointer or leading dimension");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (n > (int64_t)1 << 30) {
    set_last_error("n too large");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (dtype != MSQRT_REAL64 && dtype != MSQRT_COMPLEX128) {
    set_last_error("unknown dtype");
    return MSQRT_ERR_INVALID_ARG;
  }
  return MSQRT_OK;
}

msqrt_status msqrt_factor_wrap(msqrt_prec prec, msqrt_struct structure, msqrt_dtype dtype,
                               int64_t n, const void* Qp, const void* Sp, int on_device,
                               msqrt_factor_t* out) {
  MSQRT_API_BEGIN
  if (!out || n < 1 || !Qp || !Sp) {
    set_last_error("invalid argument");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (dtype != MSQRT_REAL64 || structure != MSQRT_STRUCT_HPD) {
    set_last_error("factor_wrap supports real HPD factors in this build");
    return MSQRT_ERR_UNSUPPORTED;
  }
  if (prec != MSQRT_PREC_FP32 && prec != MSQRT_PREC_FP64) {
    set_last_error("factor_wrap: prec must be FP32 or FP64");
    return MSQRT_ERR_INVALID_ARG;
  }
  std::unique_ptr<Factor> f(new Factor());
  f->n = n; f->batch = 1; f->dtype = dtype; f->structure = structure; f->prec = prec;
  const size_t es = prec == MSQRT_PREC_FP64 ? 8 : 4;
  f->Q.alloc(es * n * n);
  f->S.alloc(es * n);
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  MSQRT_HIP(hipMemcpy(f->Q.p, Qp, es * n * n, kind));
  MSQRT_HIP(hipMemcpy(f->S.p, Sp, es * n, kind));
  f->kexp.assign(1, 0);
  f->anorm.assign(1, 0.0);
  f->upload_scales(nullptr);
  MSQRT_HIP(hipDeviceSynchronize());
  *out = reinterpret_cast<msqrt_factor_t>(f.release());
  return MSQRT_OK;
  MSQRT_API_END
}

msqrt_status msqrt_factor_export(msqrt_factor_t fh, void* Qh, void* Sh, int* scale_exp) {
  MSQRT_API_BEGIN
  Factor* f = reinterpret_cast<Factor*>(fh);
  if (!f) return MSQRT_ERR_INVALID_ARG;
  const size_t es = f->prec == MSQRT_PREC_FP64 ? 8 : 4;
  const int64_t n = f->n;
  MSQRT_HIP(hipDeviceSynchronize());
  if (Qh) MSQRT_HIP(hipMemcpy(Qh, f->Q.p, es * n * n * f->batch, hipMemcpyDeviceToHost));
  const int64_t scount = f->real_schur ? n * n : n * f->batch;
  if (Sh) MSQRT_HIP(hipMemcpy(Sh, f->S.p, es * scount, hipMemcpyDeviceToHost));
  if (scale_exp) *scale_exp = f->kexp.empty() ? 0 : f->kexp[0];
  return MSQRT_OK;
  MSQRT_API_END
}

}  // extern "C"

namespace {

// Static scratch of the allocation-free refinement entry point: one copy per
// GPU, alive until the process ends.  Host code never uses the array's name
// as an address; it takes each device's address from hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_addr;  // device -> address of its scratch

// Address of the current device's scratch, looked up once per device.
unsigned char* scratch_address() {
  int dev = 0;
  MSQRT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    throw Error{MSQRT_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
  }
  g_scratch_addr[dev] = (unsigned char*)p;
  return (unsigned char*)p;
}

// Carves the workspace of one HPD refinement call out of `base` (256-byte
// aligned pieces); returns the bytes needed (base may be null to size it).
size_t carve_refine_ws(const Factor* f, unsigned char* base, RefineWs* ws) {
  const int64_t n = f->n, batch = f->batch, nn = n * n;
  const size_t es = f->prec == MSQRT_PREC_FP64 ? 8 : 4;
  const int64_t nt = ceil_div(n, 32);
  const int64_t nparts = std::max<int64_t>(residual_tiles((int)n), nt * (nt + 1) / 2) * batch + 64;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + off : nullptr;
    off += up(bytes);
    return p;
  };
  ws->w1 = take(es * nn * batch);
  ws->w2 = take(es * nn * batch);
  ws->best = (double*)take(sizeof(double) * nn * batch);
  ws->part = (double*)take(sizeof(double) * nparts);
  ws->rn = (double*)take(sizeof(double) * batch);
  ws->flags = (int*)take(sizeof(int) * batch);
  return off;
}

// msqrt_refine with the factor's cached buffers (ws = null) or a caller
// workspace.  With a workspace nothing is allocated on the device and no
// phase timers are recorded (info->t_ms stays zero).
msqrt_status refine_call(Factor* f, const void* dA, int64_t lda, int64_t strideA, void* dX,
                         int64_t ldx, int64_t strideX, int init_from_factor, int maxit, double tol,
                         hipStream_t stream, msqrt_info* info, const RefineWs* ws) {
  if (!f || !dA || !dX || lda < f->n || ldx < f->n || maxit < 0 || std::isnan(tol)) {
    set_last_error("msqrt_refine: invalid argument");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (f->batch > 1 && (strideA < lda * f->n || strideX < ldx * f->n)) {
    set_last_error("msqrt_refine: batch strides too small");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (info) { std::memset(info, 0, sizeof(*info)); info->prec_used = f->prec; info->struct_used = f->structure; }
  PhaseTimer tm(stream, ws ? nullptr : info);
  // ||A||_F of the (scaled) matrix the refinement measures against.  The
  // factor's scale exponents are kept; the norm is recomputed because A may be
  // a nearby matrix.
  {
    std::vector<int> k = f->kexp;
    int flags = 0;
    if (f->structure == MSQRT_STRUCT_GENERAL) {
      flags = analyse_input_general(f, (const double*)dA, lda, f->dtype == MSQRT_COMPLEX128, stream) & 1;
    } else {
      // An HPD factor refines a symmetric A from a symmetric X: the residual
      // is formed as A - X X^T from the lower triangle, which equals A - X^2
      // only for exactly symmetric A and X.
      flags = analyse_input(f, (const double*)dA, lda, strideA, true, stream, ws);
      if (!init_from_factor && !(flags & 3))
        flags |= validate_flags(f, (const double*)dX, ldx, strideX, stream, ws);
    }
    f->kexp = k;
    f->upload_scales(stream);
    if (flags & 1) {
      set_last_error("msqrt_refine: A or X holds Inf or NaN");
      return MSQRT_ERR_NONFINITE;
    }
    if (flags & 2) {
      set_last_error("msqrt_refine: an HPD factor needs an exactly symmetric A and starting X");
      return MSQRT_ERR_INVALID_ARG;
    }
  }
  for (int64_t b = 0; b < f->batch; ++b) f->anorm_scaled[b] = f->anorm[b] * std::ldexp(1.0, -2 * f->kexp[b]);
  double* X = (double*)dX;
  if (f->structure == MSQRT_STRUCT_GENERAL) {
    msqrt_status s = refine(f, (const double*)dA, lda, strideA, X, ldx, strideX, init_from_factor,
                            maxit, tol, stream, info, tm);
    MSQRT_HIP(hipStreamSynchronize(stream));
    tm.collect();
    if (info) info->scale_exp = f->kexp.empty() ? 0 : f->kexp[0];
    return s;
  }
  // Refinement runs on the scaled problem A/4^k: bring X to that scale.
  launch_scale_inplace(stream, (int)f->n, X, ldx, strideX, f->rscale_dev(), (int)f->batch);
  msqrt_status s = refine(f, (const double*)dA, lda, strideA, X, ldx, strideX, init_from_factor,
                          maxit, tol, stream, info, tm, ws);
  launch_scale_inplace(stream, (int)f->n, X, ldx, strideX, f->uscale_dev(), (int)f->batch);
  MSQRT_HIP(hipStreamSynchronize(stream));
  tm.collect();
  if (info) info->scale_exp = f->kexp.empty() ? 0 : f->kexp[0];
  return s;
}

}  // namespace

extern "C" {

msqrt_status msqrt_refine(msqrt_factor_t fh, const void* dA, int64_t lda, int64_t strideA,
                          void* dX, int64_t ldx, int64_t strideX, int init_from_factor, int maxit,
                          double tol, hipStream_t stream, msqrt_info* info) {
  MSQRT_API_BEGIN
  Factor* f = reinterpret_cast<Factor*>(fh);
  if (f && f->embed) {
    // complex Hermitian: refine the real representations of A and X
    const int64_t n = f->n / 2, n2 = f->n, s2 = n2 * n2;
    if (!dA || !dX || lda < n || ldx < n) {
      set_last_error("msqrt_refine: invalid argument");
      return MSQRT_ERR_INVALID_ARG;
    }
    DevBuf eb, xb;
    double* E = eb.ensure<double>(s2 * f->batch);
    double* XE = xb.ensure<double>(s2 * f->batch);
    launch_embed_complex(stream, (int)n, (const double*)dA, lda, 2 * strideA, E, s2, (int)f->batch);
    if (!init_from_factor)
      launch_embed_complex(stream, (int)n, (const double*)dX, ldx, 2 * strideX, XE, s2, (int)f->batch);
    const msqrt_status st = refine_call(f, E, n2, s2, XE, n2, s2, init_from_factor, maxit, tol,
                                        stream, info, nullptr);
    if (st == MSQRT_OK || st == MSQRT_ERR_NOT_CONVERGED || st == MSQRT_ERR_DIVERGED) {
      launch_extract_complex(stream, (int)n, XE, s2, (double*)dX, ldx, 2 * strideX, (int)f->batch);
      MSQRT_HIP(hipStreamSynchronize(stream));
    }
    return st;
  }
  return refine_call(f, dA, lda, strideA, dX, ldx, strideX, init_from_factor, maxit, tol, stream,
                     info, nullptr);
  MSQRT_API_END
}

msqrt_status msqrt_refine_noalloc(msqrt_factor_t fh, const void* dA, int64_t lda,
                                  int64_t strideA, void* dX, int64_t ldx, int64_t strideX,
                                  int init_from_factor, int maxit, double tol, hipStream_t stream,
                                  msqrt_info* info) {
  MSQRT_API_BEGIN
  Factor* f = reinterpret_cast<Factor*>(fh);
  if (!f) {
    set_last_error("msqrt_refine_noalloc: invalid argument");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (f->structure != MSQRT_STRUCT_HPD || f->embed) {
    set_last_error("msqrt_refine_noalloc: real HPD factors only");
    return MSQRT_ERR_UNSUPPORTED;
  }
  RefineWs ws;
  const size_t need = carve_refine_ws(f, nullptr, &ws);
  if (need > kNoAllocScratchBytes) {
    set_last_error("msqrt_refine_noalloc: n = " + std::to_string(f->n) + ", batch = " +
                   std::to_string(f->batch) + " needs " + std::to_string(need) +
                   " bytes of scratch; the static scratch holds " +
                   std::to_string(kNoAllocScratchBytes) + " bytes");
    return MSQRT_ERR_INVALID_ARG;
  }
  carve_refine_ws(f, scratch_address(), &ws);
  return refine_call(f, dA, lda, strideA, dX, ldx, strideX, init_from_factor, maxit, tol, stream,
                     info, &ws);
  MSQRT_API_END
}

msqrt_status msqrt_factor(const msqrt_options* opt, msqrt_dtype dtype, int64_t n, const void* dA,
                          int64_t lda, int64_t strideA, hipStream_t stream, msqrt_factor_t* out) {
  MSQRT_API_BEGIN
  msqrt_options o;
  msqrt_default_options(&o);
  if (opt) o = *opt;
  msqrt_status cs = check_common(dtype, n, dA, lda, o.batch);
  if (cs != MSQRT_OK) return cs;
  if (!out) return MSQRT_ERR_INVALID_ARG;
  std::unique_ptr<Factor> f(new Factor());
  f->n = n; f->batch = o.batch; f->dtype = dtype; f->blks = o.blks;
  if (dtype == MSQRT_COMPLEX128 && o.structure != MSQRT_STRUCT_GENERAL && n > 0 &&
      2 * n <= sytrd_max_n()) {
    // complex Hermitian input: HPD factor of the real representation
    const int64_t n2 = 2 * n, s2 = n2 * n2;
    DevBuf eb;
    double* E = eb.ensure<double>(s2 * o.batch);
    const int flags = embed_and_check(n, o.batch, dA, lda, strideA, E, stream);
    if (flags & 1) {
      set_last_error("input contains Inf or NaN");
      return MSQRT_ERR_NONFINITE;
    }
    if (!(flags & 2)) {
      msqrt_options oe = o;
      oe.structure = MSQRT_STRUCT_HPD;
      f->n = n2;
      f->dtype = MSQRT_REAL64;
      msqrt_status st = build_factor(f.get(), oe, E, n2, s2, stream, nullptr);
      if (st != MSQRT_OK) return st;
      f->embed = true;
      f->dtype = MSQRT_COMPLEX128;
      *out = reinterpret_cast<msqrt_factor_t>(f.release());
      return MSQRT_OK;
    }
    if (o.structure == MSQRT_STRUCT_HPD) {
      set_last_error("structure HPD requested but the input is not exactly Hermitian");
      return MSQRT_ERR_INVALID_ARG;
    }
  }
  msqrt_status st = build_factor(f.get(), o, (const double*)dA, lda, strideA, stream, nullptr);
  if (st != MSQRT_OK) return st;
  *out = reinterpret_cast<msqrt_factor_t>(f.release());
  return MSQRT_OK;
  MSQRT_API_END
}

}  // extern "C"

namespace {

// The solve of msqrt_sqrtm after argument checks: factor, refinement and
// precision escalation.
msqrt_status sqrtm_impl(const msqrt_options& o, msqrt_dtype dtype, int64_t n, const void* dA,
                        int64_t lda, int64_t strideA, void* dX, int64_t ldx, int64_t strideX,
                        hipStream_t stream, msqrt_info* info, msqrt_factor_t* keep,
                        PhaseTimer& tm) {

  msqrt_prec prec = o.prec;
  if (prec == MSQRT_PREC_AUTO) prec = select_precision(o, dtype, n, dA, lda, strideA, stream, info, tm);
  msqrt_status last = MSQRT_ERR_DEVICE;
  int fallbacks = 0;
  std::unique_ptr<Factor> reuse;  // float factor kept for the BF16SPLIT -> FP32 step
  for (;;) {
    std::unique_ptr<Factor> f;
    msqrt_status st = MSQRT_OK;
    if (reuse) {
      // BF16SPLIT and FP32 share the float factorisation: escalate by
      // repeating only the refinement with float transforms
      f = std::move(reuse);
      f->prec = prec;
    } else {
      f.reset(new Factor());
      f->n = n; f->batch = o.batch; f->dtype = dtype; f->blks = o.blks;
      msqrt_options oo = o;
      oo.prec = prec;
      st = build_factor(f.get(), oo, (const double*)dA, lda, strideA, stream, &tm);
    }
    if (st == MSQRT_OK) {
      for (int64_t b = 0; b < f->batch; ++b) f->anorm_scaled[b] = f->anorm[b] * std::ldexp(1.0, -2 * f->kexp[b]);
      st = refine(f.get(), (const double*)dA, lda, strideA, (double*)dX, ldx, strideX, 1, o.maxit,
                  o.tol, stream, info, tm);
      if (f->structure == MSQRT_STRUCT_HPD) {
        tm.begin(MSQRT_T_VALIDATE);
        launch_scale_inplace(stream, (int)n, (double*)dX, ldx, strideX, f->uscale_dev(), (int)o.batch);
        tm.end();
      }
      MSQRT_HIP(hipStreamSynchronize(stream));
      tm.collect();
      if (info) { info->prec_used = prec; info->struct_used = f->structure; info->scale_exp = f->kexp[0]; }
    }
    last = st;
    const bool retryable = st == MSQRT_ERR_DIVERGED || st == MSQRT_ERR_NOT_CONVERGED ||
                           st == MSQRT_ERR_NO_PRINCIPAL;
    if (st == MSQRT_OK || !o.fallback || !retryable || prec == MSQRT_PREC_FP64) {
      if (keep && st == MSQRT_OK) *keep = reinterpret_cast<msqrt_factor_t>(f.release());
      break;
    }
    if (prec == MSQRT_PREC_BF16SPLIT && st != MSQRT_ERR_NO_PRINCIPAL) {
      // the float factor itself was usable: retry its refinement in FP32
      prec = MSQRT_PREC_FP32;
      reuse = std::move(f);
    } else {
      // a failed float factorisation fails again in FP32: go to FP64
      prec = MSQRT_PREC_FP64;
    }
    ++fallbacks;
  }
  if (info) info->fallbacks = fallbacks;
  return last;
}

// Real representation of a batch of interleaved complex n x n matrices into
// E (2n x 2n per entry, ld 2n, stride 4n^2).  Returns the validation flags of
// E (bit0 non-finite, bit1 E not exactly symmetric, i.e. A not exactly
// Hermitian).
int embed_and_check(int64_t n, int64_t batch, const void* dA, int64_t lda, int64_t strideA,
                    double* E, hipStream_t st) {
  const int64_t n2 = 2 * n, s2 = n2 * n2;
  launch_embed_complex(st, (int)n, (const double*)dA, lda, 2 * strideA, E, s2, (int)batch);
  DevBuf fl, pt;
  int* flags = fl.ensure<int>(batch);
  const int64_t nt = ceil_div(n2, 32);
  double* part = pt.ensure<double>(nt * (nt + 1) / 2 * batch + 64);
  launch_fill_i32(st, flags, (int)batch, 0);
  launch_validate(st, (int)n2, E, n2, s2, (int)batch, 1, flags, part);
  std::vector<int> hf(batch);
  MSQRT_HIP(hipMemcpyAsync(hf.data(), flags, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
  MSQRT_HIP(hipStreamSynchronize(st));
  int agg = 0;
  for (int v : hf) agg |= v;
  return agg;
}

// Complex Hermitian positive definite input (Alg. 3 over C): the principal
// root of A is read off the principal root of its real representation E,
// which the real symmetric route computes (E is symmetric positive definite
// exactly when A is Hermitian positive definite, and the representation is
// an algebra homomorphism, so sqrt(E) represents sqrt(A)).  *handled is
// false when the input is not exactly Hermitian under structure AUTO or too
// large for the symmetric route: the caller then takes the general path.
msqrt_status sqrtm_hermitian(const msqrt_options& o, int64_t n, const void* dA, int64_t lda,
                             int64_t strideA, void* dX, int64_t ldx, int64_t strideX,
                             hipStream_t stream, msqrt_info* info, msqrt_factor_t* keep,
                             PhaseTimer& tm, bool* handled) {
  *handled = false;
  const int64_t n2 = 2 * n, s2 = n2 * n2;
  if (n2 > sytrd_max_n()) {
    if (o.structure != MSQRT_STRUCT_HPD) return MSQRT_OK;
    *handled = true;
    set_last_error("complex Hermitian route supports n <= " + std::to_string(sytrd_max_n() / 2));
    return MSQRT_ERR_UNSUPPORTED;
  }
  DevBuf eb, xb;
  double* E = eb.ensure<double>(s2 * o.batch);
  double* XE = xb.ensure<double>(s2 * o.batch);
  tm.begin(MSQRT_T_VALIDATE);
  const int flags = embed_and_check(n, o.batch, dA, lda, strideA, E, stream);
  tm.end();
  if (flags & 1) {
    *handled = true;
    set_last_error("input contains Inf or NaN");
    return MSQRT_ERR_NONFINITE;
  }
  if (flags & 2) {
    if (o.structure != MSQRT_STRUCT_HPD) return MSQRT_OK;
    *handled = true;
    set_last_error("structure HPD requested but the input is not exactly Hermitian");
    return MSQRT_ERR_INVALID_ARG;
  }
  *handled = true;
  msqrt_options oe = o;
  oe.structure = MSQRT_STRUCT_HPD;
  msqrt_factor_t kf = nullptr;
  const msqrt_status st = sqrtm_impl(oe, MSQRT_REAL64, n2, E, n2, s2, XE, n2, s2, stream, info,
                                     keep ? &kf : nullptr, tm);
  if (st == MSQRT_OK || st == MSQRT_ERR_NOT_CONVERGED || st == MSQRT_ERR_DIVERGED) {
    launch_extract_complex(stream, (int)n, XE, s2, (double*)dX, ldx, 2 * strideX, (int)o.batch);
    MSQRT_HIP(hipStreamSynchronize(stream));
  }
  if (kf) {
    reinterpret_cast<Factor*>(kf)->embed = true;
    reinterpret_cast<Factor*>(kf)->dtype = MSQRT_COMPLEX128;
    *keep = kf;
  }
  return st;
}

}  // namespace

extern "C" {

msqrt_status msqrt_sqrtm(const msqrt_options* opt, msqrt_dtype dtype, int64_t n, const void* dA,
                         int64_t lda, int64_t strideA, void* dX, int64_t ldx, int64_t strideX,
                         hipStream_t stream, msqrt_info* info, msqrt_factor_t* keep) {
  MSQRT_API_BEGIN
  msqrt_options o;
  msqrt_default_options(&o);
  if (opt) o = *opt;
  msqrt_status cs = check_common(dtype, n, dA, lda, o.batch);
  if (cs != MSQRT_OK) return cs;
  if (n > 0 && (!dX || ldx < n)) return MSQRT_ERR_INVALID_ARG;
  if (o.batch > 1 && (strideA < lda * n || strideX < ldx * n)) {
    set_last_error("batch strides too small");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  if (keep) *keep = nullptr;
  if (n == 0) return MSQRT_OK;
  PhaseTimer tm(stream, info);
  if (dtype == MSQRT_COMPLEX128 && o.structure != MSQRT_STRUCT_GENERAL) {
    bool handled = false;
    msqrt_status st = sqrtm_hermitian(o, n, dA, lda, strideA, dX, ldx, strideX, stream, info, keep,
                                      tm, &handled);
    if (handled) return st;
  }
  return sqrtm_impl(o, dtype, n, dA, lda, strideA, dX, ldx, strideX, stream, info, keep, tm);
  MSQRT_API_END
}

msqrt_status msqrt_rootm(const msqrt_options* opt, int p, msqrt_dtype dtype, int64_t n,
                         const void* dA, int64_t lda, void* dX, int64_t ldx, hipStream_t stream,
                         msqrt_info* info) {
  MSQRT_API_BEGIN
  msqrt_options o;
  msqrt_default_options(&o);
  if (opt) o = *opt;
  if (p == 2) {
    o.batch = 1;
    return msqrt_sqrtm(&o, dtype, n, dA, lda, lda * n, dX, ldx, ldx * n, stream, info, nullptr);
  }
  if (p != 3) {
    set_last_error("msqrt_rootm: p must be 2 or 3");
    return MSQRT_ERR_UNSUPPORTED;
  }
  msqrt_status cs = check_common(dtype, n, dA, lda, 1);
  if (cs != MSQRT_OK) return cs;
  if (n > 0 && (!dX || ldx < n)) return MSQRT_ERR_INVALID_ARG;
  if (o.batch != 1) {
    set_last_error("msqrt_rootm: one matrix per call");
    return MSQRT_ERR_UNSUPPORTED;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return MSQRT_OK;
  PhaseTimer tm(stream, info);
  const int cplx = dtype == MSQRT_COMPLEX128;
  msqrt_prec prec = o.prec == MSQRT_PREC_FP64 ? MSQRT_PREC_FP64 : MSQRT_PREC_FP32;
  msqrt_status last = MSQRT_ERR_DEVICE;
  int fallbacks = 0;
  for (;;) {
    Factor f;
    f.n = n; f.batch = 1; f.dtype = dtype; f.blks = o.blks; f.root = 3;
    f.structure = MSQRT_STRUCT_GENERAL;
    f.prec = prec;
    tm.begin(MSQRT_T_VALIDATE);
    const int flags = analyse_input_general(&f, (const double*)dA, lda, cplx, stream);
    tm.end();
    if (flags & 1) {
      set_last_error("input contains Inf or NaN");
      return MSQRT_ERR_NONFINITE;
    }
    msqrt_status st = prec == MSQRT_PREC_FP64
                          ? factor_root3<double>(&f, (const double*)dA, lda, cplx, stream, &tm)
                          : factor_root3<float>(&f, (const double*)dA, lda, cplx, stream, &tm);
    if (st == MSQRT_OK)
      st = prec == MSQRT_PREC_FP64
               ? refine_root3<double>(&f, (const double*)dA, lda, (double*)dX, ldx, 1, o.maxit,
                                      o.tol, stream, info, tm)
               : refine_root3<float>(&f, (const double*)dA, lda, (double*)dX, ldx, 1, o.maxit,
                                     o.tol, stream, info, tm);
    MSQRT_HIP(hipStreamSynchronize(stream));
    tm.collect();
    if (info) {
      info->prec_used = prec;
      info->struct_used = MSQRT_STRUCT_GENERAL;
      info->scale_exp = f.kexp.empty() ? 0 : f.kexp[0];
    }
    last = st;
    const bool retryable = st == MSQRT_ERR_DIVERGED || st == MSQRT_ERR_NOT_CONVERGED ||
                           st == MSQRT_ERR_NO_PRINCIPAL;
    if (st == MSQRT_OK || !o.fallback || !retryable || prec == MSQRT_PREC_FP64) break;
    prec = MSQRT_PREC_FP64;
    ++fallbacks;
  }
  if (info) info->fallbacks = fallbacks;
  return last;
  MSQRT_API_END
}

msqrt_status msqrt_sqrtm_backward(msqrt_factor_t fh, const void* dX, int64_t ldx,
                                  const void* dGbar, int64_t ldgb, void* dG, int64_t ldg,
                                  int64_t stride, int maxit, double tol, hipStream_t stream,
                                  msqrt_info* info) {
  MSQRT_API_BEGIN
  Factor* f = reinterpret_cast<Factor*>(fh);
  const int64_t nu = f ? (f->embed ? f->n / 2 : f->n) : 0;  // the caller's order
  if (!f || !dX || !dGbar || !dG || ldx < nu || ldgb < nu || ldg < nu || maxit < 0) {
    set_last_error("msqrt_sqrtm_backward: invalid argument");
    return MSQRT_ERR_INVALID_ARG;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  PhaseTimer tm(stream, info);
  if (f->embed) {
    // complex Hermitian X: X G + G X = Gbar holds exactly when the real
    // representations satisfy the same equation
    const int64_t n = f->n / 2, n2 = f->n, s2 = n2 * n2;
    DevBuf xb, gb, ob;
    double* XE = xb.ensure<double>(s2 * f->batch);
    double* GB = gb.ensure<double>(s2 * f->batch);
    double* GE = ob.ensure<double>(s2 * f->batch);
    launch_embed_complex(stream, (int)n, (const double*)dX, ldx, 2 * stride, XE, s2, (int)f->batch);
    launch_embed_complex(stream, (int)n, (const double*)dGbar, ldgb, 2 * stride, GB, s2,
                         (int)f->batch);
    const msqrt_status st = backward(f, XE, n2, GB, n2, GE, n2, s2, maxit, tol, stream, info, tm);
    if (st == MSQRT_OK || st == MSQRT_ERR_NOT_CONVERGED || st == MSQRT_ERR_DIVERGED) {
      launch_extract_complex(stream, (int)n, GE, s2, (double*)dG, ldg, 2 * stride, (int)f->batch);
      MSQRT_HIP(hipStreamSynchronize(stream));
    }
    return st;
  }
  return backward(f, (const double*)dX, ldx, (const double*)dGbar, ldgb, (double*)dG, ldg, stride,
                  maxit, tol, stream, info, tm);
  MSQRT_API_END
}

}  // extern "C"
