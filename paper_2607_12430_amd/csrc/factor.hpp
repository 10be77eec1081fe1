// Factor object and the host-side pieces shared between the runtime files.
#pragma once

#include <cmath>
#include <vector>

#include "../../include/msqrt.h"
#include "common.hpp"

namespace msqrt {

// Process-wide cache of device allocations keyed by (device, size), so that
// repeated solves of the same size do not pay for hipMalloc / hipFree.
void* pool_alloc(size_t bytes);
void pool_free(void* p, size_t bytes);

// Owning device allocation that only grows.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) pool_free(p, bytes);
  }
  void alloc(size_t b) {
    if (p && b <= bytes) return;
    if (p) pool_free(p, bytes);
    p = nullptr;
    bytes = 0;
    if (b == 0) return;
    // round up to 1 MiB granules above 1 MiB so near sizes share cache entries
    const size_t g = b > (1u << 20) ? ((b + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1)) : ((b + 255) & ~(size_t)255);
    p = pool_alloc(g);
    bytes = g;
  }
  template <typename T>
  T* ensure(int64_t count) {
    alloc((size_t)count * sizeof(T));
    return (T*)p;
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

// Workspace of the tile-dataflow triangular solvers.
struct TrsylvWork {
  DevBuf flags, ticket;
};

struct Factor {
  int64_t n = 0, batch = 1;
  msqrt_dtype dtype = MSQRT_REAL64;
  msqrt_struct structure = MSQRT_STRUCT_HPD;
  msqrt_prec prec = MSQRT_PREC_FP32;
  int blks = 32;
  std::vector<int> kexp;             // A_b is scaled by 4^-kexp[b]
  std::vector<double> anorm;         // ||A_b||_F (unscaled)
  std::vector<double> anorm_scaled;  // ||A_b / 4^k||_F
  // The factor: Q (n x n per batch entry) and S (diagonal: n per entry;
  // general: n x n upper triangular), in the factor precision.
  DevBuf Q, S;
  DevBuf scales;  // [3 * batch] doubles: 4^-k, 2^-k, 2^k
  // refinement workspaces
  DevBuf ws1, ws2, part, rnorm, active, best;
  // factorisation workspaces
  DevBuf fw1, fw2, fw3, fw4, fw5;
  // general path: Q in the four layouts of the refinement products, the
  // wide float64 iterate and its stacked copy, the Sylvester right-hand side,
  // the per-plane residual scales and the tile-solver state
  DevBuf gq, gx, gt, gsc;
  bool gq_ready = false;
  // Complex Hermitian input solved through its real representation
  // [[Re A, -Im A], [Im A, Re A]]: n is 2 n_user and the factor is the HPD
  // factor of that real matrix.
  bool embed = false;
  // Root order p of the factor (2: square root; 3: cube root, Sec. 4): the
  // input is scaled by 2^(-p k), the root by 2^-k.
  int root = 2;
  // Real input on the general path with the real Schur form (remark on real
  // input in Sec. 2.2.1): Q real n x n, S = T^{1/2} real quasi-upper-
  // triangular n x n (both in the factor precision), qpart the device tile
  // partition of S (qnt tiles) that keeps every 2x2 block inside one tile.
  bool real_schur = false;
  DevBuf qpart;
  std::vector<int> qpart_h;
  int qnt = 0;
  TrsylvWork tw;

  void upload_scales(hipStream_t st) {
    const int64_t b = batch;
    std::vector<double> h(3 * b);
    anorm_scaled.assign(b, 0.0);
    for (int64_t i = 0; i < b; ++i) {
      const int k = kexp.empty() ? 0 : kexp[i];
      h[i] = std::ldexp(1.0, -root * k);
      h[b + i] = std::ldexp(1.0, -k);
      h[2 * b + i] = std::ldexp(1.0, k);
      if ((int64_t)anorm.size() > i) anorm_scaled[i] = anorm[i] * h[i];
    }
    double* d = scales.ensure<double>(3 * b);
    MSQRT_HIP(hipMemcpyAsync(d, h.data(), sizeof(double) * 3 * b, hipMemcpyHostToDevice, st));
    MSQRT_HIP(hipStreamSynchronize(st));
  }
  const double* ascale_dev() const { return scales.as<double>(); }
  const double* rscale_dev() const { return scales.as<double>() + batch; }
  const double* uscale_dev() const { return scales.as<double>() + 2 * batch; }
};

// Phase timers (hipEvents on the call's stream, read at the next sync point).

struct PhaseTimer {
  hipStream_t st;
  msqrt_info* info;
  struct Pending { int phase; hipEvent_t a, b; };
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  int cur = -1;
  hipEvent_t cur_ev = nullptr;
  PhaseTimer(hipStream_t s, msqrt_info* i) : st(s), info(i) {}
  ~PhaseTimer() {
    for (auto& p : pend) { pool.push_back(p.a); pool.push_back(p.b); }
    for (auto e : pool) hipEventDestroy(e);
    if (cur_ev) hipEventDestroy(cur_ev);
  }
  hipEvent_t ev() {
    hipEvent_t e;
    if (!pool.empty()) { e = pool.back(); pool.pop_back(); return e; }
    MSQRT_HIP(hipEventCreate(&e));
    return e;
  }
  void begin(int phase) {
    if (!info) return;
    end();
    cur = phase;
    cur_ev = ev();
    MSQRT_HIP(hipEventRecord(cur_ev, st));
  }
  void end() {
    if (!info || cur < 0) return;
    hipEvent_t e = ev();
    MSQRT_HIP(hipEventRecord(e, st));
    pend.push_back({cur, cur_ev, e});
    cur = -1;
    cur_ev = nullptr;
  }
  // Call after a stream synchronisation.
  void collect() {
    if (!info) return;
    for (auto& p : pend) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess && p.phase >= 0 && p.phase < 12)
        info->t_ms[p.phase] += ms;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pend.clear();
  }
};

// Convergence bookkeeping of every refinement loop: the stopping rule of
// Alg. 2 (relative residual <= tol) and the reading of the paper's remark
// that the iteration diverges for too ill-conditioned inputs (Sec. 5.1):
// diverged when the residual is not finite, exceeds 10x the first one or grew
// on two consecutive sweeps; stagnated when it failed to drop below 0.9x the
// previous one on two consecutive sweeps.  h holds every residual so far.
enum class Verdict { Continue, Converged, Diverged, Stagnated };

inline Verdict judge(const std::vector<double>& h, double tol) {
  const double r = h.back();
  if (!std::isfinite(r)) return Verdict::Diverged;
  if (r <= tol) return Verdict::Converged;
  if (r > 10.0 * h.front()) return Verdict::Diverged;
  const size_t k = h.size();
  if (k >= 3 && h[k - 1] > h[k - 2] && h[k - 2] > h[k - 3]) return Verdict::Diverged;
  if (k >= 3 && h[k - 1] > 0.9 * h[k - 2] && h[k - 2] > 0.9 * h[k - 3]) return Verdict::Stagnated;
  return Verdict::Continue;
}

// Verdict after residual number it (it = corrections applied so far).  A
// negative tol nullifies the stopping test, as the paper's accuracy
// experiments do (Sec. 5.1): exactly maxit corrections are applied and the
// last iterate is kept (a non-finite residual still stops the loop).
inline Verdict judge_step(const std::vector<double>& h, double tol, int it, int maxit) {
  if (tol < 0) {
    if (!std::isfinite(h.back())) return Verdict::Diverged;
    return it >= maxit ? Verdict::Converged : Verdict::Continue;
  }
  Verdict v = judge(h, tol);
  if (v == Verdict::Continue && it >= maxit) v = Verdict::Stagnated;
  return v;
}

// Validates A (finiteness, optional exact symmetry), computes ||A_b||_F and
// the scale exponents into f.  Returns the OR of the per-entry flags
// (bit0 non-finite, bit1 not symmetric).
// Device buffers of one HPD refinement call when the caller provides them
// (allocation-free entry point): W1, W2 hold n x n x batch values of the
// factor precision, best n x n x batch doubles, part the per-tile partial
// sums (max of the residual tiles and the validation blocks, times batch,
// plus 64), rn batch doubles, flags batch ints.  nullptr everywhere else:
// the factor's own cached buffers are used.
struct RefineWs {
  void* w1 = nullptr;
  void* w2 = nullptr;
  double* best = nullptr;
  double* part = nullptr;
  double* rn = nullptr;
  int* flags = nullptr;
};

int analyse_input(Factor* f, const double* A, int64_t lda, int64_t sA, bool check_sym,
                  hipStream_t st, const RefineWs* ws = nullptr);
// Finiteness (bit0) and exact symmetry failures (bit1) of a batch of n x n
// matrices with the factor's n and batch; the factor's scales are untouched.
int validate_flags(Factor* f, const double* M, int64_t ld, int64_t sM, hipStream_t st,
                   const RefineWs* ws = nullptr);

// Factorisation of the scaled input into f (Q, S, structure, prec).
msqrt_status build_factor(Factor* f, const msqrt_options& o, const double* A, int64_t lda,
                          int64_t sA, hipStream_t st, PhaseTimer* tm);
// General path (complex Schur, Alg. 2); A is real (cplx = 0) or interleaved
// complex, ld in elements.
int analyse_input_general(Factor* f, const double* A, int64_t lda, int cplx, hipStream_t st);
template <typename T>
msqrt_status factor_general(Factor* f, const double* A, int64_t lda, int cplx, hipStream_t st,
                            PhaseTimer* tm);
// Cube root (Sec. 4, p = 3) on the general path: complex Schur form of the
// scaled input, U = T^{1/3}, and the refinement with residual A - X^3.
template <typename T>
msqrt_status factor_root3(Factor* f, const double* A, int64_t lda, int cplx, hipStream_t st,
                          PhaseTimer* tm);
template <typename T>
msqrt_status refine_root3(Factor* f, const double* A, int64_t lda, double* X, int64_t ldx,
                          int init, int maxit, double tol, hipStream_t st, msqrt_info* info,
                          PhaseTimer& tm);
template <typename T>
msqrt_status refine_general(Factor* f, const double* A, int64_t lda, double* X, int64_t ldx,
                            int init, int maxit, double tol, hipStream_t st, msqrt_info* info,
                            PhaseTimer& tm);
// Real route of the general path (real Schur form, quasi-triangular root and
// Sylvester solves).
template <typename T>
msqrt_status factor_real(Factor* f, const double* A, int64_t lda, hipStream_t st, PhaseTimer* tm);
template <typename T>
msqrt_status refine_real(Factor* f, const double* A, int64_t lda, double* X, int64_t ldx, int init,
                         int maxit, double tol, hipStream_t st, msqrt_info* info, PhaseTimer& tm);
template <typename T>
msqrt_status backward_real(Factor* f, const double* X, int64_t ldx, const double* Gbar,
                           int64_t ldgb, double* G, int64_t ldg, int maxit, double tol,
                           hipStream_t st, msqrt_info* info, PhaseTimer& tm);
template <typename T>
msqrt_status backward_general(Factor* f, const double* X, int64_t ldx, const double* Gbar,
                              int64_t ldgb, double* G, int64_t ldg, int maxit, double tol,
                              hipStream_t st, msqrt_info* info, PhaseTimer& tm);

// Precision choice for MSQRT_PREC_AUTO.
msqrt_prec select_precision(const msqrt_options& o, msqrt_dtype dtype, int64_t n, const void* A,
                            int64_t lda, int64_t sA, hipStream_t st, msqrt_info* info,
                            PhaseTimer& tm);
// Adjoint solve for msqrt_sqrtm_backward.
msqrt_status backward(Factor* f, const double* X, int64_t ldx, const double* Gbar, int64_t ldgb,
                      double* G, int64_t ldg, int64_t stride, int maxit, double tol,
                      hipStream_t st, msqrt_info* info, PhaseTimer& tm);

}  // namespace msqrt
