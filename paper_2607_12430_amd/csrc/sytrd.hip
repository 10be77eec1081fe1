// Householder tridiagonalisation of a symmetric matrix (first step of the
// spectral decomposition used by Alg. 3), blocked by panels of nb columns.
//
// Panel: one cooperative launch of G = TR x TR workgroups that walks the
// panel's columns with ONE grid barrier per column.  For column j with
// updated sub-column u (rows j+1..n-1) the reflector is v = (u - beta e1) c,
// c = 1/(alpha - beta).  Because every quantity the panel needs from v is
// linear in v, each workgroup forms its tile of the trailing product with the
// *unnormalised* u (A22 u), plus partial sums of ||u||^2, u^T A22 u,
// u^T A22 e1, V^T u and W^T u, before the barrier.  After the barrier every
// workgroup finishes the reflector scalars, y = A22 v - V (W^T v) - W (V^T v)
// and w = tau y - (tau/2)(tau y^T v) v for the rows it needs, and prepares
// the next column's u -- so the classic two reductions per column (norm,
// then product) cost a single synchronisation.
//
// The trailing matrix is kept as a full symmetric square (both triangles), so
// each workgroup reads its tile row-wise with coalesced loads and no
// cross-tile reduction of the product is needed beyond the TR partial vectors.
// After the panel: A22 -= [V W] [W V]^T on the MFMA GEMM (symmetric output).
#include "gemm.hpp"
#include "kernels.hpp"
#include "tridiag.hpp"

namespace msqrt {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxTs = 1024;  // max tile size handled by one workgroup
constexpr int kNbMax = 32;

// Two-level grid barrier: 16 workgroups per group counter, then one top
// counter; the last arrival bumps the generation word.  Counters are reset by
// their last arrival, so consecutive barriers (and launches) reuse them.
// A spin limit keeps a broken launch from hanging: it raises bar[1].
__device__ inline void grid_barrier(unsigned* bar, int G) {
  __syncthreads();
  if (threadIdx.x == 0) {
    constexpr int GS = 16;
    const int ng = (G + GS - 1) / GS;
    const int g = blockIdx.x / GS;
    const int gsz = min(GS, G - g * GS);
    const unsigned gen = __hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    unsigned* gc = &bar[32 * (1 + g)];
    unsigned* tc = &bar[32 * (1 + ng)];
    const unsigned a = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool released = false;
    if (a == (unsigned)gsz - 1) {
      __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      const unsigned b = __hip_atomic_fetch_add(tc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (b == (unsigned)ng - 1) {
        __hip_atomic_store(tc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        __hip_atomic_store(&bar[0], gen + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        released = true;
      }
    }
    if (!released) {
      unsigned spins = 0;
      while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        // A timed-out barrier is sticky: later barriers stop waiting at once.
        if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
        if (++spins > (1u << 24)) {
          __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
}

template <typename T>
struct PanelArgs {
  int n, p, nb;  // matrix size, first column of the panel, panel width
  int TR;        // tiles per dimension; G = TR * TR workgroups
  int r0, ts;    // tile grid origin (p + 1) and tile size
  T* A;          // n x n, ld n, full symmetric storage
  T* VW;         // n x 2nb: [V W]
  T* WV;         // n x 2nb: [W V]
  T* d;
  T* e;
  T* tau;
  T* ypart;      // [2][TR][n]
  double* sp;    // [2][G][4]
  double* vp;    // [2][TR][2 kNbMax]
  unsigned* bar;
};

template <typename T>
__global__ __launch_bounds__(kThreads) void sytrd_panel_kernel(PanelArgs<T> a) {
  const int n = a.n, nb = a.nb, TR = a.TR, G = TR * TR;
  const int blk = blockIdx.x, bi = blk % TR, bj = blk / TR;
  const int I0 = a.r0 + bi * a.ts, I1 = min(n, I0 + a.ts);
  const int K0 = a.r0 + bj * a.ts, K1 = min(n, K0 + a.ts);
  const int tid = threadIdx.x;
  const int64_t ld = n;
  const int p = a.p;
  T* A = a.A;

  __shared__ T uI[kMaxTs], uK[kMaxTs];
  __shared__ T vI[kMaxTs], wI[kMaxTs], vK[kMaxTs], wK[kMaxTs];  // newest column's v, w
  // Pivot rows r = p+1+q (q < nb) of V and W for all panel columns, and their
  // u for the current column: every workgroup keeps its own copy, so no value
  // written by another workgroup in the current phase is ever read.
  __shared__ T PV[kNbMax][kNbMax + 1], PW[kNbMax][kNbMax + 1], PU[kNbMax];
  __shared__ T VTv[kNbMax], WTv[kNbMax];
  __shared__ double red[kThreads / kWave];
  __shared__ double sc[8];

  // ---- prologue: u for the first column of the panel
  {
    const int j = p;
    for (int r = tid; r < I1 - I0; r += kThreads) uI[r] = (I0 + r >= j + 1) ? A[I0 + r + (int64_t)j * ld] : T(0);
    for (int r = tid; r < K1 - K0; r += kThreads) uK[r] = (K0 + r >= j + 1) ? A[K0 + r + (int64_t)j * ld] : T(0);
    for (int q = tid; q < nb; q += kThreads) PU[q] = (p + 1 + q < n) ? A[p + 1 + q + (int64_t)j * ld] : T(0);
  }
  __syncthreads();

  for (int jj = 0; jj < nb; ++jj) {
    const int j = p + jj;
    const int buf = jj & 1;
    // ---- tile product z_I = A(I, K) u_K and partial u_I^T z_I
    double s_uAu = 0.0;
    {
      const int kb = max(K0, j + 1);
      for (int r = tid; r < I1 - I0; r += kThreads) {
        const int i = I0 + r;
        T z = T(0);
        if (i >= j + 1) {
          const T* col = A + i;
#pragma unroll 8
          for (int k = kb; k < K1; ++k) z += col[(int64_t)k * ld] * uK[k - K0];
        }
        a.ypart[((int64_t)buf * TR + bj) * n + i] = z;
        s_uAu += (double)uI[r] * (double)z;
      }
    }
    s_uAu = block_sum(s_uAu, red);
    // ---- row-owner partials (bj == 0): ||u(2:)||^2, u^T a1, V^T u, W^T u
    double s_sig = 0.0, s_ua1 = 0.0;
    if (bj == 0) {
      for (int r = tid; r < I1 - I0; r += kThreads) {
        const int i = I0 + r;
        const double u = (double)uI[r];
        if (i >= j + 2) s_sig += u * u;
        if (i >= j + 1) s_ua1 += u * (double)A[i + (int64_t)(j + 1) * ld];
      }
      // 2 jj dot products over the rows of I: wave w takes columns w, w+4, ...
      const int wave = tid / kWave, lane = tid % kWave;
      for (int c = wave; c < 2 * jj; c += kThreads / kWave) {
        const int col = c < jj ? c : nb + (c - jj);
        double s = 0.0;
        for (int r = lane; r < I1 - I0; r += kWave) s += (double)a.VW[I0 + r + (int64_t)col * ld] * (double)uI[r];
        s = wave_sum(s);
        if (lane == 0) a.vp[((int64_t)buf * TR + bi) * (2 * kNbMax) + c] = s;
      }
    }
    s_sig = block_sum(s_sig, red);
    s_ua1 = block_sum(s_ua1, red);
    if (tid == 0) {
      double* spb = a.sp + ((int64_t)buf * G + blk) * 4;
      spb[0] = s_uAu;
      spb[1] = s_sig;
      spb[2] = s_ua1;
      // alpha = u_{j+1} (pivot row q = jj) and d_j = updated A(j, j), read
      // before the barrier: owners overwrite column j right after it.
      double dj = (double)A[j + (int64_t)j * ld];
      if (jj > 0)
        for (int t = 0; t < jj; ++t) dj -= 2.0 * (double)PV[jj - 1][t] * (double)PW[jj - 1][t];
      sc[0] = dj;
      sc[3] = (double)PU[jj];
    }

    grid_barrier(a.bar, G);

    // ---- reflector scalars (every workgroup, redundantly)
    if (tid == 0) {
      double uAu = 0.0, sig = 0.0, ua1 = 0.0;
      for (int b = 0; b < G; ++b) uAu += a.sp[((int64_t)buf * G + b) * 4 + 0];
      for (int b = 0; b < TR; ++b) {
        sig += a.sp[((int64_t)buf * G + b) * 4 + 1];
        ua1 += a.sp[((int64_t)buf * G + b) * 4 + 2];
      }
      const double alpha = sc[3];
      double beta, tau, c;
      if (sig == 0.0) {
        beta = alpha; tau = 0.0; c = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + sig), alpha);
        tau = (beta - alpha) / beta;
        c = 1.0 / (alpha - beta);
      }
      if (blk == 0) {
        a.d[j] = (T)sc[0];
        a.e[j] = (T)beta;
        a.tau[j] = (T)tau;
      }
      sc[0] = uAu; sc[1] = sig; sc[2] = ua1;
      sc[4] = beta; sc[5] = tau; sc[6] = c;
    }
    __syncthreads();
    const double beta = sc[4], tau = sc[5], c = sc[6];
    // V^T v and W^T v (length jj); V(j+1, :), W(j+1, :) are pivot row jj.
    for (int t = tid; t < jj; t += kThreads) {
      double vtu = 0.0, wtu = 0.0;
      for (int b = 0; b < TR; ++b) {
        vtu += a.vp[((int64_t)buf * TR + b) * (2 * kNbMax) + t];
        wtu += a.vp[((int64_t)buf * TR + b) * (2 * kNbMax) + jj + t];
      }
      VTv[t] = (T)(c * (vtu - beta * (double)PV[jj][t]));
      WTv[t] = (T)(c * (wtu - beta * (double)PW[jj][t]));
    }
    __syncthreads();
    if (tid == 0) {
      const double a11 = (double)A[j + 1 + (int64_t)(j + 1) * ld];
      const double vAv = c * c * (sc[0] - 2.0 * beta * sc[2] + beta * beta * a11);
      double vw = 0.0;
      for (int t = 0; t < jj; ++t) vw += (double)VTv[t] * (double)WTv[t];
      sc[7] = tau * (vAv - 2.0 * vw);  // w0^T v
    }
    __syncthreads();
    const double wv = sc[7];
    const bool zero_refl = (sc[1] == 0.0);

    // y_i, v_i, w_i of the current column for a row i >= j+1 (u_i given).
    auto finish_row = [&](int i, T ui, T& vi, T& wi) {
      if (zero_refl) {
        vi = (i == j + 1) ? T(1) : T(0);
        wi = T(0);
        return;
      }
      double yz = 0.0;
      for (int b = 0; b < TR; ++b) yz += (double)a.ypart[((int64_t)buf * TR + b) * n + i];
      double y = c * (yz - beta * (double)A[i + (int64_t)(j + 1) * ld]);
      for (int t = 0; t < jj; ++t)
        y -= (double)a.VW[i + (int64_t)t * ld] * (double)WTv[t] +
             (double)a.VW[i + (int64_t)(nb + t) * ld] * (double)VTv[t];
      const double v = (i == j + 1) ? 1.0 : c * (double)ui;
      vi = (T)v;
      wi = (T)(tau * y - 0.5 * tau * wv * v);
    };

    // Pivot rows (every workgroup): rows p+1+q >= j+1, i.e. q >= jj.
    for (int q = jj + tid; q < nb; q += kThreads) {
      const int r = p + 1 + q;
      T vi = T(0), wi = T(0);
      if (r < n) finish_row(r, PU[q], vi, wi);
      PV[q][jj] = vi;
      PW[q][jj] = wi;
    }
    // Rows of I and K; owners (bj == 0) publish V, W and the explicit
    // reflector column A(:, j).
    for (int r = tid; r < I1 - I0; r += kThreads) {
      const int i = I0 + r;
      T vi = T(0), wi = T(0);
      if (i >= j + 1) finish_row(i, uI[r], vi, wi);
      vI[r] = vi;
      wI[r] = wi;
      if (bj == 0) {
        a.VW[i + (int64_t)jj * ld] = vi;
        a.VW[i + (int64_t)(nb + jj) * ld] = wi;
        a.WV[i + (int64_t)jj * ld] = wi;
        a.WV[i + (int64_t)(nb + jj) * ld] = vi;
        A[i + (int64_t)j * ld] = vi;
      }
    }
    for (int r = tid; r < K1 - K0; r += kThreads) {
      const int i = K0 + r;
      T vi = T(0), wi = T(0);
      if (i >= j + 1) finish_row(i, uK[r], vi, wi);
      vK[r] = vi;
      wK[r] = wi;
    }
    __syncthreads();
    if (jj + 1 == nb) break;
    // ---- next column jn = j+1: u_i = A(i, jn) - sum_{t <= jj} V(i,t) W(jn,t) + W(i,t) V(jn,t)
    // with row jn's coefficients = pivot row jj.
    const int jn = j + 1;
    auto upd = [&](int i, T vnew, T wnew) -> T {
      T u = A[i + (int64_t)jn * ld];
      for (int t = 0; t < jj; ++t)
        u -= a.VW[i + (int64_t)t * ld] * PW[jj][t] + a.VW[i + (int64_t)(nb + t) * ld] * PV[jj][t];
      return u - (vnew * PW[jj][jj] + wnew * PV[jj][jj]);
    };
    for (int r = tid; r < I1 - I0; r += kThreads) {
      const int i = I0 + r;
      uI[r] = (i >= jn + 1) ? upd(i, vI[r], wI[r]) : T(0);
    }
    for (int r = tid; r < K1 - K0; r += kThreads) {
      const int i = K0 + r;
      uK[r] = (i >= jn + 1) ? upd(i, vK[r], wK[r]) : T(0);
    }
    for (int q = jj + 1 + tid; q < nb; q += kThreads) {
      const int r = p + 1 + q;
      if (r >= n) { PU[q] = T(0); continue; }
      T u = A[r + (int64_t)jn * ld];
      for (int t = 0; t <= jj; ++t) u -= PV[q][t] * PW[jj][t] + PW[q][t] * PV[jj][t];
      PU[q] = u;
    }
    __syncthreads();
  }
}

// Last diagonal entry after the final trailing update.
template <typename T>
__global__ void copy_last_diag(const T* A, int n, T* d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) d[n - 1] = A[(n - 1) + (int64_t)(n - 1) * n];
}

}  // namespace

template <typename T>
void sytrd(hipStream_t st, int n, T* A, T* d, T* e, T* tau, SytrdWork& w) {
  if (n <= 0) return;
  if (n == 1) {
    hipLaunchKernelGGL(copy_last_diag<T>, 1, 64, 0, st, (const T*)A, n, d);
    MSQRT_LAUNCH_CHECK();
    return;
  }
  const int nb = kNbMax;
  T* VW = w.VW.ensure<T>((int64_t)n * 2 * nb);
  T* WV = w.WV.ensure<T>((int64_t)n * 2 * nb);
  T* ypart = w.ypart.ensure<T>((int64_t)2 * 16 * n);
  double* sp = w.sp.ensure<double>((int64_t)2 * 256 * 4);
  double* vp = w.vp.ensure<double>((int64_t)2 * 16 * 2 * kNbMax);
  unsigned* bar = w.bar.ensure<unsigned>(32 * 40);
  MSQRT_HIP(hipMemsetAsync(bar, 0, sizeof(unsigned) * 32 * 40, st));
  for (int p = 0; p < n - 1; p += nb) {
    const int nbe = std::min(nb, n - 1 - p);
    const int m = n - 1 - p;  // rows/cols of the tile region [p+1, n)
    const int TR = (int)std::min<int64_t>(16, std::max<int64_t>(1, ceil_div(m, 128)));
    const int ts = (int)ceil_div(m, TR);
    if (ts > kMaxTs) throw Error{MSQRT_ERR_UNSUPPORTED, "tridiagonal reduction supports n <= 16385"};
    MSQRT_HIP(hipMemsetAsync(VW, 0, sizeof(T) * n * 2 * nb, st));
    MSQRT_HIP(hipMemsetAsync(WV, 0, sizeof(T) * n * 2 * nb, st));
    PanelArgs<T> pa{n, p, nbe, TR, p + 1, ts, A, VW, WV, d, e, tau, ypart, sp, vp, bar};
    void* args[] = {&pa};
    MSQRT_HIP(hipLaunchCooperativeKernel((const void*)sytrd_panel_kernel<T>, dim3(TR * TR),
                                         dim3(kThreads), args, 0, st));
    // Trailing update A(q:n, q:n) -= [V W] [W V]^T, q = p + nbe.
    const int q = p + nbe;
    if (q < n) {
      const int mt = n - q;
      if (std::is_same<T, float>::value)
        gemm_store_f32(st, false, true, mt, mt, 2 * nb, (const float*)(VW + q), n, 0,
                       (const float*)(WV + q), n, 0, (float*)(A + q + (int64_t)q * n), n, 0, -1.f,
                       1.f, 1, true);
      else
        gemm_store_f64(st, false, true, mt, mt, 2 * nb, (const double*)(VW + q), n, 0,
                       (const double*)(WV + q), n, 0, (double*)(A + q + (int64_t)q * n), n, 0,
                       -1.0, 1.0, 1, true);
    }
  }
  hipLaunchKernelGGL(copy_last_diag<T>, 1, 64, 0, st, (const T*)A, n, d);
  MSQRT_LAUNCH_CHECK();
}

template void sytrd<float>(hipStream_t, int, float*, float*, float*, float*, SytrdWork&);
template void sytrd<double>(hipStream_t, int, double*, double*, double*, double*, SytrdWork&);

}  // namespace msqrt
