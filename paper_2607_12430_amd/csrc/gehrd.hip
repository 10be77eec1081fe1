// Blocked Householder reduction to upper Hessenberg form, complex, for the
// Schur factorisation of the general path (Alg. 2, first line: the Schur
// decomposition starts from a Hessenberg reduction).
//
// Panels of kNb columns.  Inside a panel, column c = p + i is brought up to
// date lazily (the panel's earlier reflectors act through the accumulated
// Y = A V T and V, T), its reflector H_c = I - tau v v^* is generated, and the
// product y = A v (A = the matrix at the start of the panel) is formed by a
// split-K gemv over the trailing columns; Y's next column is
// tau (y - Y (V^* v)).  After the panel the trailing columns are updated with
// MFMA GEMMs:  A(:, q:) -= Y V(q:, :)^*,  A(p+1:, q:) -= V T^* (V^* A(p+1:, q:)).
// Q1 = H_0 H_1 ... is then formed by applying the block reflectors to the
// identity, last block first.
#include <algorithm>

#include "kernels.hpp"
#include "schur.hpp"

namespace msqrt {

namespace {

constexpr int kNb = 32;
constexpr int kColThreads = 1024;
constexpr int kGemvRows = 256;
constexpr int kGemvCols = 64;

// Stacked-layout element access: real at p[i + j*ld], imaginary ld/2 below.
template <typename T>
__device__ inline cx<T> ld_s(const T* p, int64_t ld, int64_t i, int64_t j) {
  const T* q = p + i + j * ld;
  return {q[0], q[ld / 2]};
}
template <typename T>
__device__ inline void st_s(T* p, int64_t ld, int64_t i, int64_t j, cx<T> v) {
  T* q = p + i + j * ld;
  q[0] = v.r;
  q[ld / 2] = v.i;
}

template <typename T>
struct ColArgs {
  int n, p, i, nbp;
  T* H;            // stacked, ld 2n
  T* V;            // panel reflectors (stacked, ld 2n), column k = reflector p + k
  T* Tp;           // panel T (stacked, ld 2 kNb)
  T* Y;            // panel Y (stacked, ld 2n)
  const T* part;   // gemv partials of the previous column: chunk c at part + c * 2n
  int nchunks;
};

// Dot products d_k = sum_{r >= r0} conj(V(r, k)) x(r), k < cnt, x in the
// stacked column xcol (ld 2n).  Wave w handles k = w, w + 16, ...
template <typename T>
__device__ void panel_dots(const ColArgs<T>& a, int cnt, int r0, const T* x, cx<T>* out) {
  const int n = a.n;
  const int64_t ld = 2 * (int64_t)n;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (int k = wave; k < cnt; k += kColThreads / kWave) {
    T sr = 0, si = 0;
    const T* vk = a.V + (int64_t)k * ld;
    for (int r = r0 + lane; r < n; r += kWave) {
      const cx<T> v = {vk[r], vk[r + n]};
      const cx<T> xv = {x[r], x[r + n]};
      const cx<T> pr = cmulc(v, xv);
      sr += pr.r;
      si += pr.i;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) out[k] = {sr, si};
  }
}

template <typename T>
__global__ __launch_bounds__(kColThreads) void gehrd_col_kernel(ColArgs<T> a) {
  const int n = a.n, p = a.p, i = a.i;
  const int64_t ld = 2 * (int64_t)n, ldt = 2 * kNb;
  const int t = threadIdx.x;
  __shared__ cx<T> u[kNb], z[kNb];
  __shared__ T red[kColThreads / kWave];

  if (i > 0) {
    // Finish Y(:, i-1) = tau (y - Y(:, :i-1) (V(:, :i-1)^* v_{i-1})) and
    // T(:i-1, i-1) = -tau T(:i-1, :i-1) (V^* v_{i-1}).
    const int k1 = i - 1;
    const T* vk = a.V + (int64_t)k1 * ld;
    panel_dots(a, k1, p + 1, vk, u);
    __syncthreads();
    const cx<T> tau = ld_s(a.Tp, ldt, k1, k1);
    if (t < k1) {
      cx<T> s = {0, 0};
      for (int c = t; c < k1; ++c) s = cadd(s, cmul(ld_s(a.Tp, ldt, t, c), u[c]));
      z[t] = s;
    }
    __syncthreads();
    if (t < k1) st_s(a.Tp, ldt, t, k1, cscale(cmul(tau, z[t]), T(-1)));
    T* yk = a.Y + (int64_t)k1 * ld;
    for (int r = t; r < n; r += kColThreads) {
      cx<T> y = {0, 0};
      for (int c = 0; c < a.nchunks; ++c) {
        const T* pc = a.part + (int64_t)c * ld;
        y = cadd(y, cx<T>{pc[r], pc[r + n]});
      }
      for (int c = 0; c < k1; ++c) y = csub(y, cmul(ld_s(a.Y, ld, r, c), u[c]));
      const cx<T> v = cmul(tau, y);
      yk[r] = v.r;
      yk[r + n] = v.i;
    }
    __syncthreads();
  }
  if (i >= a.nbp) return;
  const int c = p + i;
  T* hc = a.H + (int64_t)c * ld;
  // w = A(:, c) - Y(:, :i) V(c, :i)^*
  for (int r = t; r < n; r += kColThreads) {
    cx<T> w = {hc[r], hc[r + n]};
    for (int k = 0; k < i; ++k) w = csub(w, cmul(ld_s(a.Y, ld, r, k), cconj(ld_s(a.V, ld, c, k))));
    hc[r] = w.r;
    hc[r + n] = w.i;
  }
  __syncthreads();
  // w <- w - V T^* (V^* w)   (rows > p)
  if (i > 0) {
    panel_dots(a, i, p + 1, hc, u);
    __syncthreads();
    if (t < i) {
      // (T^* u)_t = sum_{j <= t} conj(T(j, t)) u_j
      cx<T> s = {0, 0};
      for (int j = 0; j <= t; ++j) s = cadd(s, cmulc(ld_s(a.Tp, ldt, j, t), u[j]));
      z[t] = s;
    }
    __syncthreads();
    for (int r = p + 1 + t; r < n; r += kColThreads) {
      cx<T> w = {hc[r], hc[r + n]};
      for (int k = 0; k < i; ++k) w = csub(w, cmul(ld_s(a.V, ld, r, k), z[k]));
      hc[r] = w.r;
      hc[r + n] = w.i;
    }
    __syncthreads();
  }
  // Reflector from w(c+1 : n)
  T s2 = 0;
  for (int r = c + 2 + t; r < n; r += kColThreads) s2 += hc[r] * hc[r] + hc[r + n] * hc[r + n];
  s2 = block_sum(s2, red);
  const cx<T> alpha = {hc[c + 1], hc[c + 1 + n]};
  cx<T> tau = {0, 0}, scal = {0, 0};
  T beta = alpha.r;
  const bool trivial = (s2 == T(0) && alpha.i == T(0));
  if (!trivial) {
    beta = -copysign(sqrt(alpha.r * alpha.r + alpha.i * alpha.i + s2), alpha.r);
    tau = {(beta - alpha.r) / beta, -alpha.i / beta};
    scal = cdiv(cx<T>{T(1), T(0)}, csub(alpha, cx<T>{beta, T(0)}));
  }
  T* vi = a.V + (int64_t)i * ld;
  for (int r = t; r < n; r += kColThreads) {
    cx<T> v = {0, 0};
    if (r == c + 1) v = {T(1), T(0)};
    else if (r > c + 1) v = trivial ? cx<T>{0, 0} : cmul(cx<T>{hc[r], hc[r + n]}, scal);
    vi[r] = v.r;
    vi[r + n] = v.i;
  }
  __syncthreads();
  for (int r = c + 1 + t; r < n; r += kColThreads) {
    if (r == c + 1) {
      hc[r] = trivial ? alpha.r : beta;
      hc[r + n] = trivial ? alpha.i : T(0);
    } else {
      hc[r] = T(0);
      hc[r + n] = T(0);
    }
  }
  if (t == 0) st_s(a.Tp, ldt, i, i, tau);
}

// y partials: part[chunk] = H(:, c0 + chunk*kGemvCols ...) v(...)
template <typename T>
__global__ __launch_bounds__(kGemvRows) void gehrd_gemv_kernel(int n, int c0, const T* H,
                                                              const T* v, T* part) {
  const int64_t ld = 2 * (int64_t)n;
  const int r = blockIdx.x * kGemvRows + threadIdx.x;
  const int j0 = c0 + blockIdx.y * kGemvCols;
  const int j1 = min(n, j0 + kGemvCols);
  __shared__ T vr[kGemvCols], vim[kGemvCols];
  if (threadIdx.x < j1 - j0) {
    vr[threadIdx.x] = v[j0 + threadIdx.x];
    vim[threadIdx.x] = v[j0 + threadIdx.x + n];
  }
  __syncthreads();
  if (r >= n) return;
  T sr = 0, si = 0;
  for (int j = j0; j < j1; ++j) {
    const T hr = H[r + j * ld], hi = H[r + n + j * ld];
    const T a = vr[j - j0], b = vim[j - j0];
    sr += hr * a - hi * b;
    si += hr * b + hi * a;
  }
  T* pc = part + (int64_t)blockIdx.y * ld;
  pc[r] = sr;
  pc[r + n] = si;
}

template <typename T>
__global__ void cset_identity_kernel(int n, T* re, T* im, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  re[i + j * ld] = i == j ? T(1) : T(0);
  if (im) im[i + j * ld] = T(0);
}

// ---- real data (the real Schur route): the same blocked reduction with
// real reflectors H_c = I - tau v v^T, matrices n x n with ld n.

template <typename T>
struct RColArgs {
  int n, p, i, nbp;
  T* H;            // ld n
  T* V;            // panel reflectors (ld n), column k = reflector p + k
  T* Tp;           // panel T (ld kNb)
  T* Y;            // panel Y (ld n)
  const T* part;   // gemv partials of the previous column: chunk c at part + c * n
  int nchunks;
};

// d_k = sum_{r >= r0} V(r, k) x(r), k < cnt; wave w handles k = w, w + 16, ...
template <typename T>
__device__ void rpanel_dots(const RColArgs<T>& a, int cnt, int r0, const T* x, T* out) {
  const int n = a.n;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (int k = wave; k < cnt; k += kColThreads / kWave) {
    T s = 0;
    const T* vk = a.V + (int64_t)k * n;
    for (int r = r0 + lane; r < n; r += kWave) s += vk[r] * x[r];
    s = wave_sum(s);
    if (lane == 0) out[k] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(kColThreads) void rgehrd_col_kernel(RColArgs<T> a) {
  const int n = a.n, p = a.p, i = a.i;
  const int64_t ld = n;
  const int t = threadIdx.x;
  __shared__ T u[kNb], z[kNb];
  __shared__ T red[kColThreads / kWave];
  if (i > 0) {
    // Y(:, i-1) = tau (y - Y(:, :i-1) (V(:, :i-1)^T v_{i-1})),
    // T(:i-1, i-1) = -tau T(:i-1, :i-1) (V^T v_{i-1})
    const int k1 = i - 1;
    const T* vk = a.V + (int64_t)k1 * ld;
    rpanel_dots(a, k1, p + 1, vk, u);
    __syncthreads();
    const T tau = a.Tp[k1 + k1 * kNb];
    if (t < k1) {
      T s = 0;
      for (int c = t; c < k1; ++c) s += a.Tp[t + c * kNb] * u[c];
      z[t] = s;
    }
    __syncthreads();
    if (t < k1) a.Tp[t + k1 * kNb] = -tau * z[t];
    T* yk = a.Y + (int64_t)k1 * ld;
    for (int r = t; r < n; r += kColThreads) {
      T y = 0;
      for (int c = 0; c < a.nchunks; ++c) y += a.part[(int64_t)c * ld + r];
      for (int c = 0; c < k1; ++c) y -= a.Y[r + (int64_t)c * ld] * u[c];
      yk[r] = tau * y;
    }
    __syncthreads();
  }
  if (i >= a.nbp) return;
  const int c = p + i;
  T* hc = a.H + (int64_t)c * ld;
  // w = A(:, c) - Y(:, :i) V(c, :i)^T
  for (int r = t; r < n; r += kColThreads) {
    T w = hc[r];
    for (int k = 0; k < i; ++k) w -= a.Y[r + (int64_t)k * ld] * a.V[c + (int64_t)k * ld];
    hc[r] = w;
  }
  __syncthreads();
  // w <- w - V T^T (V^T w)   (rows > p)
  if (i > 0) {
    rpanel_dots(a, i, p + 1, hc, u);
    __syncthreads();
    if (t < i) {
      T s = 0;
      for (int j = 0; j <= t; ++j) s += a.Tp[j + t * kNb] * u[j];
      z[t] = s;
    }
    __syncthreads();
    for (int r = p + 1 + t; r < n; r += kColThreads) {
      T w = hc[r];
      for (int k = 0; k < i; ++k) w -= a.V[r + (int64_t)k * ld] * z[k];
      hc[r] = w;
    }
    __syncthreads();
  }
  // reflector from w(c+1 : n)
  T s2 = 0;
  for (int r = c + 2 + t; r < n; r += kColThreads) s2 += hc[r] * hc[r];
  s2 = block_sum(s2, red);
  const T alpha = hc[c + 1];
  T tau = 0, scal = 0, beta = alpha;
  const bool trivial = s2 == T(0);
  if (!trivial) {
    beta = -copysign(sqrt(alpha * alpha + s2), alpha);
    tau = (beta - alpha) / beta;
    scal = T(1) / (alpha - beta);
  }
  T* vi = a.V + (int64_t)i * ld;
  for (int r = t; r < n; r += kColThreads) {
    T v = 0;
    if (r == c + 1) v = T(1);
    else if (r > c + 1) v = trivial ? T(0) : hc[r] * scal;
    vi[r] = v;
  }
  __syncthreads();
  for (int r = c + 1 + t; r < n; r += kColThreads) hc[r] = r == c + 1 ? beta : T(0);
  if (t == 0) a.Tp[i + i * kNb] = tau;
}

// y partials: part[chunk] = H(:, c0 + chunk*kGemvCols ...) v(...)
template <typename T>
__global__ __launch_bounds__(kGemvRows) void rgehrd_gemv_kernel(int n, int c0, const T* H,
                                                               const T* v, T* part) {
  const int r = blockIdx.x * kGemvRows + threadIdx.x;
  const int j0 = c0 + blockIdx.y * kGemvCols;
  const int j1 = min(n, j0 + kGemvCols);
  __shared__ T vs[kGemvCols];
  if (threadIdx.x < j1 - j0) vs[threadIdx.x] = v[j0 + threadIdx.x];
  __syncthreads();
  if (r >= n) return;
  T s = 0;
  for (int j = j0; j < j1; ++j) s += H[r + (int64_t)j * n] * vs[j - j0];
  part[(int64_t)blockIdx.y * n + r] = s;
}

}  // namespace

template <typename T>
void launch_cset_identity(hipStream_t st, int n, CMat<T> A) {
  if (n <= 0) return;
  const int64_t cnt = (int64_t)n * n;
  hipLaunchKernelGGL(cset_identity_kernel<T>, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st,
                     n, A.re, A.im, A.ld);
  MSQRT_LAUNCH_CHECK();
}
template void launch_cset_identity<float>(hipStream_t, int, CMat<float>);
template void launch_cset_identity<double>(hipStream_t, int, CMat<double>);

template <typename T>
void gehrd(hipStream_t st, int n, T* H, T* Z, GehrdWork& w) {
  const int64_t ld = 2 * (int64_t)n;
  const CMat<T> Hm = stacked(H, n, ld), Zm = stacked(Z, n, ld);
  launch_cset_identity<T>(st, n, Zm);
  const int nref = n - 2;  // reflectors for columns 0 .. n-3
  if (nref <= 0) return;
  const int npan = (int)ceil_div(nref, kNb);
  T* Vall = w.V.ensure<T>(ld * nref);
  T* Tall = w.Tall.ensure<T>((int64_t)npan * 2 * kNb * kNb);
  // the panel factors are upper triangular: only the upper part is written
  MSQRT_HIP(hipMemsetAsync(Tall, 0, sizeof(T) * (size_t)npan * 2 * kNb * kNb, st));
  T* Y = w.Y.ensure<T>(ld * kNb);
  const int maxchunks = (int)ceil_div(n, kGemvCols);
  T* part = w.part.ensure<T>(ld * maxchunks);
  T* Wb = w.W.ensure<T>((int64_t)2 * kNb * n);
  T* W2 = w.W2.ensure<T>((int64_t)2 * kNb * n);
  const CMat<T> Ym = stacked(Y, n, ld);
  for (int pi = 0; pi < npan; ++pi) {
    const int p = pi * kNb;
    const int nbp = std::min(kNb, nref - p);
    T* V = Vall + (int64_t)p * ld;
    T* Tp = Tall + (int64_t)pi * 2 * kNb * kNb;
    int nchunks = 0;
    for (int i = 0; i <= nbp; ++i) {
      ColArgs<T> a{n, p, i, nbp, H, V, Tp, Y, part, nchunks};
      hipLaunchKernelGGL(gehrd_col_kernel<T>, dim3(1), dim3(kColThreads), 0, st, a);
      MSQRT_LAUNCH_CHECK();
      if (i == nbp) break;
      // y = A(:, c+1:) v_i  (v_i is zero above row c+1)
      const int c0 = p + i + 1;
      nchunks = (int)ceil_div(n - c0, kGemvCols);
      hipLaunchKernelGGL(gehrd_gemv_kernel<T>, dim3((unsigned)ceil_div(n, kGemvRows), nchunks),
                         dim3(kGemvRows), 0, st, n, c0, (const T*)H,
                         (const T*)(V + (int64_t)i * ld), part);
      MSQRT_LAUNCH_CHECK();
    }
    const int q = p + nbp;
    if (q >= n) continue;
    const CMat<T> Vm = stacked(V, n, ld);
    const CMat<T> Tm = stacked(Tp, kNb, 2 * kNb);
    // A(:, q:) -= Y V(q:, :)^*
    cgemm<T>(st, 'N', 'C', n, n - q, nbp, Ym, sub(Vm, q, 0), T(-1), T(1), sub(Hm, 0, q));
    // A(p+1:, q:) -= V T^* (V^* A(p+1:, q:))
    const CMat<T> Wm = stacked(Wb, kNb, 2 * kNb), W2m = stacked(W2, kNb, 2 * kNb);
    cgemm<T>(st, 'C', 'N', nbp, n - q, n - p - 1, sub(Vm, p + 1, 0), sub(Hm, p + 1, q), T(1), T(0),
             Wm);
    cgemm<T>(st, 'C', 'N', nbp, n - q, nbp, Tm, Wm, T(1), T(0), W2m);
    cgemm<T>(st, 'N', 'N', n - p - 1, n - q, nbp, sub(Vm, p + 1, 0), W2m, T(-1), T(1),
             sub(Hm, p + 1, q));
  }
  // Q1 = B_0 B_1 ... B_last applied to I, last block first:
  // Z(p+1:, p+1:) -= V T (V^* Z(p+1:, p+1:)).
  for (int pi = npan - 1; pi >= 0; --pi) {
    const int p = pi * kNb;
    const int nbp = std::min(kNb, nref - p);
    const CMat<T> Vm = stacked(Vall + (int64_t)p * ld, n, ld);
    const CMat<T> Tm = stacked(Tall + (int64_t)pi * 2 * kNb * kNb, kNb, 2 * kNb);
    const CMat<T> Wm = stacked(Wb, kNb, 2 * kNb), W2m = stacked(W2, kNb, 2 * kNb);
    const int m = n - p - 1;
    cgemm<T>(st, 'C', 'N', nbp, m, m, sub(Vm, p + 1, 0), sub(Zm, p + 1, p + 1), T(1), T(0), Wm);
    cgemm<T>(st, 'N', 'N', nbp, m, nbp, Tm, Wm, T(1), T(0), W2m);
    cgemm<T>(st, 'N', 'N', m, m, nbp, sub(Vm, p + 1, 0), W2m, T(-1), T(1), sub(Zm, p + 1, p + 1));
  }
}

template <typename T>
void gehrd_real(hipStream_t st, int n, T* H, T* Z, GehrdWork& w) {
  const int64_t ld = n;
  const CMat<T> Hm{H, nullptr, ld}, Zm{Z, nullptr, ld};
  launch_cset_identity<T>(st, n, Zm);
  const int nref = n - 2;
  if (nref <= 0) return;
  const int npan = (int)ceil_div(nref, kNb);
  T* Vall = w.V.ensure<T>(ld * nref);
  T* Tall = w.Tall.ensure<T>((int64_t)npan * kNb * kNb);
  MSQRT_HIP(hipMemsetAsync(Tall, 0, sizeof(T) * (size_t)npan * kNb * kNb, st));
  T* Y = w.Y.ensure<T>(ld * kNb);
  const int maxchunks = (int)ceil_div(n, kGemvCols);
  T* part = w.part.ensure<T>(ld * maxchunks);
  T* Wb = w.W.ensure<T>((int64_t)kNb * n);
  T* W2 = w.W2.ensure<T>((int64_t)kNb * n);
  const CMat<T> Ym{Y, nullptr, ld};
  for (int pi = 0; pi < npan; ++pi) {
    const int p = pi * kNb;
    const int nbp = std::min(kNb, nref - p);
    T* V = Vall + (int64_t)p * ld;
    T* Tp = Tall + (int64_t)pi * kNb * kNb;
    int nchunks = 0;
    for (int i = 0; i <= nbp; ++i) {
      RColArgs<T> a{n, p, i, nbp, H, V, Tp, Y, part, nchunks};
      hipLaunchKernelGGL(rgehrd_col_kernel<T>, dim3(1), dim3(kColThreads), 0, st, a);
      MSQRT_LAUNCH_CHECK();
      if (i == nbp) break;
      const int c0 = p + i + 1;
      nchunks = (int)ceil_div(n - c0, kGemvCols);
      hipLaunchKernelGGL(rgehrd_gemv_kernel<T>, dim3((unsigned)ceil_div(n, kGemvRows), nchunks),
                         dim3(kGemvRows), 0, st, n, c0, (const T*)H,
                         (const T*)(V + (int64_t)i * ld), part);
      MSQRT_LAUNCH_CHECK();
    }
    const int q = p + nbp;
    if (q >= n) continue;
    const CMat<T> Vm{V, nullptr, ld};
    const CMat<T> Tm{Tp, nullptr, kNb};
    // A(:, q:) -= Y V(q:, :)^T
    cgemm<T>(st, 'N', 'T', n, n - q, nbp, Ym, sub(Vm, q, 0), T(-1), T(1), sub(Hm, 0, q));
    // A(p+1:, q:) -= V T^T (V^T A(p+1:, q:))
    const CMat<T> Wm{Wb, nullptr, kNb}, W2m{W2, nullptr, kNb};
    cgemm<T>(st, 'T', 'N', nbp, n - q, n - p - 1, sub(Vm, p + 1, 0), sub(Hm, p + 1, q), T(1), T(0),
             Wm);
    cgemm<T>(st, 'T', 'N', nbp, n - q, nbp, Tm, Wm, T(1), T(0), W2m);
    cgemm<T>(st, 'N', 'N', n - p - 1, n - q, nbp, sub(Vm, p + 1, 0), W2m, T(-1), T(1),
             sub(Hm, p + 1, q));
  }
  // Q1 = B_0 B_1 ... applied to I, last block first
  for (int pi = npan - 1; pi >= 0; --pi) {
    const int p = pi * kNb;
    const int nbp = std::min(kNb, nref - p);
    const CMat<T> Vm{Vall + (int64_t)p * ld, nullptr, ld};
    const CMat<T> Tm{Tall + (int64_t)pi * kNb * kNb, nullptr, kNb};
    const CMat<T> Wm{Wb, nullptr, kNb}, W2m{W2, nullptr, kNb};
    const int m = n - p - 1;
    cgemm<T>(st, 'T', 'N', nbp, m, m, sub(Vm, p + 1, 0), sub(Zm, p + 1, p + 1), T(1), T(0), Wm);
    cgemm<T>(st, 'N', 'N', nbp, m, nbp, Tm, Wm, T(1), T(0), W2m);
    cgemm<T>(st, 'N', 'N', m, m, nbp, sub(Vm, p + 1, 0), W2m, T(-1), T(1), sub(Zm, p + 1, p + 1));
  }
}

template void gehrd_real<float>(hipStream_t, int, float*, float*, GehrdWork&);
template void gehrd_real<double>(hipStream_t, int, double*, double*, GehrdWork&);
template void gehrd<float>(hipStream_t, int, float*, float*, GehrdWork&);
template void gehrd<double>(hipStream_t, int, double*, double*, GehrdWork&);

}  // namespace msqrt
