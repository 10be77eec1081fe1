// Learned precision selector: matrix features, the 16-64-64-3 network
// (forward, gradient, Adam), on-device inference and the cost-model choice
// used by MSQRT_PREC_AUTO.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/msqrt_selector.h"
#include "factor.hpp"
#include "kernels.hpp"

namespace msqrt {

namespace {

constexpr int NF = MSQRT_SEL_NFEAT, HID = 64, NO = 3, NP = MSQRT_SEL_NPARAM;
constexpr int OFF_B1 = HID * NF, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + NO * HID;
static_assert(OFF_B3 + NO == NP, "parameter layout");
constexpr int kFT = 32;
constexpr int kGradSamples = 64;  // samples per gradient workgroup

__device__ inline void elem(const double* A, int64_t lda, int cplx, int64_t i, int64_t j,
                            double& re, double& im) {
  if (cplx) {
    re = A[2 * (i + j * lda)];
    im = A[2 * (i + j * lda) + 1];
  } else {
    re = A[i + j * lda];
    im = 0.0;
  }
}

// Per 32 x 32 tile (I, J): row partial sums of |a| and |a|^2 (into
// rowabs/rowsq[J * n + row]), column partials (colabs/colsq[I * n + col]),
// and sum |a_ij - a'_ji|^2, sum Re(a_ij a_ji), sum |a_ij|^2 (a' = a for real,
// conj(a) for complex) into tpart[3 * tile + k]; exact-symmetry flag.
__global__ __launch_bounds__(256) void feat_tiles_kernel(int n, const double* A, int64_t lda,
                                                         int cplx, int nt, double* rowabs,
                                                         double* rowsq, double* colabs,
                                                         double* colsq, double* tpart, int* flag) {
  __shared__ double ar[kFT][kFT + 1], ai[kFT][kFT + 1];  // tile (I, J): [col][row]
  __shared__ double pr[kFT][kFT + 1], pi[kFT][kFT + 1];  // tile (J, I): [col][row]
  __shared__ double red[4];
  const int I = blockIdx.x % nt, J = blockIdx.x / nt;
  const int t = threadIdx.x;
  for (int x = t; x < kFT * kFT; x += blockDim.x) {
    const int i = x % kFT, j = x / kFT;
    double re = 0, im = 0, qr = 0, qi = 0;
    const int64_t gi = kFT * I + i, gj = kFT * J + j;
    if (gi < n && gj < n) elem(A, lda, cplx, gi, gj, re, im);
    const int64_t hi = kFT * J + i, hj = kFT * I + j;  // partner tile (J, I)
    if (hi < n && hj < n) elem(A, lda, cplx, hi, hj, qr, qi);
    ar[j][i] = re;
    ai[j][i] = im;
    pr[j][i] = qr;
    pi[j][i] = qi;
  }
  __syncthreads();
  double asym = 0, tra2 = 0, fro = 0;
  int bad = 0;
  for (int x = t; x < kFT * kFT; x += blockDim.x) {
    const int i = x % kFT, j = x / kFT;
    if (kFT * I + i >= n || kFT * J + j >= n) continue;
    const double re = ar[j][i], im = ai[j][i];
    const double br = pr[i][j], bi = pi[i][j];  // a_ji
    const double tr = br, ti = cplx ? -bi : bi;  // partner as in A^T / A^H
    const double dr = re - tr, di = im - ti;
    if (dr != 0.0 || di != 0.0) bad = 1;
    asym += dr * dr + di * di;
    tra2 += re * br - im * bi;
    fro += re * re + im * im;
  }
  if (bad) atomicOr(flag, 1);
  if (t < kFT) {
    const int i = t;
    const int64_t gi = kFT * I + i;
    if (gi < n) {
      double sa = 0, sq = 0;
      for (int j = 0; j < kFT; ++j) {
        if (kFT * J + j >= n) break;
        const double m2 = ar[j][i] * ar[j][i] + ai[j][i] * ai[j][i];
        sa += sqrt(m2);
        sq += m2;
      }
      rowabs[(int64_t)J * n + gi] = sa;
      rowsq[(int64_t)J * n + gi] = sq;
    }
  } else if (t < 2 * kFT) {
    const int j = t - kFT;
    const int64_t gj = kFT * J + j;
    if (gj < n) {
      double sa = 0, sq = 0;
      for (int i = 0; i < kFT; ++i) {
        if (kFT * I + i >= n) break;
        const double m2 = ar[j][i] * ar[j][i] + ai[j][i] * ai[j][i];
        sa += sqrt(m2);
        sq += m2;
      }
      colabs[(int64_t)I * n + gj] = sa;
      colsq[(int64_t)I * n + gj] = sq;
    }
  }
  asym = block_sum(asym, red);
  tra2 = block_sum(tra2, red);
  fro = block_sum(fro, red);
  if (t == 0) {
    tpart[3 * blockIdx.x + 0] = asym;
    tpart[3 * blockIdx.x + 1] = tra2;
    tpart[3 * blockIdx.x + 2] = fro;
  }
}

__device__ inline double lg10(double x, double floor_) { return log10(fmax(x, floor_)); }

__global__ __launch_bounds__(1024) void feat_final_kernel(int n, const double* A, int64_t lda,
                                                          int cplx, int nt, const double* rowabs,
                                                          const double* rowsq,
                                                          const double* colabs,
                                                          const double* colsq, const double* tpart,
                                                          const int* flag, float* F) {
  __shared__ double red[16];
  double rn_max = 0, rn_min = INFINITY, cn_max = 0, cn_min = INFINITY, ninf = 0, none = 0;
  double gmin = INFINITY, dmax = 0, dmin = INFINITY, trr = 0, tri = 0, cnt_neg = 0, cnt_disc = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double ra = 0, rs = 0, ca = 0, cs = 0;
    for (int b = 0; b < nt; ++b) {
      ra += rowabs[(int64_t)b * n + i];
      rs += rowsq[(int64_t)b * n + i];
      ca += colabs[(int64_t)b * n + i];
      cs += colsq[(int64_t)b * n + i];
    }
    double dr, di;
    elem(A, lda, cplx, i, i, dr, di);
    const double ad = sqrt(dr * dr + di * di);
    rn_max = fmax(rn_max, sqrt(rs));
    rn_min = fmin(rn_min, sqrt(rs));
    cn_max = fmax(cn_max, sqrt(cs));
    cn_min = fmin(cn_min, sqrt(cs));
    ninf = fmax(ninf, ra);
    none = fmax(none, ca);
    const double g = dr - (ra - ad);
    gmin = fmin(gmin, g);
    cnt_disc += g <= 0.0 ? 1.0 : 0.0;
    cnt_neg += dr <= 0.0 ? 1.0 : 0.0;
    dmax = fmax(dmax, ad);
    dmin = fmin(dmin, ad);
    trr += dr;
    tri += di;
  }
  rn_max = block_max(rn_max, red);
  rn_min = -block_max(-rn_min, red);
  cn_max = block_max(cn_max, red);
  cn_min = -block_max(-cn_min, red);
  ninf = block_max(ninf, red);
  none = block_max(none, red);
  gmin = -block_max(-gmin, red);
  dmax = block_max(dmax, red);
  dmin = -block_max(-dmin, red);
  trr = block_sum(trr, red);
  tri = block_sum(tri, red);
  cnt_neg = block_sum(cnt_neg, red);
  cnt_disc = block_sum(cnt_disc, red);
  double asym = 0, tra2 = 0, fro2 = 0;
  for (int b = threadIdx.x; b < nt * nt; b += blockDim.x) {
    asym += tpart[3 * b];
    tra2 += tpart[3 * b + 1];
    fro2 += tpart[3 * b + 2];
  }
  asym = block_sum(asym, red);
  tra2 = block_sum(tra2, red);
  fro2 = block_sum(fro2, red);
  if (threadIdx.x != 0) return;
  const double fro = sqrt(fro2), rms = fro / sqrt((double)n);
  const double g = gmin / rms;
  double f[NF];
  f[0] = log2((double)n) / 10.0;
  f[1] = flag[0] ? 0.0 : 1.0;
  f[2] = log10(sqrt(asym) / fro + 1e-16) / 16.0;
  f[3] = lg10(dmax / rms, 1e-30);
  f[4] = lg10(dmin / rms, 1e-30);
  f[5] = cnt_neg / n;
  f[6] = g / (1.0 + fabs(g));
  f[7] = cnt_disc / n;
  f[8] = lg10(rn_max / fmax(rn_min, 1e-300), 1e-30);
  f[9] = lg10(cn_max / fmax(cn_min, 1e-300), 1e-30);
  f[10] = lg10(none / fro, 1e-30);
  f[11] = lg10(ninf / fro, 1e-30);
  f[12] = log10(1.0 + n * fro2 / fmax(trr * trr + tri * tri, 1e-300));
  f[13] = tra2 / fro2;
  f[14] = trr / (sqrt((double)n) * fro);
  f[15] = lg10(dmax / fmax(dmin, 1e-30), 1e-30);
  for (int k = 0; k < NF; ++k) F[k] = (float)f[k];
}

// ---- network

__device__ inline void forward_one(const float* P, const float* x, float* h1, float* h2,
                                   float* out) {
  for (int o = 0; o < HID; ++o) {
    float s = P[OFF_B1 + o];
    for (int i = 0; i < NF; ++i) s += P[o * NF + i] * x[i];
    h1[o] = fmaxf(s, 0.f);
  }
  for (int o = 0; o < HID; ++o) {
    float s = P[OFF_B2 + o];
    for (int i = 0; i < HID; ++i) s += P[OFF_W2 + o * HID + i] * h1[i];
    h2[o] = fmaxf(s, 0.f);
  }
  for (int o = 0; o < NO; ++o) {
    float s = P[OFF_B3 + o];
    for (int i = 0; i < HID; ++i) s += P[OFF_W3 + o * HID + i] * h2[i];
    out[o] = s;
  }
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(int B, const float* X, const float* P,
                                                          float* out) {
  __shared__ float p[NP];
  for (int k = threadIdx.x; k < NP; k += blockDim.x) p[k] = P[k];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  float x[NF], h1[HID], h2[HID], o[NO];
  for (int i = 0; i < NF; ++i) x[i] = X[(int64_t)s * NF + i];
  forward_one(p, x, h1, h2, o);
  for (int i = 0; i < NO; ++i) out[(int64_t)s * NO + i] = o[i];
}

// One workgroup per kGradSamples samples: forward and backward of each
// sample (threads 0..63), then the per-parameter sums over the group's
// samples (all threads) into part[block * NP + p].
__global__ __launch_bounds__(256) void mlp_grad_kernel(int B, const float* X, const float* Y,
                                                       const float* P, float* part,
                                                       float* lpart) {
  extern __shared__ float sm[];
  float* p = sm;                               // NP
  float* xs = p + NP;                          // 64 x 16
  float* h1s = xs + kGradSamples * NF;         // 64 x 64
  float* h2s = h1s + kGradSamples * HID;       // 64 x 64
  float* d1s = h2s + kGradSamples * HID;       // 64 x 64
  float* d2s = d1s + kGradSamples * HID;       // 64 x 64
  float* dos = d2s + kGradSamples * HID;       // 64 x 3
  __shared__ float lred[kGradSamples];
  const int t = threadIdx.x;
  for (int k = t; k < NP; k += blockDim.x) p[k] = P[k];
  __syncthreads();
  const int s0 = blockIdx.x * kGradSamples;
  if (t < kGradSamples) {
    const int s = s0 + t;
    float* x = xs + t * NF;
    float* h1 = h1s + t * HID;
    float* h2 = h2s + t * HID;
    float* d1 = d1s + t * HID;
    float* d2 = d2s + t * HID;
    float* dout = dos + t * NO;
    float l = 0.f;
    if (s < B) {
      for (int i = 0; i < NF; ++i) x[i] = X[(int64_t)s * NF + i];
      float o[NO];
      forward_one(p, x, h1, h2, o);
      for (int c = 0; c < NO; ++c) {
        const float diff = o[c] - Y[(int64_t)s * NO + c];
        l += diff * diff;
        dout[c] = 2.f * diff / (float)(B * NO);
      }
      for (int i = 0; i < HID; ++i) {
        float s2 = 0.f;
        for (int c = 0; c < NO; ++c) s2 += dout[c] * p[OFF_W3 + c * HID + i];
        d2[i] = h2[i] > 0.f ? s2 : 0.f;
      }
      for (int i = 0; i < HID; ++i) {
        float s1 = 0.f;
        for (int o2 = 0; o2 < HID; ++o2) s1 += d2[o2] * p[OFF_W2 + o2 * HID + i];
        d1[i] = h1[i] > 0.f ? s1 : 0.f;
      }
    } else {
      for (int i = 0; i < NF; ++i) x[i] = 0.f;
      for (int i = 0; i < HID; ++i) h1[i] = h2[i] = d1[i] = d2[i] = 0.f;
      for (int c = 0; c < NO; ++c) dout[c] = 0.f;
    }
    lred[t] = l;
  }
  __syncthreads();
  for (int k = t; k < NP; k += blockDim.x) {
    float g = 0.f;
    if (k < OFF_B1) {
      const int o = k / NF, i = k % NF;
      for (int s = 0; s < kGradSamples; ++s) g += d1s[s * HID + o] * xs[s * NF + i];
    } else if (k < OFF_W2) {
      const int o = k - OFF_B1;
      for (int s = 0; s < kGradSamples; ++s) g += d1s[s * HID + o];
    } else if (k < OFF_B2) {
      const int o = (k - OFF_W2) / HID, i = (k - OFF_W2) % HID;
      for (int s = 0; s < kGradSamples; ++s) g += d2s[s * HID + o] * h1s[s * HID + i];
    } else if (k < OFF_W3) {
      const int o = k - OFF_B2;
      for (int s = 0; s < kGradSamples; ++s) g += d2s[s * HID + o];
    } else if (k < OFF_B3) {
      const int o = (k - OFF_W3) / HID, i = (k - OFF_W3) % HID;
      for (int s = 0; s < kGradSamples; ++s) g += dos[s * NO + o] * h2s[s * HID + i];
    } else {
      const int o = k - OFF_B3;
      for (int s = 0; s < kGradSamples; ++s) g += dos[s * NO + o];
    }
    part[(int64_t)blockIdx.x * NP + k] = g;
  }
  if (t == 0) {
    float l = 0.f;
    for (int s = 0; s < kGradSamples; ++s) l += lred[s];
    lpart[blockIdx.x] = l;
  }
}

__global__ void mlp_reduce_kernel(int nblk, int B, const float* part, const float* lpart,
                                  float* grad, float* loss) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < NP) {
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += part[(int64_t)b * NP + k];
    grad[k] = g;
  }
  if (k == 0) {
    float l = 0.f;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    loss[0] = l / (float)(B * NO);
  }
}

__global__ void mlp_adam_kernel(const float* g, float* p, float* m, float* v, float lr, float b1,
                                float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NP) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Normalisation and forward pass of one feature vector (64 threads).
__global__ __launch_bounds__(64) void infer_kernel(const float* F, const float* mean,
                                                   const float* scale, const float* P,
                                                   float* out) {
  __shared__ float x[NF], h1[HID], h2[HID];
  const int t = threadIdx.x;
  if (t < NF) x[t] = (F[t] - mean[t]) / scale[t];
  __syncthreads();
  float s = P[OFF_B1 + t];
  for (int i = 0; i < NF; ++i) s += P[t * NF + i] * x[i];
  h1[t] = fmaxf(s, 0.f);
  __syncthreads();
  s = P[OFF_B2 + t];
  for (int i = 0; i < HID; ++i) s += P[OFF_W2 + t * HID + i] * h1[i];
  h2[t] = fmaxf(s, 0.f);
  __syncthreads();
  if (t < NO) {
    s = P[OFF_B3 + t];
    for (int i = 0; i < HID; ++i) s += P[OFF_W3 + t * HID + i] * h2[i];
    out[t] = s;
  }
}

// ---- installed selector

struct Installed {
  bool set = false;
  std::vector<float> params, mean, scale;
  std::vector<double> cost;
};
std::mutex g_sel_mu;
Installed g_sel;
std::map<int, void*> g_sel_dev;  // per device: params | mean | scale | features | out

float* device_selector(hipStream_t st) {
  int dev = 0;
  MSQRT_HIP(hipGetDevice(&dev));
  auto it = g_sel_dev.find(dev);
  float* d;
  if (it == g_sel_dev.end()) {
    void* p = nullptr;
    MSQRT_HIP(hipMalloc(&p, sizeof(float) * (NP + 4 * NF + 8)));
    g_sel_dev[dev] = p;
    d = (float*)p;
  } else {
    d = (float*)it->second;
  }
  MSQRT_HIP(hipMemcpyAsync(d, g_sel.params.data(), sizeof(float) * NP, hipMemcpyHostToDevice, st));
  MSQRT_HIP(hipMemcpyAsync(d + NP, g_sel.mean.data(), sizeof(float) * NF, hipMemcpyHostToDevice, st));
  MSQRT_HIP(hipMemcpyAsync(d + NP + NF, g_sel.scale.data(), sizeof(float) * NF,
                           hipMemcpyHostToDevice, st));
  return d;
}

}  // namespace

void selector_release() {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (auto& kv : g_sel_dev) {
    if (hipSetDevice(kv.first) == hipSuccess) (void)hipFree(kv.second);
  }
  if (have) (void)hipSetDevice(cur);
  g_sel_dev.clear();
}

void launch_features(hipStream_t st, int n, const double* A, int64_t lda, int cplx, float* F) {
  const int nt = (int)ceil_div(n, kFT);
  DevBuf work;
  double* w = work.ensure<double>(4 * (int64_t)nt * n + 3 * (int64_t)nt * nt + 8);
  double* rowabs = w;
  double* rowsq = rowabs + (int64_t)nt * n;
  double* colabs = rowsq + (int64_t)nt * n;
  double* colsq = colabs + (int64_t)nt * n;
  double* tpart = colsq + (int64_t)nt * n;
  int* flag = (int*)(tpart + 3 * (int64_t)nt * nt);
  MSQRT_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  hipLaunchKernelGGL(feat_tiles_kernel, dim3(nt * nt), dim3(256), 0, st, n, A, lda, cplx, nt,
                     rowabs, rowsq, colabs, colsq, tpart, flag);
  MSQRT_LAUNCH_CHECK();
  hipLaunchKernelGGL(feat_final_kernel, dim3(1), dim3(1024), 0, st, n, A, lda, cplx, nt,
                     (const double*)rowabs, (const double*)rowsq, (const double*)colabs,
                     (const double*)colsq, (const double*)tpart, (const int*)flag, F);
  MSQRT_LAUNCH_CHECK();
  // keep the workspace alive until the kernels have run
  MSQRT_HIP(hipStreamSynchronize(st));
}

// Precision for MSQRT_PREC_AUTO: the installed selector's choice (per batch
// entry; the highest precision chosen for any entry), FP32 without one.
msqrt_prec select_precision(const msqrt_options& o, msqrt_dtype dtype, int64_t n, const void* A,
                            int64_t lda, int64_t sA, hipStream_t st, msqrt_info* info,
                            PhaseTimer& tm) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  if (!g_sel.set || n < 1) return MSQRT_PREC_FP32;
  tm.begin(MSQRT_T_SELECT);
  float* d = device_selector(st);
  float* dF = d + NP + 2 * NF;
  float* dOut = dF + NF;
  const int cplx = dtype == MSQRT_COMPLEX128;
  const int64_t stride_el = cplx ? 2 * sA : sA;
  int best = 0;
  for (int64_t b = 0; b < o.batch; ++b) {
    launch_features(st, (int)n, (const double*)A + b * stride_el, lda, cplx, dF);
    hipLaunchKernelGGL(infer_kernel, dim3(1), dim3(64), 0, st, (const float*)dF,
                       (const float*)(d + NP), (const float*)(d + NP + NF), (const float*)d, dOut);
    MSQRT_LAUNCH_CHECK();
    float y[NO], f1[NF];
    MSQRT_HIP(hipMemcpyAsync(y, dOut, sizeof(y), hipMemcpyDeviceToHost, st));
    MSQRT_HIP(hipMemcpyAsync(f1, dF, sizeof(f1), hipMemcpyDeviceToHost, st));
    MSQRT_HIP(hipStreamSynchronize(st));
    const int s = (f1[1] > 0.5f && !cplx) ? 0 : 1;  // cost model: HPD or general
    const double nn = (double)n;
    auto t = [&](int q) {
      const double* c = &g_sel.cost[(7 * s + q) * 3];
      return std::max(0.0, c[0] * nn * nn * nn + c[1] * nn * nn + c[2]);
    };
    double best_cost = INFINITY;
    int choice = 1;
    // the network predicts log(1 + corrections)
    for (int p = 0; p < NO; ++p) y[p] = (float)std::expm1(std::min((double)y[p], 5.0));
    for (int p = 0; p < NO; ++p) {
      const double yp = std::min(std::max((double)y[p], 0.0), (double)o.maxit + 10.0);
      const double c = t(p) + (yp + 1.0) * t(6) + yp * t(3 + p);
      if (c < best_cost) { best_cost = c; choice = p; }
    }
    best = std::max(best, choice);
    if (info && b == 0)
      for (int p = 0; p < NO; ++p) info->predicted_steps[p] = y[p];
  }
  tm.end();
  static const msqrt_prec map[3] = {MSQRT_PREC_BF16SPLIT, MSQRT_PREC_FP32, MSQRT_PREC_FP64};
  return map[best];
}

}  // namespace msqrt

using namespace msqrt;

#define SEL_TRY try {
#define SEL_CATCH                                       \
  }                                                     \
  catch (const Error& e) {                              \
    set_last_error(e.msg);                              \
    return (msqrt_status)e.status;                      \
  }                                                     \
  catch (...) {                                         \
    set_last_error("unknown error");                    \
    return MSQRT_ERR_DEVICE;                            \
  }

extern "C" {

msqrt_status msqrt_features(msqrt_dtype dtype, int64_t n, const void* dA, int64_t lda, float* dF,
                            hipStream_t stream) {
  SEL_TRY
  if (n < 1 || !dA || !dF || lda < n || (dtype != MSQRT_REAL64 && dtype != MSQRT_COMPLEX128)) {
    set_last_error("msqrt_features: invalid argument");
    return MSQRT_ERR_INVALID_ARG;
  }
  launch_features(stream, (int)n, (const double*)dA, lda, dtype == MSQRT_COMPLEX128, dF);
  return MSQRT_OK;
  SEL_CATCH
}

msqrt_status msqrt_mlp_forward(int64_t batch, const float* dX, const float* dP, float* dOut,
                               hipStream_t stream) {
  SEL_TRY
  if (batch < 1 || !dX || !dP || !dOut) return MSQRT_ERR_INVALID_ARG;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)ceil_div(batch, 256)), dim3(256), 0,
                     stream, (int)batch, dX, dP, dOut);
  MSQRT_LAUNCH_CHECK();
  return MSQRT_OK;
  SEL_CATCH
}

msqrt_status msqrt_mlp_grad(int64_t batch, const float* dX, const float* dY, const float* dP,
                            float* dGrad, float* dLoss, hipStream_t stream) {
  SEL_TRY
  if (batch < 1 || !dX || !dY || !dP || !dGrad || !dLoss) return MSQRT_ERR_INVALID_ARG;
  const int nblk = (int)ceil_div(batch, kGradSamples);
  DevBuf work;
  float* part = work.ensure<float>((int64_t)nblk * NP + nblk + 8);
  float* lpart = part + (int64_t)nblk * NP;
  const size_t lds = sizeof(float) * (NP + kGradSamples * (NF + 4 * HID + NO));
  static bool attr = false;
  if (!attr) {
    MSQRT_HIP(hipFuncSetAttribute((const void*)mlp_grad_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(256), lds, stream, (int)batch, dX, dY, dP,
                     part, lpart);
  MSQRT_LAUNCH_CHECK();
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)ceil_div(NP, 256)), dim3(256), 0, stream,
                     nblk, (int)batch, (const float*)part, (const float*)lpart, dGrad, dLoss);
  MSQRT_LAUNCH_CHECK();
  MSQRT_HIP(hipStreamSynchronize(stream));
  return MSQRT_OK;
  SEL_CATCH
}

msqrt_status msqrt_mlp_adam(const float* dGrad, float* dP, float* dM, float* dV, int step,
                            float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  SEL_TRY
  if (!dGrad || !dP || !dM || !dV || step < 1) return MSQRT_ERR_INVALID_ARG;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)ceil_div(NP, 256)), dim3(256), 0, stream,
                     dGrad, dP, dM, dV, lr, beta1, beta2, eps, c1, c2);
  MSQRT_LAUNCH_CHECK();
  return MSQRT_OK;
  SEL_CATCH
}

msqrt_status msqrt_selector_set(const float* params, const float* feat_mean,
                                const float* feat_scale, const double* cost, int ncost) {
  if (!params || !feat_mean || !feat_scale || !cost || ncost != MSQRT_SEL_NCOST) {
    set_last_error("msqrt_selector_set: invalid argument");
    return MSQRT_ERR_INVALID_ARG;
  }
  for (int i = 0; i < NF; ++i)
    if (!(feat_scale[i] > 0.f)) {
      set_last_error("msqrt_selector_set: feature scales must be positive");
      return MSQRT_ERR_INVALID_ARG;
    }
  std::lock_guard<std::mutex> lk(g_sel_mu);
  g_sel.params.assign(params, params + NP);
  g_sel.mean.assign(feat_mean, feat_mean + NF);
  g_sel.scale.assign(feat_scale, feat_scale + NF);
  g_sel.cost.assign(cost, cost + ncost);
  g_sel.set = true;
  return MSQRT_OK;
}

msqrt_status msqrt_selector_load(const char* path) {
  if (!path) return MSQRT_ERR_INVALID_ARG;
  FILE* fp = std::fopen(path, "rb");
  if (!fp) {
    set_last_error(std::string("msqrt_selector_load: cannot open ") + path);
    return MSQRT_ERR_INVALID_ARG;
  }
  char magic[8];
  int32_t hdr[3];
  std::vector<float> p(NP), m(NF), s(NF);
  std::vector<double> c(MSQRT_SEL_NCOST);
  bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "MSQSEL01", 8) == 0 &&
            std::fread(hdr, sizeof(int32_t), 3, fp) == 3 && hdr[0] == NP && hdr[1] == NF &&
            hdr[2] == MSQRT_SEL_NCOST && std::fread(p.data(), sizeof(float), NP, fp) == (size_t)NP &&
            std::fread(m.data(), sizeof(float), NF, fp) == (size_t)NF &&
            std::fread(s.data(), sizeof(float), NF, fp) == (size_t)NF &&
            std::fread(c.data(), sizeof(double), MSQRT_SEL_NCOST, fp) == (size_t)MSQRT_SEL_NCOST;
  std::fclose(fp);
  if (!ok) {
    set_last_error(std::string("msqrt_selector_load: malformed file ") + path);
    return MSQRT_ERR_INVALID_ARG;
  }
  return msqrt_selector_set(p.data(), m.data(), s.data(), c.data(), MSQRT_SEL_NCOST);
}

void msqrt_selector_clear(void) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  g_sel.set = false;
}

int msqrt_selector_installed(void) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  return g_sel.set ? 1 : 0;
}

}  // extern "C"
