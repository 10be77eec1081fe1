// Back-transformation Q = H_0 H_1 ... H_{n-2} Z of the tridiagonal
// eigenvectors (completing the spectral decomposition A = Q diag(lam) Q^T).
//
// Reflectors are grouped in blocks of kBlk = 128: H_B ... H_{B+127} =
// I - V T V^T (compact WY, T upper triangular from the Gram matrix V^T V).
// VT = V T is formed once per block; the blocks are then applied from the
// last to the first as  Z(B+1:, :) -= VT (V^T Z(B+1:, :)),  the inner product
// V^T Z as a split-K MFMA GEMM (partials over row chunks, summed in a fixed
// order, so results are reproducible) and the update as one MFMA GEMM.
#include <algorithm>

#include "kernels.hpp"
#include "tridiag.hpp"

namespace msqrt {

namespace {

constexpr int kBlk = 128;

// Zero the rows above each explicit reflector (v_j(i) = 0 for i <= j) so that
// full-height products can be used; the unit entry v_j(j+1) = 1 is already
// stored.
template <typename T>
__global__ void clean_reflectors(int n, T* V, int64_t sV) {
  const int j = blockIdx.x;
  V += (int64_t)blockIdx.y * sV;
  for (int i = threadIdx.x; i <= j && i < n; i += blockDim.x) V[i + (int64_t)j * n] = T(0);
}

// T factor of one block from its Gram matrix G = V^T V (forward, columnwise):
// T(i,i) = tau_i,  T(0:i, i) = -tau_i T(0:i, 0:i) G(0:i, i).
// Column i is a triangular matrix-vector product, so each row r of T has
// kParts lanes that sum every kParts-th term of its row (adjacent lanes of
// one wave, combined with lane shuffles): the serial chain of a column is
// i / kParts products instead of i.
constexpr int kParts = 8;
constexpr int kLarftThreads = kBlk * kParts;
template <typename T>
__global__ __launch_bounds__(kLarftThreads) void larft_kernel(int nb_total, const T* G, const T* tau,
                                                              T* Tm, int64_t sG, int64_t sTau,
                                                              int64_t sTm) {
  static_assert(kWave % kParts == 0, "a row's lanes lie in one wave");
  const int blk = blockIdx.x;
  G += (int64_t)blockIdx.y * sG;
  tau += (int64_t)blockIdx.y * sTau;
  Tm += (int64_t)blockIdx.y * sTm;
  const int B = blk * kBlk;
  const int nbk = min(kBlk, nb_total - B);
  const T* g = G + (int64_t)blk * kBlk * kBlk;
  T* t = Tm + (int64_t)blk * kBlk * kBlk;
  const int r = threadIdx.x / kParts, part = threadIdx.x % kParts;
  // Row r of T lives in LDS (padded to avoid bank conflicts on columns).
  __shared__ T tl[kBlk][kBlk + 1];
  __shared__ T col[kBlk];
  for (int x = threadIdx.x; x < kBlk * (kBlk + 1); x += kLarftThreads) (&tl[0][0])[x] = T(0);
  __syncthreads();
  for (int i = 0; i < nbk; ++i) {
    if (threadIdx.x < i) col[threadIdx.x] = g[threadIdx.x + (int64_t)i * kBlk];
    __syncthreads();
    T acc = T(0);
    if (r < i)
      for (int c = r + part; c < i; c += kParts) acc += tl[r][c] * col[c];
#pragma unroll
    for (int m = kParts / 2; m >= 1; m /= 2) acc += __shfl_xor(acc, m, kParts);
    if (part == 0) {
      if (r < i) tl[r][i] = -tau[B + i] * acc;
      if (r == i) tl[i][i] = tau[B + i];
    }
    __syncthreads();
  }
  for (int x = threadIdx.x; x < kBlk * kBlk; x += kLarftThreads) t[x % kBlk + (int64_t)(x / kBlk) * kBlk] = tl[x % kBlk][x / kBlk];
}

template <typename T>
__global__ void sum_partials(int count, int splits, const T* P, int64_t stride, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  T s = T(0);
  for (int q = 0; q < splits; ++q) s += P[i + q * stride];
  out[i] = s;
}

}  // namespace

template <typename T>
void ormtr(hipStream_t st, int n, const T* Vc, const T* tau, T* Z, OrmtrWork& w) {
  if (n - 1 <= 0) return;
  hipLaunchKernelGGL(clean_reflectors<T>, dim3(n), dim3(256), 0, st, n, const_cast<T*>(Vc),
                     (int64_t)0);
  MSQRT_LAUNCH_CHECK();
  ormtr_blocks<T>(st, n, n - 1, 1, Vc, tau, Z, w);
}

template <typename T>
void ormtr_blocks(hipStream_t st, int n, int nref, int off, const T* Vc, const T* tau, T* Z,
                  OrmtrWork& w) {
  if (nref <= 0) return;
  const T* V = Vc;
  const int nblk = (int)ceil_div(nref, kBlk);
  T* G = w.gram.ensure<T>((int64_t)nblk * kBlk * kBlk * 2);
  T* Tm = G + (int64_t)nblk * kBlk * kBlk;
  T* VT = w.VT.ensure<T>((int64_t)nblk * kBlk * n);
  // Gram matrices of all blocks (full height: rows above a reflector are 0).
  const int full = nref / kBlk;
  auto gemm = [&](bool ta, bool tb, int M, int N, int K, const T* A, int64_t lda, int64_t sA,
                  const T* B, int64_t ldb, int64_t sB, T* C, int64_t ldc, int64_t sC, T alpha,
                  T beta, int batch) {
    if (std::is_same<T, float>::value)
      gemm_store_f32(st, ta, tb, M, N, K, (const float*)A, lda, sA, (const float*)B, ldb, sB,
                     (float*)C, ldc, sC, (float)alpha, (float)beta, batch, false);
    else
      gemm_store_f64(st, ta, tb, M, N, K, (const double*)A, lda, sA, (const double*)B, ldb, sB,
                     (double*)C, ldc, sC, (double)alpha, (double)beta, batch, false);
  };
  MSQRT_HIP(hipMemsetAsync(G, 0, sizeof(T) * (size_t)nblk * kBlk * kBlk, st));
  if (full > 0)
    gemm(true, false, kBlk, kBlk, n, V, n, (int64_t)kBlk * n, V, n, (int64_t)kBlk * n, G, kBlk,
         (int64_t)kBlk * kBlk, T(1), T(0), full);
  if (full < nblk) {
    // rows above the block's first reflector are zero: K = n - r0
    const int nbk = nref - full * kBlk, r0 = std::min(n - 1, full * kBlk + off);
    const T* Vb = V + (int64_t)full * kBlk * n + r0;
    gemm(true, false, nbk, nbk, n - r0, Vb, n, 0, Vb, n, 0, G + (int64_t)full * kBlk * kBlk, kBlk, 0,
         T(1), T(0), 1);
  }
  hipLaunchKernelGGL(larft_kernel<T>, dim3(nblk), dim3(kLarftThreads), 0, st, nref, (const T*)G, tau, Tm,
                     (int64_t)0, (int64_t)0, (int64_t)0);
  MSQRT_LAUNCH_CHECK();
  // VT_b = V_b T_b (n x nbk)
  if (full > 0)
    gemm(false, false, n, kBlk, kBlk, V, n, (int64_t)kBlk * n, Tm, kBlk, (int64_t)kBlk * kBlk, VT,
         n, (int64_t)kBlk * n, T(1), T(0), full);
  if (full < nblk) {
    const int nbk = nref - full * kBlk;
    gemm(false, false, n, nbk, nbk, V + (int64_t)full * kBlk * n, n, 0,
         Tm + (int64_t)full * kBlk * kBlk, kBlk, 0, VT + (int64_t)full * kBlk * n, n, 0, T(1),
         T(0), 1);
  }
  // Apply the blocks, last to first.
  const int splits_max = 16;
  T* Wp = w.Wpart.ensure<T>((int64_t)splits_max * kBlk * n);
  T* W = w.W.ensure<T>((int64_t)kBlk * n);
  for (int b = nblk - 1; b >= 0; --b) {
    const int B = b * kBlk;
    const int nbk = std::min(kBlk, nref - B);
    const int r0 = B + off;
    const int rows = n - r0;
    const T* Vb = V + (int64_t)B * n;
    int splits = (int)std::min<int64_t>(splits_max, std::max<int64_t>(1, ceil_div(rows, 256)));
    const int chunk = (int)ceil_div(rows, splits);
    splits = (int)ceil_div(rows, chunk);
    const int klast = rows - (splits - 1) * chunk;
    // Wp[q] = V_b(rows chunk q)^T Z(rows chunk q, :)   (nbk x n each)
    gemm_store_splitk<T>(st, true, false, nbk, n, chunk, klast, Vb + r0, n, chunk, Z + r0, n,
                         chunk, Wp, nbk, (int64_t)nbk * n, splits);
    const int cnt = nbk * n;
    hipLaunchKernelGGL(sum_partials<T>, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, cnt,
                       splits, (const T*)Wp, (int64_t)nbk * n, W);
    MSQRT_LAUNCH_CHECK();
    // Z(r0:, :) -= VT_b(r0:, :) W
    gemm(false, false, rows, n, nbk, VT + (int64_t)b * kBlk * n + r0, n, 0, W, nbk, 0, Z + r0, n,
         0, T(-1), T(1), 1);
  }
}

template <typename T>
void ormtr_batched(hipStream_t st, int n, int batch, const T* Vc, int64_t sV, const T* tau,
                   int64_t sTau, T* Z, int64_t sZ, OrmtrWork& w) {
  if (batch == 1) {
    ormtr<T>(st, n, Vc, tau, Z, w);
    return;
  }
  const int nref = n - 1;
  if (nref <= 0 || batch <= 0) return;
  const int nblk = (int)ceil_div(nref, kBlk);
  const int full = nref / kBlk;
  const int64_t sG = (int64_t)nblk * kBlk * kBlk * 2, sVT = (int64_t)nblk * kBlk * n;
  T* Gall = w.gram.ensure<T>(sG * batch);
  T* VTall = w.VT.ensure<T>(sVT * batch);
  T* Wall = w.W.ensure<T>((int64_t)kBlk * n * batch);
  auto gemm = [&](bool ta, bool tb, int M, int N, int K, const T* A, int64_t lda, int64_t sA,
                  const T* B, int64_t ldb, int64_t sB, T* C, int64_t ldc, int64_t sC, T alpha,
                  T beta, int nb) {
    if (std::is_same<T, float>::value)
      gemm_store_f32(st, ta, tb, M, N, K, (const float*)A, lda, sA, (const float*)B, ldb, sB,
                     (float*)C, ldc, sC, (float)alpha, (float)beta, nb, false);
    else
      gemm_store_f64(st, ta, tb, M, N, K, (const double*)A, lda, sA, (const double*)B, ldb, sB,
                     (double*)C, ldc, sC, (double)alpha, (double)beta, nb, false);
  };
  // clean reflectors, Gram matrices, T factors and VT = V T of every entry:
  // one launch per reflector block (batched over entries) for each product
  T* V = const_cast<T*>(Vc);
  const int64_t offT = (int64_t)nblk * kBlk * kBlk;  // T factors follow the Gram blocks
  hipLaunchKernelGGL(clean_reflectors<T>, dim3(n, batch), dim3(256), 0, st, n, V, sV);
  MSQRT_LAUNCH_CHECK();
  MSQRT_HIP(hipMemsetAsync(Gall, 0, sizeof(T) * (size_t)(sG * batch), st));
  for (int b = 0; b < nblk; ++b) {
    // rows above the block's first reflector (row b kBlk + 1) are zero
    const int nbk = std::min(kBlk, nref - b * kBlk), r0 = std::min(n - 1, b * kBlk + 1);
    const T* Vb = Vc + (int64_t)b * kBlk * n + r0;
    gemm(true, false, nbk, nbk, n - r0, Vb, n, sV, Vb, n, sV, Gall + (int64_t)b * kBlk * kBlk, kBlk,
         sG, T(1), T(0), batch);
  }
  hipLaunchKernelGGL(larft_kernel<T>, dim3(nblk, batch), dim3(kLarftThreads), 0, st, nref, (const T*)Gall,
                     tau, Gall + offT, sG, sTau, sG);
  MSQRT_LAUNCH_CHECK();
  for (int b = 0; b < nblk; ++b) {
    const int nbk = std::min(kBlk, nref - b * kBlk);
    gemm(false, false, n, nbk, nbk, Vc + (int64_t)b * kBlk * n, n, sV,
         Gall + offT + (int64_t)b * kBlk * kBlk, kBlk, sG, VTall + (int64_t)b * kBlk * n, n, sVT,
         T(1), T(0), batch);
  }
  // the blocks, last to first, each applied to every entry by two batched
  // GEMMs (the batch supplies the parallelism that split-K gives one matrix)
  for (int b = nblk - 1; b >= 0; --b) {
    const int B = b * kBlk;
    const int nbk = std::min(kBlk, nref - B);
    const int r0 = B + 1;
    const int rows = n - r0;
    // W_m = V_m(r0:, B:B+nbk)^T Z_m(r0:, :)
    gemm(true, false, nbk, n, rows, Vc + (int64_t)B * n + r0, n, sV, Z + r0, n, sZ, Wall, nbk,
         (int64_t)kBlk * n, T(1), T(0), batch);
    // Z_m(r0:, :) -= VT_m(r0:, block) W_m
    gemm(false, false, rows, n, nbk, VTall + (int64_t)b * kBlk * n + r0, n, sVT, Wall, nbk,
         (int64_t)kBlk * n, Z + r0, n, sZ, T(-1), T(1), batch);
  }
}

template void ormtr<float>(hipStream_t, int, const float*, const float*, float*, OrmtrWork&);
template void ormtr<double>(hipStream_t, int, const double*, const double*, double*, OrmtrWork&);
template void ormtr_batched<float>(hipStream_t, int, int, const float*, int64_t, const float*,
                                   int64_t, float*, int64_t, OrmtrWork&);
template void ormtr_batched<double>(hipStream_t, int, int, const double*, int64_t, const double*,
                                    int64_t, double*, int64_t, OrmtrWork&);
template void ormtr_blocks<float>(hipStream_t, int, int, int, const float*, const float*, float*,
                                  OrmtrWork&);
template void ormtr_blocks<double>(hipStream_t, int, int, int, const double*, const double*,
                                   double*, OrmtrWork&);

}  // namespace msqrt
