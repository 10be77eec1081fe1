// Elementwise and reduction kernels: validation, norms, casts, scaling.
// All are HBM-bound; each thread handles a contiguous run within a column so
// that a wave reads consecutive addresses.
#include "kernels.hpp"

namespace msqrt {

namespace {

constexpr int kEwThreads = 256;

// One block per 32 x 32 tile (lower triangle of tiles) and batch entry: reads
// the tile and its mirror with coalesced loads, compares through LDS, and
// accumulates finiteness, exact symmetry (a_ij == a_ji) and the sum of squares
// (off-diagonal tiles count both copies).
__global__ __launch_bounds__(kEwThreads) void validate_kernel(int n, const double* __restrict__ A,
                                                              int64_t lda, int64_t sA,
                                                              int check_sym, int* flags,
                                                              double* partials) {
  __shared__ double red[kEwThreads / kWave];
  __shared__ double tT[32][33];
  const int b = blockIdx.y;
  const double* a = A + (int64_t)b * sA;
  const int id = blockIdx.x;
  int ti = (int)((sqrt(8.0 * id + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= id) ++ti;
  while (ti * (ti + 1) / 2 > id) --ti;
  const int tj = id - ti * (ti + 1) / 2;
  const int i0 = ti * 32, j0 = tj * 32;
  const int lx = threadIdx.x % 32, ly = threadIdx.x / 32;  // 32 x 8
  double ss = 0.0;
  int bad = 0, asym = 0;
  // mirror tile (rows j0.., cols i0..) into LDS, transposed
  if (ti != tj) {
    for (int c = ly; c < 32; c += 8) {
      const int row = j0 + lx, col = i0 + c;
      tT[c][lx] = (row < n && col < n) ? a[row + (int64_t)col * lda] : 0.0;
    }
  }
  __syncthreads();
  for (int c = ly; c < 32; c += 8) {
    const int row = i0 + lx, col = j0 + c;
    if (row < n && col < n) {
      const double v = a[row + (int64_t)col * lda];
      if (!isfinite(v)) bad = 1;
      if (ti == tj) {
        ss += v * v;
        if (check_sym && row > col && v != a[col + (int64_t)row * lda]) asym = 1;
      } else {
        const double w = tT[lx][c];  // a(col, row)
        if (!isfinite(w)) bad = 1;
        ss += v * v + w * w;
        if (check_sym && v != w) asym = 1;
      }
    }
  }
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) partials[(int64_t)b * gridDim.x + blockIdx.x] = ss;
  if (bad) atomicOr(&flags[b], 1);
  if (asym) atomicOr(&flags[b], 2);
}

// p[i] = v for i < count (clears flags without a memset node).
__global__ __launch_bounds__(kEwThreads) void fill_i32_kernel(int* p, int count, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ __launch_bounds__(kEwThreads) void reduce_sqrt_kernel(const double* __restrict__ p,
                                                                 int count, double* out) {
  __shared__ double red[kEwThreads / kWave];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) s += p[(int64_t)b * count + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[b] = sqrt(s);
}

template <typename TO>
__global__ __launch_bounds__(kEwThreads) void cast_scale_kernel(int n, const double* __restrict__ A,
                                                                int64_t lda, int64_t sA,
                                                                const double* scale,
                                                                TO* __restrict__ B, int64_t ldb,
                                                                int64_t sB) {
  const int b = blockIdx.z;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double sc = scale ? scale[b] : 1.0;
  if (i < n) B[(int64_t)b * sB + i + (int64_t)j * ldb] = (TO)(sc * A[(int64_t)b * sA + i + (int64_t)j * lda]);
}

template <typename T>
__global__ __launch_bounds__(kEwThreads) void scale_cols_kernel(int n, const T* __restrict__ Q,
                                                                int64_t ldq, int64_t sQ,
                                                                const T* __restrict__ s, int64_t sS,
                                                                T* __restrict__ W, int64_t ldw,
                                                                int64_t sW) {
  const int b = blockIdx.z;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) W[(int64_t)b * sW + i + (int64_t)j * ldw] = Q[(int64_t)b * sQ + i + (int64_t)j * ldq] * s[(int64_t)b * sS + j];
}

__global__ __launch_bounds__(kEwThreads) void scale_inplace_kernel(int n, double* X, int64_t ldx,
                                                                   int64_t sX,
                                                                   const double* scale) {
  const int b = blockIdx.z;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) X[(int64_t)b * sX + i + (int64_t)j * ldx] *= scale[b];
}

// Real representation of a complex matrix (interleaved complex, column
// index j): E = [[Re A, -Im A], [Im A, Re A]] (2n x 2n, ld 2n).  The map is an
// algebra homomorphism, E is symmetric exactly when A is Hermitian and
// positive definite exactly when A is.
__global__ __launch_bounds__(kEwThreads) void embed_complex_kernel(int n, const double* __restrict__ A,
                                                                   int64_t lda, int64_t sA,
                                                                   double* __restrict__ E,
                                                                   int64_t sE) {
  const int b = blockIdx.z;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* a = A + (int64_t)b * sA + 2 * ((int64_t)i + (int64_t)j * lda);
  const double re = a[0], im = a[1];
  double* e = E + (int64_t)b * sE;
  const int64_t ld = 2 * (int64_t)n;
  e[i + j * ld] = re;
  e[n + i + j * ld] = im;
  e[i + (n + j) * ld] = -im;
  e[n + i + (n + j) * ld] = re;
}

// Complex matrix back from a real representation, averaging the two copies
// of each part: X = (E11 + E22)/2 + i (E21 - E12)/2.
__global__ __launch_bounds__(kEwThreads) void extract_complex_kernel(int n, const double* __restrict__ E,
                                                                     int64_t sE, double* __restrict__ X,
                                                                     int64_t ldx, int64_t sX) {
  const int b = blockIdx.z;
  const int j = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* e = E + (int64_t)b * sE;
  const int64_t ld = 2 * (int64_t)n;
  double* x = X + (int64_t)b * sX + 2 * ((int64_t)i + (int64_t)j * ldx);
  x[0] = 0.5 * (e[i + j * ld] + e[n + i + (n + j) * ld]);
  x[1] = 0.5 * (e[n + i + j * ld] - e[i + (n + j) * ld]);
}

}  // namespace

int launch_validate(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA, int batch,
                    int check_sym, int* flags, double* partials) {
  const int nt = (int)ceil_div(n, 32);
  const int nblk = nt * (nt + 1) / 2;
  if (n <= 0) return 0;
  hipLaunchKernelGGL(validate_kernel, dim3(nblk, batch), dim3(kEwThreads), 0, st, n, A, lda, sA,
                     check_sym, flags, partials);
  MSQRT_LAUNCH_CHECK();
  return nblk;
}

void launch_embed_complex(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA,
                          double* E, int64_t sE, int batch) {
  if (n <= 0) return;
  hipLaunchKernelGGL(embed_complex_kernel, dim3((unsigned)ceil_div(n, kEwThreads), n, batch), dim3(kEwThreads),
                     0, st, n, A, lda, sA, E, sE);
  MSQRT_LAUNCH_CHECK();
}

void launch_extract_complex(hipStream_t st, int n, const double* E, int64_t sE, double* X,
                            int64_t ldx, int64_t sX, int batch) {
  if (n <= 0) return;
  hipLaunchKernelGGL(extract_complex_kernel, dim3((unsigned)ceil_div(n, kEwThreads), n, batch),
                     dim3(kEwThreads), 0, st, n, E, sE, X, ldx, sX);
  MSQRT_LAUNCH_CHECK();
}

void launch_fill_i32(hipStream_t st, int* p, int count, int v) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((count + kEwThreads - 1) / kEwThreads), dim3(kEwThreads),
                     0, st, p, count, v);
  MSQRT_LAUNCH_CHECK();
}

void launch_reduce_sqrt(hipStream_t st, const double* partials, int count, int batch, double* out) {
  hipLaunchKernelGGL(reduce_sqrt_kernel, dim3(batch), dim3(kEwThreads), 0, st, partials, count, out);
  MSQRT_LAUNCH_CHECK();
}

void launch_cast_scale_f64_f32(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA,
                               const double* scale, float* B, int64_t ldb, int64_t sB, int batch) {
  if (n <= 0) return;
  dim3 grid((unsigned)ceil_div(n, kEwThreads), n, batch);
  hipLaunchKernelGGL(cast_scale_kernel<float>, grid, dim3(kEwThreads), 0, st, n, A, lda, sA, scale, B, ldb, sB);
  MSQRT_LAUNCH_CHECK();
}

void launch_cast_scale_f64_f64(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA,
                               const double* scale, double* B, int64_t ldb, int64_t sB, int batch) {
  if (n <= 0) return;
  dim3 grid((unsigned)ceil_div(n, kEwThreads), n, batch);
  hipLaunchKernelGGL(cast_scale_kernel<double>, grid, dim3(kEwThreads), 0, st, n, A, lda, sA, scale, B, ldb, sB);
  MSQRT_LAUNCH_CHECK();
}

void launch_copy_f64(hipStream_t st, int n, const double* A, int64_t lda, int64_t sA, double* B,
                     int64_t ldb, int64_t sB, int batch) {
  launch_cast_scale_f64_f64(st, n, A, lda, sA, nullptr, B, ldb, sB, batch);
}

template <typename T>
void launch_scale_cols(hipStream_t st, int n, const T* Q, int64_t ldq, int64_t sQ, const T* s,
                       int64_t sS, T* W, int64_t ldw, int64_t sW, int batch) {
  if (n <= 0) return;
  dim3 grid((unsigned)ceil_div(n, kEwThreads), n, batch);
  hipLaunchKernelGGL(scale_cols_kernel<T>, grid, dim3(kEwThreads), 0, st, n, Q, ldq, sQ, s, sS, W, ldw, sW);
  MSQRT_LAUNCH_CHECK();
}
template void launch_scale_cols<float>(hipStream_t, int, const float*, int64_t, int64_t,
                                       const float*, int64_t, float*, int64_t, int64_t, int);
template void launch_scale_cols<double>(hipStream_t, int, const double*, int64_t, int64_t,
                                        const double*, int64_t, double*, int64_t, int64_t, int);

void launch_scale_inplace(hipStream_t st, int n, double* X, int64_t ldx, int64_t sX,
                          const double* scale, int batch) {
  if (n <= 0) return;
  dim3 grid((unsigned)ceil_div(n, kEwThreads), n, batch);
  hipLaunchKernelGGL(scale_inplace_kernel, grid, dim3(kEwThreads), 0, st, n, X, ldx, sX, scale);
  MSQRT_LAUNCH_CHECK();
}

}  // namespace msqrt
