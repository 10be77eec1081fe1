// Shared device/host helpers for the msqrt HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace msqrt {

constexpr int kWave = 64;

// Error raised by host code; converted to a status at the C-ABI boundary.
struct Error {
  int status;
  std::string msg;
};

void set_last_error(const std::string& msg);

#define MSQRT_HIP(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::msqrt::Error{6, std::string(#call) + ": " + hipGetErrorString(e_) + " at " \
                                  + __FILE__ + ":" + std::to_string(__LINE__)};          \
  } while (0)

#define MSQRT_LAUNCH_CHECK() MSQRT_HIP(hipGetLastError())

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Device-side reductions

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    T o = __shfl_xor(v, off, kWave);
    v = v > o ? v : o;
  }
  return v;
}

// Block-wide sum for blockDim.x a multiple of 64 (<= 1024).  All threads get
// the result.  `sh` must hold blockDim.x/64 elements.
template <typename T>
__device__ inline T block_sum(T v, T* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  return r;
}

template <typename T>
__device__ inline T block_max(T v, T* sh) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  T r = sh[0];
  for (int i = 1; i < nw; ++i) r = r > sh[i] ? r : sh[i];
  return r;
}

}  // namespace msqrt
