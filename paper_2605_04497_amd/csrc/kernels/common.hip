// Small element-wise kernels: zero fill (used instead of hipMemsetAsync so
// the call sequence stays safe to capture in a HIP graph) and FP64 -> FP32.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "../qts_device.h"

namespace qts {

size_t raise_lds_limit(const void* fn) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> done;
  int dev = 0;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(fn, dev);
  const auto it = done.find(key);
  if (it != done.end()) return it->second;
  hipFuncAttributes fa;
  check_hip(hipFuncGetAttributes(&fa, fn), "hipFuncGetAttributes");
  const size_t limit = (size_t)kMaxLdsBytes - fa.sharedSizeBytes;
  check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)limit),
            "hipFuncSetAttribute");
  done.emplace(key, limit);
  return limit;
}

__global__ void __launch_bounds__(256) fill_zero_kernel(double* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

__global__ void __launch_bounds__(256) cast_kernel(const double* __restrict__ src,
                                                   float* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = (float)src[i];
}

// Counter-based hash (the "lowbias32" integer mixer) to uniform floats.
__global__ void __launch_bounds__(256) fill_uniform_kernel(float* __restrict__ p, int64_t n,
                                                           uint32_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint32_t x = (uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u ^ seed;
    x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
    p[i] = -3.0f + 6.0f * (float)(x >> 8) * (1.0f / 16777216.0f);
  }
}

__global__ void __launch_bounds__(256) widen_kernel(const float* __restrict__ src,
                                                    double* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = (double)src[i];
}

// out[i] = sum over r = 0, 1, ..., nrows - 1 of part[r * n + i], added in that
// order (a reduction whose result does not depend on scheduling).
__global__ void __launch_bounds__(256) sum_rows_kernel(const double* __restrict__ part,
                                                       int64_t nrows, int64_t n,
                                                       double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double acc = 0.0;
    for (int64_t r = 0; r < nrows; ++r) acc += part[r * n + i];
    out[i] = acc;
  }
}

static unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

void launch_fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n);
  check_hip(hipGetLastError(), "fill_zero launch");
}

void launch_fill_uniform(float* p, int64_t n, uint32_t seed, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_uniform_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, seed);
  check_hip(hipGetLastError(), "fill_uniform launch");
}

void launch_widen_f32_f64(const float* src, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(widen_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  check_hip(hipGetLastError(), "widen launch");
}

void launch_sum_rows(const double* part, int64_t nrows, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(sum_rows_kernel, dim3(grid_for(n)), dim3(256), 0, s, part, nrows, n, out);
  check_hip(hipGetLastError(), "sum_rows launch");
}

void launch_cast_f64_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cast_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  check_hip(hipGetLastError(), "cast launch");
}

}  // namespace qts
