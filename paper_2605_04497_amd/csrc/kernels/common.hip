// Small element-wise kernels: zero fill (used instead of hipMemsetAsync so
// the call sequence stays safe to capture in a HIP graph), FP64 -> FP32, and
// tiled transposes (the feature-major layouts of wide feature spaces).
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

// dst[b][c][r] = src[b][r][c] for r < R, c < C (row strides lds, ldd; batch
// strides sbs, dbs): 32 x 32 tiles through LDS, so both the reads and the
// writes are coalesced.
template <typename Ti, typename To>
__global__ void __launch_bounds__(256)
transpose_kernel(const Ti* __restrict__ src, int64_t R, int64_t C, int64_t lds, int64_t sbs,
                 To* __restrict__ dst, int64_t ldd, int64_t dbs, int64_t tiles_c) {
  __shared__ Ti tile[32][33];
  const int64_t t = blockIdx.x;
  const int64_t r0 = (t / tiles_c) * 32, c0 = (t % tiles_c) * 32;
  const Ti* sp = src + (int64_t)blockIdx.y * sbs;
  To* dp = dst + (int64_t)blockIdx.y * dbs;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + j, c = c0 + tx;
    if (r < R && c < C) tile[j][tx] = sp[r * lds + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t c = c0 + j, r = r0 + tx;
    if (r < R && c < C) dp[c * ldd + r] = (To)tile[tx][j];
  }
}

template <typename Ti, typename To>
static void transpose_t(const Ti* src, int64_t R, int64_t C, int64_t lds, int64_t sbs, To* dst,
                        int64_t ldd, int64_t dbs, int32_t nbatch, hipStream_t s) {
  if (R <= 0 || C <= 0 || nbatch <= 0) return;
  const int64_t tiles_c = (C + 31) / 32;
  const int64_t tiles = ((R + 31) / 32) * tiles_c;
  if (tiles > 0x7fffffff || nbatch > 65535) fail(QTS_E_UNSUPPORTED, "transpose too large");
  hipLaunchKernelGGL((transpose_kernel<Ti, To>), dim3((unsigned)tiles, (unsigned)nbatch),
                     dim3(256), 0, s, src, R, C, lds, sbs, dst, ldd, dbs, tiles_c);
  check_hip(hipGetLastError(), "transpose launch");
}

void launch_transpose(const float* src, int64_t R, int64_t C, int64_t lds, int64_t sbs,
                      float* dst, int64_t ldd, int64_t dbs, int32_t nbatch, hipStream_t s) {
  transpose_t(src, R, C, lds, sbs, dst, ldd, dbs, nbatch, s);
}
void launch_transpose(const double* src, int64_t R, int64_t C, int64_t lds, int64_t sbs,
                      double* dst, int64_t ldd, int64_t dbs, int32_t nbatch, hipStream_t s) {
  transpose_t(src, R, C, lds, sbs, dst, ldd, dbs, nbatch, s);
}
void launch_transpose(const double* src, int64_t R, int64_t C, int64_t lds, int64_t sbs,
                      float* dst, int64_t ldd, int64_t dbs, int32_t nbatch, hipStream_t s) {
  transpose_t(src, R, C, lds, sbs, dst, ldd, dbs, nbatch, s);
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
