// VALU issue-rate probe for the MI355X vector ALUs (not part of the library).
//
// Each thread runs NCH independent chains of one instruction form for `iters`
// iterations; a launch holds 256 * W workgroups of 4 waves, so W waves per
// SIMD.  The rate printed is wave instructions per CU per clock at the
// 2.4 GHz peak engine clock, from HIP events around one launch.  It separates
// forms whose operands are all vector registers from forms that read one
// scalar register (a wave-uniform kernel argument), which issue slower.
//
// Build and run:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       paper_2605_04497_amd/csrc/probes/valu_issue.hip -o /tmp/valu_issue && /tmp/valu_issue
// `/tmp/valu_issue FORM W` runs one case (FORM one of the names printed, FP32),
// so that a counter run (rocprofv3 --pmc) covers a known instruction count:
// two launches, of 16 and 20 000 iterations, each of 16 chains on 4 W waves
// per CU.
//
// Memory: every thread writes out[blockIdx.x * 256 + threadIdx.x] once, and
// thread 0 of each workgroup nothing else; the largest grid is kMaxBlocks
// workgroups, the size of `out`.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

constexpr int kMaxWavesPerSimd = 16;
constexpr int kCUs = 256;
constexpr int kMaxBlocks = kCUs * kMaxWavesPerSimd;

__device__ __forceinline__ float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }

enum Form {
  kFmaShared,   // a = fma(a, v, u): v, u vector registers shared by the chains
  kMulChain,    // a = a * w_i: a vector register per chain
  kFmaDot,      // a = fma(w_i, v, a): the accumulate form of a dot product
  kCmpSel,      // a = a > u ? a * v : a + u (compare, multiply, add, select)
  kFmaScalar,   // a = fma(a, s, u): s a scalar register (kernel argument)
  kMulScalar,   // a = a * s
  kFmaLiteral,  // a = fma(a, K, u): K a literal constant in the instruction
  kMulLiteral,  // a = a * K
};

template <typename T, int NCH, int FORM>
__global__ __launch_bounds__(256) void probe(T* out, int iters, float sb, float sc, double sd) {
  T a[NCH], w[NCH];
  const T v = (T)sb + (T)threadIdx.x * (T)1e-9;
  const T u = (T)sc + (T)threadIdx.x * (T)1e-9;
  const T s = sizeof(T) == 8 ? (T)sd : (T)sb;  // a kernel argument: a scalar register
#pragma unroll
  for (int i = 0; i < NCH; ++i) {
    a[i] = (T)threadIdx.x * (T)1e-3 + (T)i;
    w[i] = v + (T)i * (T)1e-7;
  }
#pragma unroll 4
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NCH; ++i) {
      if (FORM == kFmaShared) a[i] = fm(a[i], v, u);
      else if (FORM == kMulChain) a[i] = a[i] * w[i];
      else if (FORM == kFmaDot) a[i] = fm(w[i], v, a[i]);
      else if (FORM == kCmpSel) a[i] = (a[i] > u) ? a[i] * v : a[i] + u;
      else if (FORM == kFmaScalar) a[i] = fm(a[i], s, u);
      else if (FORM == kMulScalar) a[i] = a[i] * s;
      else if (FORM == kFmaLiteral) a[i] = fm(a[i], (T)0.7853981, u);
      else a[i] = a[i] * (T)0.7853981;
    }
  }
  T r = 0;
#pragma unroll
  for (int i = 0; i < NCH; ++i) r += a[i];
  out[blockIdx.x * 256 + threadIdx.x] = r;
}

template <typename T, int NCH, int FORM>
void run(const char* name, int waves_per_simd, void* out, int instr_per_step) {
  const int blocks = kCUs * waves_per_simd;
  const int iters = 20000;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hipLaunchKernelGGL((probe<T, NCH, FORM>), dim3(blocks), dim3(256), 0, 0, (T*)out, 16, 0.999f,
                     1e-4f, 0.999);
  (void)hipEventRecord(e0);
  hipLaunchKernelGGL((probe<T, NCH, FORM>), dim3(blocks), dim3(256), 0, 0, (T*)out, iters,
                     0.999f, 1e-4f, 0.999);
  (void)hipEventRecord(e1);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  const double wave_instr = (double)blocks * 4 * iters * NCH * instr_per_step;
  const double cu_clocks = kCUs * 2.4e9 * ms * 1e-3;
  printf("%-11s %s chains=%2d waves/SIMD=%2d: %7.3f ms, %.3f wave instructions per CU-clock\n",
         name, sizeof(T) == 4 ? "f32" : "f64", NCH, waves_per_simd, ms, wave_instr / cu_clocks);
  fflush(stdout);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace

int main(int argc, char** argv) {
  void* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * kMaxBlocks * 256) != hipSuccess) return 1;
  if (argc == 3) {
    const int w = atoi(argv[2]);
    if (w < 1 || w > kMaxWavesPerSimd) {
      fprintf(stderr, "W must be 1..%d\n", kMaxWavesPerSimd);
      return 2;
    }
    const char* f = argv[1];
    if (!strcmp(f, "fma")) run<float, 16, kFmaShared>("fma", w, out, 1);
    else if (!strcmp(f, "mul")) run<float, 16, kMulChain>("mul", w, out, 1);
    else if (!strcmp(f, "fma-dot")) run<float, 16, kFmaDot>("fma-dot", w, out, 1);
    else if (!strcmp(f, "cmp-select")) run<float, 16, kCmpSel>("cmp-select", w, out, 4);
    else if (!strcmp(f, "fma-sgpr")) run<float, 16, kFmaScalar>("fma-sgpr", w, out, 1);
    else if (!strcmp(f, "mul-sgpr")) run<float, 16, kMulScalar>("mul-sgpr", w, out, 1);
    else if (!strcmp(f, "fma-literal")) run<float, 16, kFmaLiteral>("fma-literal", w, out, 1);
    else if (!strcmp(f, "mul-literal")) run<float, 16, kMulLiteral>("mul-literal", w, out, 1);
    else {
      fprintf(stderr, "unknown form %s\n", f);
      return 2;
    }
    (void)hipFree(out);
    return 0;
  }
  for (int w : {4, 8, 16}) run<float, 16, kFmaShared>("fma", w, out, 1);
  for (int w : {4, 8, 16}) run<float, 16, kMulChain>("mul", w, out, 1);
  for (int w : {4, 8, 16}) run<float, 16, kFmaDot>("fma-dot", w, out, 1);
  for (int w : {4, 8}) run<float, 16, kCmpSel>("cmp-select", w, out, 4);
  for (int w : {4, 8, 16}) run<float, 16, kFmaScalar>("fma-sgpr", w, out, 1);
  for (int w : {4, 8, 16}) run<float, 16, kMulScalar>("mul-sgpr", w, out, 1);
  for (int w : {4, 8, 16}) run<float, 16, kFmaLiteral>("fma-literal", w, out, 1);
  for (int w : {4, 8, 16}) run<float, 16, kMulLiteral>("mul-literal", w, out, 1);
  for (int w : {4, 8}) run<double, 8, kFmaShared>("fma", w, out, 1);
  for (int w : {4, 8}) run<double, 8, kMulChain>("mul", w, out, 1);
  for (int w : {4, 8}) run<double, 8, kFmaScalar>("fma-sgpr", w, out, 1);
  for (int w : {4, 8}) run<double, 8, kMulScalar>("mul-sgpr", w, out, 1);
  (void)hipFree(out);
  return 0;
}
