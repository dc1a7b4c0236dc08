// Pairwise Shapley interaction indices (Theorem 1 with |S| = 2, Eq. 9-10,
// 8 nodes) and first-order values, per sample.
//
// For a path P with unique features j, factors F_j(m) = b_j + t_m c_j
// (c_j = o_j - b_j), H(m) = prod_j F_j(m):
//   SII_ik += val c_i c_k sum_m w_m prod_{j != i,k} F_j(m)
//          =  sum_m g_i(m) r_k(m),   r_k = c_k / F_k,  g_i = w val H r_i
//   phi_i  += sum_m g_i(m)
// F_j(m) = 0 happens only when b_j = 0 and o_j = 0; then every product that
// excludes j still contains F_j = 0 and every term with j in S has c_j = 0, so
// the whole path contributes exactly zero: such lanes are masked (their zero
// factor is replaced by 1 to keep the reciprocals finite).
//
// Work mapping (gfx950, wave64): a workgroup owns one explained sample and a
// chunk of paths of one capacity class; each lane takes one path (the table
// is slot-major, so a wave's 64 paths load coalesced).  The sample's pair
// triangle (pair i < k at k(k-1)/2 + i; features are sorted inside a path, so
// f_i < f_k) and its phi row accumulate in LDS with atomics, then flush to the
// FP64 global accumulators: the sum within a chunk of at most 64k paths is in
// the kernel precision, the sum across chunks in FP64.  When the FP64 triangle
// does not fit in LDS (TRI_LDS = false) pairs go straight to the global FP64
// triangle.  NH < 8 splits the nodes over passes to bound the registers held
// by r (the node sum is additive).
#include <hip/hip_runtime.h>

#include "../qts_device.h"

namespace qts {

namespace {

template <typename T>
__device__ __forceinline__ T fmaP(T a, T b, T c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaP<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

__device__ __forceinline__ float rcpP(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpP(double x) { return 1.0 / x; }

}  // namespace

template <typename T, int C, int NH, bool TRI_LDS>
__global__ void __launch_bounds__(512)
pairs_kernel(const int32_t* __restrict__ pd, const int32_t* __restrict__ pleaf,
             const int32_t* __restrict__ feat, const float* __restrict__ lo,
             const float* __restrict__ hi, const T* __restrict__ bb, const T* __restrict__ cbb,
             int32_t np, int32_t chunk, const double* __restrict__ leaf_val,
             const float* __restrict__ X, int64_t M, int64_t ldx, int32_t F,
             double* __restrict__ tri64, double* __restrict__ phi64, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t ntri = (int64_t)F * (F - 1) / 2;
  T* phis = reinterpret_cast<T*>(smem);                 // [F]
  T* tris = phis + F;                                   // [ntri] when TRI_LDS
  float* xrow = reinterpret_cast<float*>(tris + (TRI_LDS ? ntri : 0));  // [F]

  const int64_t s = (int64_t)blockIdx.x % M;
  const int ch = (int)((int64_t)blockIdx.x / M);
  const int p0 = ch * chunk;
  const int p1 = min(np, p0 + chunk);

  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    xrow[i] = X[s * ldx + i];
    phis[i] = T(0);
  }
  if (TRI_LDS)
    for (int64_t e = threadIdx.x; e < ntri; e += blockDim.x) tris[e] = T(0);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  for (int base = p0 + wave * 64; base < p1; base += nw * 64) {
    const int p = base + lane;
    const bool valid = p < p1;
    const int pc = valid ? p : p1 - 1;  // clamped index for the loads
    const int d = valid ? pd[pc] : 0;
    T val = valid ? (T)leaf_val[pleaf[pc]] : T(0);

#pragma unroll
    for (int pass = 0; pass < kNodes / NH; ++pass) {
      const int m0 = pass * NH;
      T H[NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) H[m] = T(1);
      T r[C][NH];
      int rb[C];
      bool dead = false;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int64_t e = (int64_t)j * np + pc;
        const int fm = feat[e];
        const int f = fm & kFeatureMask;
        const float x = xrow[f];
        const bool miss = (fm & kMissingOkBit) != 0;
        const bool lower = miss ? !(x < lo[e]) : (x >= lo[e]);
        const bool upper = !(x >= hi[e]);
        const T b = bb[e];
        const T c = (lower & upper) ? cbb[e] : -b;
        const bool z = (b == T(0)) & (c == T(0));
        dead |= z;
        const T bz = z ? T(1) : b;
        rb[j] = (f * (f - 1)) >> 1;
#pragma unroll
        for (int m = 0; m < NH; ++m) {
          const T Fv = fmaP(nc.t[m0 + m], c, bz);
          H[m] *= Fv;
          r[j][m] = c * rcpP(Fv);
        }
      }
      if (dead) val = T(0);
      T G[NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) G[m] = nc.w[m0 + m] * val * H[m];
      const bool live = val != T(0);

#pragma unroll
      for (int i = 0; i < C; ++i) {
        if (i < d) {
          T g[NH];
          T ph = T(0);
#pragma unroll
          for (int m = 0; m < NH; ++m) {
            g[m] = G[m] * r[i][m];
            ph += g[m];
          }
          const int fi = feat[(int64_t)i * np + pc] & kFeatureMask;
          if (live)
            __hip_atomic_fetch_add(&phis[fi], ph, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          // pairs (i, k > i) in groups of four: the four values are computed
          // into separate registers before their atomics issue, so the LDS
          // queue sees back-to-back atomics instead of one per dependency
          // chain (inert slots k >= d have r = 0 and are not stored)
#pragma unroll
          for (int kb = i + 1; kb < C; kb += 4) {
            T pr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k = kb + u;
              if (k < C) {
                pr[u] = g[0] * r[k < C ? k : 0][0];
#pragma unroll
                for (int m = 1; m < NH; ++m) pr[u] = fmaP(g[m], r[k < C ? k : 0][m], pr[u]);
              }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k = kb + u;
              if (k < C && k < d && live) {
                if (TRI_LDS)
                  __hip_atomic_fetch_add(&tris[rb[k < C ? k : 0] + fi], pr[u], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                else
                  unsafeAtomicAdd(&tri64[s * ntri + rb[k < C ? k : 0] + fi], (double)pr[u]);
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();

  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    const T v = phis[i];
    if (v != T(0)) unsafeAtomicAdd(&phi64[s * F + i], (double)v);
  }
  if (TRI_LDS) {
    for (int64_t e = threadIdx.x; e < ntri; e += blockDim.x) {
      const T v = tris[e];
      if (v != T(0)) unsafeAtomicAdd(&tri64[s * ntri + e], (double)v);
    }
  }
}

// Generic form for long paths (any capacity up to 64): one wavefront per
// path.  Lane j owns slot j (o_j, c_j, F_j(m), r_j(m) = c_j / F_j(m)); the
// node products H(m) are reduced across lanes; then the wave's lanes take the
// d(d-1)/2 pairs of the path in turn, reading r from a per-wave LDS area.
template <typename T, bool TRI_LDS>
__global__ void __launch_bounds__(256)
pairs_generic_kernel(const int32_t* __restrict__ pd, const int32_t* __restrict__ pleaf,
                     const int32_t* __restrict__ feat, const float* __restrict__ lo,
                     const float* __restrict__ hi, const T* __restrict__ bb,
                     const T* __restrict__ cbb, int32_t np, int32_t chunk,
                     const double* __restrict__ leaf_val, const float* __restrict__ X, int64_t M,
                     int64_t ldx, int32_t F, double* __restrict__ tri64,
                     double* __restrict__ phi64, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t ntri = (int64_t)F * (F - 1) / 2;
  const int nw = blockDim.x >> 6;
  T* phis = reinterpret_cast<T*>(smem);                     // [F]
  T* tris = phis + F;                                       // [ntri] when TRI_LDS
  T* rall = tris + (TRI_LDS ? ntri : 0);                    // [nw][64][8]
  int* fall = reinterpret_cast<int*>(rall + (size_t)nw * 64 * kNodes);  // [nw][64]
  float* xrow = reinterpret_cast<float*>(fall + nw * 64);   // [F]

  const int64_t s = (int64_t)blockIdx.x % M;
  const int ch = (int)((int64_t)blockIdx.x / M);
  const int p0 = ch * chunk;
  const int p1 = min(np, p0 + chunk);
  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    xrow[i] = X[s * ldx + i];
    phis[i] = T(0);
  }
  if (TRI_LDS)
    for (int64_t e = threadIdx.x; e < ntri; e += blockDim.x) tris[e] = T(0);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  T* rw = rall + (size_t)wave * 64 * kNodes;
  int* fw = fall + wave * 64;
  for (int p = p0 + wave; p < p1; p += nw) {
    const int d = pd[p];
    const T val = (T)leaf_val[pleaf[p]];
    T Fv[kNodes];
    bool z = false;
    if (lane < d) {
      const int64_t e = (int64_t)lane * np + p;
      const int fm = feat[e];
      const int f = fm & kFeatureMask;
      const float x = xrow[f];
      const bool miss = (fm & kMissingOkBit) != 0;
      const bool lower = miss ? !(x < lo[e]) : (x >= lo[e]);
      const bool upper = !(x >= hi[e]);
      const T b = bb[e];
      const T c = (lower & upper) ? cbb[e] : -b;
      z = (b == T(0)) & (c == T(0));
      const T bz = z ? T(1) : b;
#pragma unroll
      for (int m = 0; m < kNodes; ++m) {
        Fv[m] = fmaP(nc.t[m], c, bz);
        rw[lane * kNodes + m] = c * rcpP(Fv[m]);
      }
      fw[lane] = f;
    } else {
#pragma unroll
      for (int m = 0; m < kNodes; ++m) Fv[m] = T(1);
    }
    // a factor that vanishes at every node zeroes the whole path
    if (__any(z) || val == T(0)) continue;
    // H(m) = prod over the lanes' factors (butterfly product)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int m = 0; m < kNodes; ++m) Fv[m] *= __shfl_xor(Fv[m], off, 64);
    T G[kNodes];
#pragma unroll
    for (int m = 0; m < kNodes; ++m) G[m] = nc.w[m] * val * Fv[m];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < d) {
      T ph = T(0);
#pragma unroll
      for (int m = 0; m < kNodes; ++m) ph = fmaP(G[m], rw[lane * kNodes + m], ph);
      __hip_atomic_fetch_add(&phis[fw[lane]], ph, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    const int npair = d * (d - 1) / 2;
    for (int q = lane; q < npair; q += 64) {
      // pair q -> (i < k): k(k-1)/2 <= q < k(k+1)/2
      int k = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
      while (k * (k - 1) / 2 > q) --k;
      while ((k + 1) * k / 2 <= q) ++k;
      const int i = q - k * (k - 1) / 2;
      T pr = T(0);
#pragma unroll
      for (int m = 0; m < kNodes; ++m)
        pr = fmaP(G[m] * rw[i * kNodes + m], rw[k * kNodes + m], pr);
      const int fi = fw[i], fk = fw[k];
      const int64_t idx = (int64_t)fk * (fk - 1) / 2 + fi;
      if (TRI_LDS)
        __hip_atomic_fetch_add(&tris[idx], pr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        unsafeAtomicAdd(&tri64[s * ntri + idx], (double)pr);
    }
    // the next path overwrites this wave's r and feature slots
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();

  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    const T v = phis[i];
    if (v != T(0)) unsafeAtomicAdd(&phi64[s * F + i], (double)v);
  }
  if (TRI_LDS) {
    for (int64_t e = threadIdx.x; e < ntri; e += blockDim.x) {
      const T v = tris[e];
      if (v != T(0)) unsafeAtomicAdd(&tri64[s * ntri + e], (double)v);
    }
  }
}

// Phi[s] from the FP64 accumulators: off-diagonal SII/2, diagonal
// phi_i - sum_{k != i} Phi[i][k] (rows sum to phi).
template <typename TO>
__global__ void __launch_bounds__(256)
pairs_finalize_kernel(const double* __restrict__ tri64, const double* __restrict__ phi64,
                      int64_t M, int32_t F, TO* __restrict__ Phi, TO* __restrict__ phi_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* rows = reinterpret_cast<double*>(smem);  // [F]
  const int64_t ntri = (int64_t)F * (F - 1) / 2;
  for (int64_t s = blockIdx.x; s < M; s += gridDim.x) {
    const double* t = tri64 + s * ntri;
    for (int i = threadIdx.x; i < F; i += blockDim.x) {
      double sum = 0.0;
      const int64_t ri = (int64_t)i * (i - 1) / 2;
      for (int k = 0; k < i; ++k) sum += t[ri + k];
      for (int k = i + 1; k < F; ++k) sum += t[(int64_t)k * (k - 1) / 2 + i];
      rows[i] = sum;
    }
    __syncthreads();
    const int64_t FF = (int64_t)F * F;
    for (int64_t e = threadIdx.x; e < FF; e += blockDim.x) {
      const int i = (int)(e / F);
      const int k = (int)(e - (int64_t)i * F);
      double v;
      if (i == k) {
        v = phi64[s * F + i] - 0.5 * rows[i];
      } else {
        const int a = i < k ? i : k, b = i < k ? k : i;
        v = 0.5 * t[(int64_t)b * (b - 1) / 2 + a];
      }
      Phi[s * FF + e] = (TO)v;
    }
    if (phi_out)
      for (int i = threadIdx.x; i < F; i += blockDim.x) phi_out[s * F + i] = (TO)phi64[s * F + i];
    __syncthreads();
  }
}

namespace {

size_t pairs_lds_bytes(int F, size_t tsize, bool tri_lds) {
  const size_t ntri = (size_t)F * (F - 1) / 2;
  return (size_t)F * tsize + (tri_lds ? ntri * tsize : 0) + (size_t)F * sizeof(float);
}

constexpr int kGenericThreads = 256;

size_t generic_lds_bytes(int F, size_t tsize, bool tri_lds) {
  const int nw = kGenericThreads / 64;
  return pairs_lds_bytes(F, tsize, tri_lds) + (size_t)nw * 64 * kNodes * tsize +
         (size_t)nw * 64 * sizeof(int);
}

int pair_chunk(int np, int64_t M, int64_t* n_chunks_out) {
  // chunks: at most 64k paths (bounds the in-kernel precision sum), and
  // enough work items to fill the chip when there are few samples
  int64_t n_chunks = (np + 65535) / 65536;
  const int64_t fill = (2048 + M - 1) / M;
  n_chunks = std::max<int64_t>(n_chunks, std::min<int64_t>(fill, (np + 1023) / 1024));
  n_chunks = std::max<int64_t>(1, n_chunks);
  *n_chunks_out = n_chunks;
  return (int)((np + n_chunks - 1) / n_chunks);
}

// Raise a kernel's dynamic-LDS limit once; returns the usable bytes.
size_t lds_limit_of(const void* fn, size_t* cache) {
  if (*cache == 0) {
    hipFuncAttributes fa;
    check_hip(hipFuncGetAttributes(&fa, fn), "hipFuncGetAttributes");
    const size_t limit = (size_t)kMaxLdsBytes - fa.sharedSizeBytes;
    check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)limit),
              "hipFuncSetAttribute");
    *cache = limit;
  }
  return *cache;
}

template <typename T>
const T* table_b(const DeviceTable& d) {
  return std::is_same<T, float>::value ? (const T*)d.pr_b32 : (const T*)d.pr_b64;
}
template <typename T>
const T* table_cb(const DeviceTable& d) {
  return std::is_same<T, float>::value ? (const T*)d.pr_cb32 : (const T*)d.pr_cb64;
}
template <typename T>
NodeConsts<T> node_consts(const DeviceTable& d) {
  if constexpr (std::is_same<T, float>::value) return d.n32; else return d.n64;
}

template <typename T, int C, int NH>
void launch_pairs_fast(const HostTable& h, const DeviceTable& d, const PairClass& pc,
                       const float* X, int64_t M, int64_t ldx, const double* leaf_val,
                       double* tri64, double* phi64, hipStream_t s) {
  const int F = h.F;
  int64_t n_chunks = 1;
  const int chunk = pair_chunk(pc.np, M, &n_chunks);
  const int64_t grid = M * n_chunks;
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "interactions grid too large");
  static size_t cache = 0;
  const size_t lds = pairs_lds_bytes(F, sizeof(T), true);
  if (lds > lds_limit_of((const void*)pairs_kernel<T, C, NH, true>, &cache))
    fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
  hipLaunchKernelGGL((pairs_kernel<T, C, NH, true>), dim3((unsigned)grid), dim3(512), lds, s,
                     d.pr_d + pc.pbase, d.pr_leaf + pc.pbase, d.pr_feat + pc.base,
                     d.pr_lo + pc.base, d.pr_hi + pc.base, table_b<T>(d) + pc.base,
                     table_cb<T>(d) + pc.base, pc.np, chunk, leaf_val, X, M, ldx, F, tri64, phi64,
                     node_consts<T>(d));
  check_hip(hipGetLastError(), "pairs_kernel launch");
}

template <typename T, bool TRI>
void launch_pairs_generic(const HostTable& h, const DeviceTable& d, const PairClass& pc,
                          const float* X, int64_t M, int64_t ldx, const double* leaf_val,
                          double* tri64, double* phi64, hipStream_t s) {
  const int F = h.F;
  int64_t n_chunks = 1;
  const int chunk = pair_chunk(pc.np, M, &n_chunks);
  const int64_t grid = M * n_chunks;
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "interactions grid too large");
  static size_t cache = 0;
  const size_t lds = generic_lds_bytes(F, sizeof(T), TRI);
  if (lds > lds_limit_of((const void*)pairs_generic_kernel<T, TRI>, &cache))
    fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
  hipLaunchKernelGGL((pairs_generic_kernel<T, TRI>), dim3((unsigned)grid),
                     dim3(kGenericThreads), lds, s, d.pr_d + pc.pbase, d.pr_leaf + pc.pbase,
                     d.pr_feat + pc.base, d.pr_lo + pc.base, d.pr_hi + pc.base,
                     table_b<T>(d) + pc.base, table_cb<T>(d) + pc.base, pc.np, chunk, leaf_val,
                     X, M, ldx, F, tri64, phi64, node_consts<T>(d));
  check_hip(hipGetLastError(), "pairs_generic_kernel launch");
}

}  // namespace

void launch_pairs(const HostTable& h, const DeviceTable& d, const PairClass& pc, bool fp64,
                  const float* X, int64_t M, int64_t ldx, const double* lv, double* tri64,
                  double* phi64, hipStream_t s) {
  // register-resident lane-per-path instances exist where they do not spill
  if (!fp64) {
    switch (pc.cap) {
      case 4: return launch_pairs_fast<float, 4, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      case 8: return launch_pairs_fast<float, 8, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      case 12: return launch_pairs_fast<float, 12, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      case 16: return launch_pairs_fast<float, 16, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      case 20: return launch_pairs_fast<float, 20, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      case 24: return launch_pairs_fast<float, 24, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      default: break;
    }
    if (generic_lds_bytes(h.F, sizeof(float), true) > (size_t)kMaxLdsBytes - 1024)
      fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
    return launch_pairs_generic<float, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
  }
  if (pairs_lds_bytes(h.F, sizeof(double), true) <= (size_t)kMaxLdsBytes - 1024) {
    switch (pc.cap) {
      case 4: return launch_pairs_fast<double, 4, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      case 8: return launch_pairs_fast<double, 8, 8>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
      default: break;
    }
  }
  if (generic_lds_bytes(h.F, sizeof(double), true) <= (size_t)kMaxLdsBytes - 1024)
    launch_pairs_generic<double, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
  else
    launch_pairs_generic<double, false>(h, d, pc, X, M, ldx, lv, tri64, phi64, s);
}

void launch_pairs_finalize(const double* tri64, const double* phi64, int64_t M, int F, bool fp64,
                           void* Phi, void* phi, hipStream_t s) {
  if (M <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(M, 8192);
  const size_t lds = (size_t)F * sizeof(double);
  if (fp64)
    hipLaunchKernelGGL(pairs_finalize_kernel<double>, dim3(grid), dim3(256), lds, s, tri64, phi64,
                       M, F, (double*)Phi, (double*)phi);
  else
    hipLaunchKernelGGL(pairs_finalize_kernel<float>, dim3(grid), dim3(256), lds, s, tri64, phi64,
                       M, F, (float*)Phi, (float*)phi);
  check_hip(hipGetLastError(), "pairs_finalize launch");
}

}  // namespace qts
