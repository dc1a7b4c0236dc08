// Depth-first form of the pairwise interactions (section 5, Algorithm 1 at
// order 2, with Eq. 11's telescoping update for repeated features); the
// notation and the formulas are those of DfsTable (qts_internal.h).
//
// dfs_walk_kernel: the tree walk.  A wavefront walks one tree for 8 samples,
// lane = (sample, node m), so the walk is uniform across the wave; the node
// records of each window of 64 events are staged in LDS by one coalesced load
// and read back by broadcast.  Each lane carries the product C of
// the factors of the features split above the current node at t_m, kept on
// a per-level stack in LDS while a subtree is walked, and returns up the tree
// H_u(t_m), the sum of val * C over the leaves below u.  At each internal
// node it stores y_v(t_m) = w_m sum_u H_u (r_f^u - r_f^v)(t_m) for the pair
// pass.  Entering child u multiplies C by F_f^u / F_f^v (a division only when
// f was split above); a factor that vanishes identically (b = o = 0) makes
// the subtree's polynomials zero, and the guards keep its terms exactly zero.
//
// dfs_pairs_kernel: the pair pass.  A workgroup owns one sample (its pair
// triangle and phi row in LDS, FP64, as in the path form); lane = internal
// node (rows sorted by length in tiles of 64, slot-major inside a tile).  A
// row adds phi_f += sum_m y_v(m) and, for every feature j split above v,
// SII_fj += c_j sum_m y_v(m) / F_j(t_m): one update per (node, feature).
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>
#include <vector>

#include "../qts_device.h"

namespace qts {

namespace {

template <typename T>
__device__ __forceinline__ T fmaD(T a, T b, T c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaD<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

__device__ __forceinline__ float rcpD(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64: the hardware estimate and two Newton steps (see the pairs kernel).
__device__ __forceinline__ double rcpD(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// x follows the splits of an interval [lo, hi) (hi NaN: no upper bound); a
// NaN x follows them iff mok.
__device__ __forceinline__ bool follows(float x, float lo, float hi, bool mok) {
  const bool lower = mok ? !(x < lo) : (x >= lo);
  return lower & !(x >= hi);
}

}  // namespace

constexpr int kDfsSamples = 8;  // samples per wavefront of the walk (8 lanes each)

// LDS of the walk: the sample rows of the workgroup's 8 samples (stride F+1),
// then per wave the two stacks [level][64] of C and of the left subtree's H
// and the stage of 64 events' node data.
__host__ __device__ inline size_t staged_event_bytes(size_t tsize) {
  return ((4 * sizeof(int32_t) + (kDfsCoef + 2) * tsize) + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t dfs_wave_lds(int levels, size_t tsize) {
  return (((size_t)2 * levels * 64 * tsize + 15) & ~(size_t)15) + 64 * staged_event_bytes(tsize);
}
__host__ __device__ inline size_t dfs_walk_lds(int F, int levels, int waves, size_t tsize) {
  const size_t xs = (((size_t)kDfsSamples * (F + 1) * sizeof(float)) + 15) & ~(size_t)15;
  return xs + (size_t)waves * dfs_wave_lds(levels, tsize);
}

// Lane k's value, wave-uniform.
__device__ __forceinline__ int bcast(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float bcast(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double bcast(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One event's node data as the walk reads it back from LDS (wave-uniform
// address: a broadcast), 16-byte aligned.
template <typename T>
struct alignas(16) StagedEvent {
  int32_t kind, level, flags, row;
  T coef[kDfsCoef];  // b^v, 1 - b^v, b^L, 1 - b^L, b^R, 1 - b^R, b^v - b^L, b^v - b^R
  T lv[2];           // values of leaf children (0 for internal ones)
};

template <typename T>
__global__ void __launch_bounds__(1024)
dfs_walk_kernel(const DfsNode* __restrict__ nodes, const T* __restrict__ coef,
                const T* __restrict__ lvals, const int32_t* __restrict__ events,
                const int32_t* __restrict__ tree_first, const int32_t* __restrict__ tree_nodes,
                int32_t n_trees, const float* __restrict__ X, int64_t s0, int32_t mb,
                int64_t ldx, int32_t F, int32_t levels, int32_t nsg, int32_t n_rows,
                T* __restrict__ Y, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int waves = blockDim.x >> 6;
  const int sg = blockIdx.x % nsg;            // group of 8 samples
  const int tb = blockIdx.x / nsg;            // block of `waves` trees
  float* xs = reinterpret_cast<float*>(smem);
  const int xstride = F + 1;
  for (int i = threadIdx.x; i < kDfsSamples * F; i += blockDim.x) {
    const int q = i / F, f = i - q * F;
    const int sl = sg * kDfsSamples + q;
    xs[q * xstride + f] = sl < mb ? X[(s0 + sl) * ldx + f] : 0.0f;
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ti = tb * waves + wave;
  if (ti >= n_trees) return;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 3, m = lane & 7;
  const int sl = sg * kDfsSamples + q;         // sample within the batch
  const bool valid = sl < mb;
  const size_t xs_bytes = (((size_t)kDfsSamples * xstride * sizeof(float)) + 15) & ~(size_t)15;
  unsigned char* wbase = smem + xs_bytes + (size_t)wave * dfs_wave_lds(levels, sizeof(T));
  T* cst = reinterpret_cast<T*>(wbase);
  T* hst = cst + (size_t)levels * 64;
  StagedEvent<T>* stage = reinterpret_cast<StagedEvent<T>*>(hst + (size_t)levels * 64);
  T tm = nc.t[0], wm = nc.w[0];
#pragma unroll
  for (int k = 1; k < kNodes; ++k) {
    tm = m == k ? nc.t[k] : tm;
    wm = m == k ? nc.w[k] : wm;
  }

  const int first = __builtin_amdgcn_readfirstlane(tree_first[ti]);
  const int n_ev = 3 * __builtin_amdgcn_readfirstlane(tree_nodes[ti]);
  const int32_t* ev = events + 3 * (size_t)first;
  T C = T(1), H = T(0);
  // Windows of 64 events.  Pass 1, lane i on event i of the window: load its
  // node data (coalesced) into the wave's LDS stage, and test the follow
  // conditions of its split feature for all 8 samples at once (3 bits per
  // sample: above the node, left edge, right edge).  Pass 2 walks the
  // window's events in order, reading each event's data back from the stage
  // (a broadcast) and its sample's bits from the event's lane.
  for (int w0 = 0; w0 < n_ev; w0 += 64) {
    const int nwin = min(64, n_ev - w0);
    {
      const int e = ev[w0 + min(lane, nwin - 1)];
      const int r = e >> 2;
      const DfsNode nd = nodes[r];
      StagedEvent<T> se;
      se.kind = e & 3;
      se.level = nd.level;
      se.flags = nd.flags;
      se.row = nd.row;
#pragma unroll
      for (int k = 0; k < kDfsCoef; ++k) se.coef[k] = coef[(size_t)r * kDfsCoef + k];
      se.lv[0] = lvals[2 * (size_t)r];
      se.lv[1] = lvals[2 * (size_t)r + 1];
      stage[lane] = se;
      uint32_t bits = 0;
#pragma unroll
      for (int qq = 0; qq < kDfsSamples; ++qq) {
        const float x = xs[qq * xstride + nd.f];
        const uint32_t b3 =
            (follows(x, nd.lo_v, nd.hi_v, (nd.flags & kDfsMokV) != 0) ? 1u : 0u) |
            (follows(x, nd.lo_l, nd.hi_l, (nd.flags & kDfsMokL) != 0) ? 2u : 0u) |
            (follows(x, nd.lo_r, nd.hi_r, (nd.flags & kDfsMokR) != 0) ? 4u : 0u);
        bits |= b3 << (3 * qq);
      }
      // the stage is written by this wave only and read back by it below
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // one step of the walk: event k of the window, its record w
      auto step = [&](const StagedEvent<T>& w, int k) __attribute__((always_inline)) {
        const int kind = __builtin_amdgcn_readfirstlane(w.kind);
        const int level = __builtin_amdgcn_readfirstlane(w.level);
        const uint32_t mine = ((uint32_t)__builtin_amdgcn_readlane((int)bits, k) >> (3 * q)) & 7u;
        const bool ov = (mine & 1u) != 0;
        const T bv = w.coef[0], cbv = w.coef[1];
        // F_f^v; where f is not split above v the record has b = 1, 1 - b = 0
        // and no bounds, so F_f^v = 1 exactly
        const T Fv = fmaD(tm, ov ? cbv : -bv, bv);
        if (kind == kDfsEnter) {
          const T bl = w.coef[2], cbl = w.coef[3];
          const T Fl = fmaD(tm, (mine & 2u) ? cbl : -bl, bl);
          cst[level * 64 + lane] = C;
          // C times F_f^u / F_f^v; a vanishing F_f^v leaves the subtree at zero
          const T rv = rcpD(Fv);
          C = Fv == T(0) ? T(0) : C * Fl * rv;
          H = w.lv[0] * C;  // used only when the left child is a leaf
        } else if (kind == kDfsMiddle) {
          const T br = w.coef[4], cbr = w.coef[5];
          const T Fr = fmaD(tm, (mine & 4u) ? cbr : -br, br);
          const T Cv = cst[level * 64 + lane];
          hst[level * 64 + lane] = H;
          const T rv = rcpD(Fv);
          C = Fv == T(0) ? T(0) : Cv * Fr * rv;
          H = w.lv[1] * C;
        } else {
          // both subtrees done: H holds H_R, the stack H_L
          const bool ol = (mine & 2u) != 0, orr = (mine & 4u) != 0;
          const T bl = w.coef[2], cbl = w.coef[3], br = w.coef[4], cbr = w.coef[5];
          const T Fl = fmaD(tm, ol ? cbl : -bl, bl);
          const T Fr = fmaD(tm, orr ? cbr : -br, br);
          const T HL = hst[level * 64 + lane];
          const T nl = ol ? w.coef[6] : (ov ? -bl : T(0));
          const T nr = orr ? w.coef[7] : (ov ? -br : T(0));
          const T il = rcpD(Fl * Fv), ir = rcpD(Fr * Fv);
          const T tl = (Fl == T(0) || Fv == T(0)) ? T(0) : HL * nl * il;
          const T tr = (Fr == T(0) || Fv == T(0)) ? T(0) : H * nr * ir;
          if (valid) Y[((int64_t)sl * n_rows + w.row) * kNodes + m] = wm * (tl + tr);
          H = HL + H;
        }
      };
      // two steps per iteration, each record read one step ahead (the LDS
      // latency of the broadcast overlaps the previous step's arithmetic)
      StagedEvent<T> e0 = stage[0];
      for (int k = 0; k < nwin; k += 2) {
        const StagedEvent<T> e1 = stage[min(k + 1, nwin - 1)];
        step(e0, k);
        if (k + 1 < nwin) {
          e0 = stage[min(k + 2, nwin - 1)];
          step(e1, k + 1);
        }
      }
      // the next window overwrites the stage
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// Per-call values of each record's leaf children (0 for an internal child),
// from the current leaf values, in the walk's precision.
template <typename T>
__global__ void __launch_bounds__(256)
dfs_leaf_values_kernel(const DfsNode* __restrict__ nodes, int32_t n,
                       const double* __restrict__ leaf_val, T* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int l = nodes[r].leaf_l, rr = nodes[r].leaf_r;
  out[2 * (size_t)r] = l >= 0 ? (T)leaf_val[l] : T(0);
  out[2 * (size_t)r + 1] = rr >= 0 ? (T)leaf_val[rr] : T(0);
}

template <typename T>
__global__ void __launch_bounds__(1024)
dfs_pairs_kernel(const int32_t* __restrict__ row_f, const int32_t* __restrict__ row_d,
                 const int32_t* __restrict__ tile_base, const int32_t* __restrict__ tile_d,
                 const int32_t* __restrict__ feat, const float* __restrict__ lo,
                 const float* __restrict__ hi, const T* __restrict__ bb,
                 const T* __restrict__ cbb, int32_t t0, int32_t t1, int32_t chunk,
                 const T* __restrict__ Y, int32_t n_rows, const float* __restrict__ X,
                 int64_t s0, int32_t mb, int64_t ldx, int32_t F, int32_t r0, int32_t r1,
                 int32_t with_phi, int32_t ng, int32_t grp, double* __restrict__ tri64,
                 double* __restrict__ phi64, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t ntri = (int64_t)F * (F - 1) / 2;
  const int64_t base0 = (int64_t)r0 * (r0 - 1) / 2;
  const int64_t ntri_r = (int64_t)r1 * (r1 - 1) / 2 - base0;
  double* phis = reinterpret_cast<double*>(smem);  // [F]
  double* tris = phis + F;                         // [ntri_r]
  float* xrow = reinterpret_cast<float*>(tris + ntri_r);  // [F]
  const int sl = (int)(blockIdx.x % (unsigned)mb);
  const int ch = (int)(blockIdx.x / (unsigned)mb);
  const int64_t s = s0 + sl;
  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    xrow[i] = X[s * ldx + i];
    phis[i] = 0.0;
  }
  for (int64_t e = threadIdx.x; e < ntri_r; e += blockDim.x) tris[e] = 0.0;
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int tb0 = t0 + ch * chunk;
  const int tb1 = min(t1, tb0 + chunk);
  for (int tile = tb0 + wave; tile < tb1; tile += nw) {
    const int row = tile * 64 + lane;
    const int f = row_f[row];
    const int d = row_d[row];
    T y[kNodes];
    T ysum = T(0);
    const T* yp = Y + ((int64_t)sl * n_rows + row) * kNodes;
#pragma unroll
    for (int k = 0; k < kNodes; ++k) {
      y[k] = f >= 0 ? yp[k] : T(0);
      ysum += y[k];
    }
    if (with_phi && f >= 0 && ysum != T(0))
      __hip_atomic_fetch_add(&phis[f], (double)ysum, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    const int eb = __builtin_amdgcn_readfirstlane(tile_base[tile]);
    const int td = __builtin_amdgcn_readfirstlane(tile_d[tile]);
    // slots in groups of four: every load of a group issues before its first
    // use, so the wave waits for memory once per group, not once per slot
    for (int k0 = 0; k0 < td; k0 += 4) {
      int fm[4];
      float l[4], u[4], xv[4];
      T bq[4], cq[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int e = eb + 64 * min(k0 + w, td - 1) + lane;
        fm[w] = feat[e];
        l[w] = lo[e];
        u[w] = hi[e];
        bq[w] = bb[e];
        cq[w] = cbb[e];
      }
#pragma unroll
      for (int w = 0; w < 4; ++w) xv[w] = xrow[fm[w] & kFeatureMask];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int k = k0 + w;
        const T b = bq[w];
        const bool o = follows(xv[w], l[w], u[w], (fm[w] & kMissingOkBit) != 0);
        const T c = o ? cq[w] : -b;
        // a factor that vanishes identically zeroes every leaf below (y = 0)
        if (k < d && f >= 0 && !(b == T(0) && c == T(0))) {
          T acc = y[0] * rcpD(fmaD(nc.t[0], c, b));
#pragma unroll
          for (int m = 1; m < kNodes; ++m) acc = fmaD(y[m], rcpD(fmaD(nc.t[m], c, b)), acc);
          const T v = c * acc;
          const int j = fm[w] & kFeatureMask;
          const int a = min(f, j), zf = max(f, j);
          if (zf >= r0 && zf < r1 && v != T(0))
            __hip_atomic_fetch_add(&tris[(int64_t)zf * (zf - 1) / 2 + a - base0], (double)v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
    }
  }
  __syncthreads();
  const int64_t orow = s * ng + grp;
  if (with_phi)
    for (int i = threadIdx.x; i < F; i += blockDim.x) {
      const double v = phis[i];
      if (v != 0.0) unsafeAtomicAdd(&phi64[orow * F + i], v);
    }
  for (int64_t e = threadIdx.x; e < ntri_r; e += blockDim.x) {
    const double v = tris[e];
    if (v != 0.0) unsafeAtomicAdd(&tri64[orow * ntri + base0 + e], v);
  }
}

// Lane values from within a group of 8 lanes (DPP): quad_perm swaps with lane
// ^ 1 and ^ 2, and row_half_mirror (lane i <-> 7 - i of each 8).
template <int CTRL>
__device__ __forceinline__ float dpp8(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp8(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF,
                                                            false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL,
                                                            0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// Sum over each group of 8 consecutive lanes (all active), in every lane.
template <typename T>
__device__ __forceinline__ T sum8(T v) {
  v += dpp8<0xB1>(v);
  v += dpp8<0x4E>(v);
  v += dpp8<0x141>(v);
  return v;
}

__host__ __device__ __forceinline__ int64_t tet3(int64_t z) { return z * (z - 1) * (z - 2) / 6; }

// fn(integral_constant<int, 0>), ..., fn(integral_constant<int, N - 1>): an
// unrolled loop whose index is a compile-time constant (register arrays
// indexed by it stay in registers, whatever the unroller's limits).
template <typename Fn, int... I>
__device__ __forceinline__ void unroll_seq(Fn&& fn, std::integer_sequence<int, I...>) {
  (fn(std::integral_constant<int, I>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void unroll(Fn&& fn) {
  unroll_seq(fn, std::make_integer_sequence<int, N>{});
}

// The depth-first form at order 3 (Theorem 1 with |S| = 3).  Along a
// root-to-leaf path the product of three features' ratios r = c / F changes
// only where one of the three is split, by that feature's change times the
// other two ratios at the node; so, as at order 2 (Eq. 11), the index is a sum
// over internal nodes v on feature f, with the walk's y_v, of
//   SII_{f j k} += sum_m y_v(t_m) r_j^v(t_m) r_k^v(t_m)
// for every pair {j, k} of the other features split above v.  Lane = (row of
// 8, node m of 8); a lane keeps the ratios of its row's features at its node
// in registers (a row's features are sorted, so j < k means f_j < f_k); per
// pair the 8 node lanes' terms are summed across lanes, and the 8 lanes share
// the adds into the sample's packed tensor range in LDS (FP64): triples whose
// largest feature lies in [r0, r1), at tet3(c) + c2(b) + a for a < b < c.
template <typename T, int CAP, bool GLOBAL>
__global__ void __launch_bounds__(512)
dfs_triples_kernel(const int32_t* __restrict__ row_f, const int32_t* __restrict__ row_d,
                   const int32_t* __restrict__ tile_base, const int32_t* __restrict__ tile_d,
                   const int32_t* __restrict__ feat, const float* __restrict__ lo,
                   const float* __restrict__ hi, const T* __restrict__ bb,
                   const T* __restrict__ cbb, int32_t t0, int32_t t1, int32_t chunk,
                   const T* __restrict__ Y, int32_t n_rows, const float* __restrict__ X,
                   int64_t s0, int32_t mb, int64_t ldx, int32_t F, int32_t r0, int32_t r1,
                   int32_t ng, int32_t grp, double* __restrict__ acc, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t nt = tet3(F);
  const int64_t base0 = tet3(r0);
  const int64_t ntr = tet3(r1) - base0;
  double* ts = reinterpret_cast<double*>(smem);  // [ntr] (LDS form)
  float* xrow = GLOBAL ? reinterpret_cast<float*>(smem) : reinterpret_cast<float*>(ts + ntr);
  const int sl = (int)(blockIdx.x % (unsigned)mb);
  const int ch = (int)(blockIdx.x / (unsigned)mb);
  const int64_t s = s0 + sl;
  for (int i = threadIdx.x; i < F; i += blockDim.x) xrow[i] = X[s * ldx + i];
  if (!GLOBAL)
    for (int64_t e = threadIdx.x; e < ntr; e += blockDim.x) ts[e] = 0.0;
  __syncthreads();
  double* gacc = acc + (s * ng + grp) * nt + base0;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int q = lane >> 3, m = lane & 7;
  T tm = nc.t[0];
#pragma unroll
  for (int k = 1; k < kNodes; ++k) tm = m == k ? nc.t[k] : tm;
  const int tb0 = t0 + ch * chunk;
  const int tb1 = min(t1, tb0 + chunk);
  for (int tile = tb0 + wave; tile < tb1; tile += nw) {
    const int eb = __builtin_amdgcn_readfirstlane(tile_base[tile]);
    const int td = __builtin_amdgcn_readfirstlane(tile_d[tile]);
    for (int g = 0; g < 8; ++g) {
      const int ri = g * 8 + q;  // row within the tile
      const int row = tile * 64 + ri;
      const int f = row_f[row];
      const int d = f >= 0 ? row_d[row] : 0;
      const T y = f >= 0 ? Y[((int64_t)sl * n_rows + row) * kNodes + m] : T(0);
      T r[CAP];
      int fe[CAP];
#pragma unroll
      for (int k = 0; k < CAP; ++k) {
        r[k] = T(0);
        fe[k] = 0;
        if (k < d) {
          const int e = eb + 64 * k + ri;
          const int fm = feat[e];
          const T b = bb[e];
          const bool o = follows(xrow[fm & kFeatureMask], lo[e], hi[e],
                                 (fm & kMissingOkBit) != 0);
          const T c = o ? cbb[e] : -b;
          fe[k] = fm & kFeatureMask;
          // a factor that vanishes identically zeroes every leaf below (y = 0)
          if (!(b == T(0) && c == T(0))) r[k] = c * rcpD(fmaD(tm, c, b));
        }
      }
      // indices relative to the range start fit 32 bits (the range is in LDS)
      const int P_f = f * (f - 1) / 2;
      unroll<CAP>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        if (k == 0 || k >= td) return;
        const int fk = fe[k];
        const int zc = max(f, fk);  // the largest feature of every triple (f, f_j, f_k), j < k
        const bool in = k < d && zc >= r0 && zc < r1;
        // no row of the wave has triples of this slot in the range
        if (__ballot(in) == 0) return;
        const int Tc = (int)(tet3(zc) - base0);
        const int P_k = fk * (fk - 1) / 2;
        const T yk = y * r[k];
        // the slot's cross-lane sums first (independent chains), then its
        // updates under one branch
        T pk[k > 0 ? k : 1];
        unroll<k>([&](auto jc) __attribute__((always_inline)) {
          constexpr int j = decltype(jc)::value;
          pk[j] = sum8(yk * r[j]);
        });
        // every node lane of a row holds all of them: lane m adds the pairs
        // j = 8 i + m
        unroll<(k + 7) / 8>([&](auto ic) __attribute__((always_inline)) {
          constexpr int i = decltype(ic)::value;
          T v = pk[8 * i];
          int fj = fe[8 * i];
          unroll<7>([&](auto mc) __attribute__((always_inline)) {
            constexpr int mm = decltype(mc)::value + 1;
            if constexpr (8 * i + mm < k) {
              // opaque register copies: a chain of selects between array
              // elements would otherwise fold into one indexed load, which
              // takes the arrays out of registers
              T a = pk[8 * i + mm];
              int fa = fe[8 * i + mm];
              __asm__ volatile("" : "+v"(a), "+v"(fa));
              v = m == mm ? a : v;
              fj = m == mm ? fa : fj;
            }
          });
          if (in && 8 * i + m < k && v != T(0)) {
            // (a, b, c) = (f_j, f_k, f), (f_j, f, f_k) or (f, f_j, f_k)
            const int idx = f > fk ? Tc + P_k + fj
                                   : (f > fj ? Tc + P_f + fj : Tc + fj * (fj - 1) / 2 + f);
            if (GLOBAL) unsafeAtomicAdd(&gacc[idx], (double)v);
            else
              __hip_atomic_fetch_add(&ts[idx], (double)v, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        });
      });
    }
  }
  if (GLOBAL) return;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < ntr; e += blockDim.x) {
    const double v = ts[e];
    if (v != 0.0) unsafeAtomicAdd(&gacc[e], v);
  }
}

namespace {

int64_t tri_h(int64_t k) { return k * (k - 1) / 2; }

template <typename T>
void walk_t(const HostTable& h, const DeviceDfs& d, const NodeConsts<T>& nc,
            const double* leaf_val, const float* X, int64_t s0, int32_t mb, int64_t ldx, T* Y,
            T* lvals, hipStream_t s) {
  const int F = h.F;
  const int levels = d.max_level + 1;
  if (s0 == 0 && d.n_nodes > 0) {
    hipLaunchKernelGGL((dfs_leaf_values_kernel<T>), dim3((unsigned)((d.n_nodes + 255) / 256)),
                       dim3(256), 0, s, d.nodes, (int32_t)d.n_nodes, leaf_val, lvals);
    check_hip(hipGetLastError(), "dfs_leaf_values_kernel launch");
  }
  const size_t limit = raise_lds_limit((const void*)dfs_walk_kernel<T>);
  // as many waves (trees) per workgroup as the stacks allow, up to 16: the
  // walk is bound by the latency of its sequential steps, which more waves hide
  int waves = 16;
  while (waves > 1 && dfs_walk_lds(F, levels, waves, sizeof(T)) > limit) --waves;
  const size_t lds = dfs_walk_lds(F, levels, waves, sizeof(T));
  if (lds > limit) fail(QTS_E_UNSUPPORTED, "internal: tree too deep for the depth-first walk");
  const int nsg = (mb + kDfsSamples - 1) / kDfsSamples;
  const int n_tb = (d.n_trees + waves - 1) / waves;
  const int64_t grid = (int64_t)nsg * n_tb;
  if (grid <= 0) return;
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "depth-first walk grid too large");
  const T* coef = std::is_same<T, float>::value ? (const T*)d.coef32 : (const T*)d.coef64;
  hipLaunchKernelGGL((dfs_walk_kernel<T>), dim3((unsigned)grid), dim3(64 * waves), lds, s,
                     d.nodes, coef, (const T*)lvals, d.events, d.tree_first, d.tree_nodes,
                     d.n_trees, X, s0, mb, ldx, F, levels, nsg, d.n_rows, Y, nc);
  check_hip(hipGetLastError(), "dfs_walk_kernel launch");
}

template <typename T>
void pairs_t(const HostTable& h, const DeviceDfs& d, const NodeConsts<T>& nc, const float* X,
             int64_t s0, int32_t mb, int64_t ldx, const T* Y, double* tri64, double* phi64,
             int32_t tiles_per_chunk, hipStream_t s) {
  const int F = h.F;
  const void* fn = (const void*)dfs_pairs_kernel<T>;
  const size_t limit = raise_lds_limit(fn);
  const size_t fixed = (size_t)F * sizeof(double) + (size_t)F * sizeof(float);
  if (fixed >= limit) fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
  // triangle rows [r0, r1) whose FP64 entries fit beside the fixed part
  const int64_t cap = (int64_t)((limit - fixed) / sizeof(double));
  if (cap < F) fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
  for (int g = 0; g < h.n_groups; ++g) {
    const int t0 = d.group_tile[g], t1 = d.group_tile[g + 1];
    if (t1 <= t0) continue;
    const int chunk = std::max(1, tiles_per_chunk);
    const int64_t n_chunks = (t1 - t0 + chunk - 1) / chunk;
    const int64_t grid = (int64_t)mb * n_chunks;
    if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "depth-first pair grid too large");
    const T* b = std::is_same<T, float>::value ? (const T*)d.b32 : (const T*)d.b64;
    const T* cb = std::is_same<T, float>::value ? (const T*)d.cb32 : (const T*)d.cb64;
    bool first = true;
    int r0 = 0;
    while (r0 < F) {
      int r1 = r0 + 1;
      while (r1 < F && tri_h(r1 + 1) - tri_h(r0) <= cap) ++r1;
      const size_t lds = fixed + (size_t)(tri_h(r1) - tri_h(r0)) * sizeof(double);
      hipLaunchKernelGGL((dfs_pairs_kernel<T>), dim3((unsigned)grid), dim3(1024), lds, s,
                         d.row_f, d.row_d, d.tile_base, d.tile_d, d.feat, d.lo, d.hi, b, cb, t0,
                         t1, chunk, Y, d.n_rows, X, s0, mb, ldx, F, r0, r1, (int)first,
                         h.n_groups, g, tri64, phi64, nc);
      check_hip(hipGetLastError(), "dfs_pairs_kernel launch");
      first = false;
      r0 = r1;
    }
  }
}

// The third-order pass adds into the sample's tensor range in LDS and
// flushes it, one launch per range of the largest feature; where that would
// take more than kDfs3MaxRanges ranges (every range walks all rows again), it
// adds straight into the output with FP64 atomics instead.
constexpr int kDfs3MaxRanges = 4;

template <typename T, int CAP, bool G>
void triples3_launch(const HostTable& h, const DeviceDfs& d, const NodeConsts<T>& nc,
                     const float* X, int64_t s0, int32_t mb, int64_t ldx, const T* Y,
                     double* acc, int32_t chunk, int g, int r0, int r1, hipStream_t s) {
  const int F = h.F;
  const int t0 = d.group_tile[g], t1 = d.group_tile[g + 1];
  const int64_t grid = (int64_t)mb * ((t1 - t0 + chunk - 1) / chunk);
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "depth-first third-order grid too large");
  const T* b = std::is_same<T, float>::value ? (const T*)d.b32 : (const T*)d.b64;
  const T* cb = std::is_same<T, float>::value ? (const T*)d.cb32 : (const T*)d.cb64;
  const size_t lds = G ? (size_t)F * sizeof(float) + 16
                       : (((size_t)(tet3(r1) - tet3(r0)) * sizeof(double) + 15) & ~(size_t)15) +
                             (size_t)F * sizeof(float);
  hipLaunchKernelGGL((dfs_triples_kernel<T, CAP, G>), dim3((unsigned)grid), dim3(512), lds, s,
                     d.row_f, d.row_d, d.tile_base, d.tile_d, d.feat, d.lo, d.hi, b, cb, t0, t1,
                     chunk, Y, d.n_rows, X, s0, mb, ldx, F, r0, r1, h.n_groups, g, acc, nc);
  check_hip(hipGetLastError(), "dfs_triples_kernel launch");
}

template <typename T, int CAP>
void triples3_t(const HostTable& h, const DeviceDfs& d, const NodeConsts<T>& nc, const float* X,
                int64_t s0, int32_t mb, int64_t ldx, const T* Y, double* acc,
                int32_t tiles_per_chunk, hipStream_t s) {
  const int F = h.F;
  const size_t limit = raise_lds_limit((const void*)dfs_triples_kernel<T, CAP, false>);
  raise_lds_limit((const void*)dfs_triples_kernel<T, CAP, true>);
  const size_t fixed = (size_t)F * sizeof(float) + 16;
  if (fixed >= limit) fail(QTS_E_UNSUPPORTED, "n_features too large for the third-order kernel");
  const int64_t cap = (int64_t)((limit - fixed) / sizeof(double));
  // ranges of the largest feature z (z holds z(z-1)/2 triples)
  std::vector<std::pair<int, int>> ranges;
  for (int r0 = 0; r0 < F && (int)ranges.size() <= kDfs3MaxRanges;) {
    int r1 = r0 + 1;
    while (r1 < F && tet3(r1 + 1) - tet3(r0) <= cap) ++r1;
    if (tet3(r1) - tet3(r0) > cap) {
      ranges.assign(kDfs3MaxRanges + 1, {0, 0});  // one largest feature does not fit
      break;
    }
    ranges.emplace_back(r0, r1);
    r0 = r1;
  }
  const int chunk = std::max(1, tiles_per_chunk);
  for (int g = 0; g < h.n_groups; ++g) {
    if (d.group_tile[g + 1] <= d.group_tile[g]) continue;
    if ((int)ranges.size() > kDfs3MaxRanges) {
      triples3_launch<T, CAP, true>(h, d, nc, X, s0, mb, ldx, Y, acc, chunk, g, 0, F, s);
      continue;
    }
    for (const auto& rr : ranges)
      triples3_launch<T, CAP, false>(h, d, nc, X, s0, mb, ldx, Y, acc, chunk, g, rr.first,
                                     rr.second, s);
  }
}

}  // namespace

bool dfs_triples_supported(const DeviceDfs& d) { return d.max_row_d <= kDfsTriplesMaxRow; }

void launch_dfs_triples(const HostTable& h, const DeviceDfs& d, const DeviceTable& dt, bool fp64,
                        const float* X, int64_t s0, int32_t mb, int64_t ldx, const void* Y,
                        double* acc, int32_t tiles_per_chunk, hipStream_t s) {
  if (!dfs_triples_supported(d))
    fail(QTS_E_UNSUPPORTED, "internal: rows too long for the depth-first third-order pass");
  if (fp64) {
    if (d.max_row_d <= 16)
      triples3_t<double, 16>(h, d, dt.n64, X, s0, mb, ldx, (const double*)Y, acc,
                             tiles_per_chunk, s);
    else
      triples3_t<double, 32>(h, d, dt.n64, X, s0, mb, ldx, (const double*)Y, acc,
                             tiles_per_chunk, s);
  } else {
    if (d.max_row_d <= 16)
      triples3_t<float, 16>(h, d, dt.n32, X, s0, mb, ldx, (const float*)Y, acc, tiles_per_chunk,
                            s);
    else
      triples3_t<float, 32>(h, d, dt.n32, X, s0, mb, ldx, (const float*)Y, acc, tiles_per_chunk,
                            s);
  }
}

size_t dfs_walk_lds_bytes(int F, int max_level, bool fp64) {
  return dfs_walk_lds(F, max_level + 1, 1, fp64 ? sizeof(double) : sizeof(float));
}

void launch_dfs_walk(const HostTable& h, const DeviceDfs& d, const DeviceTable& dt, bool fp64,
                     const double* leaf_val, const float* X, int64_t s0, int32_t mb,
                     int64_t ldx, void* Y, void* lvals, hipStream_t s) {
  if (fp64) walk_t<double>(h, d, dt.n64, leaf_val, X, s0, mb, ldx, (double*)Y, (double*)lvals, s);
  else walk_t<float>(h, d, dt.n32, leaf_val, X, s0, mb, ldx, (float*)Y, (float*)lvals, s);
}

void launch_dfs_pairs(const HostTable& h, const DeviceDfs& d, const DeviceTable& dt, bool fp64,
                      const float* X, int64_t s0, int32_t mb, int64_t ldx, const void* Y,
                      double* tri64, double* phi64, int32_t tiles_per_chunk, hipStream_t s) {
  if (fp64)
    pairs_t<double>(h, d, dt.n64, X, s0, mb, ldx, (const double*)Y, tri64, phi64,
                    tiles_per_chunk, s);
  else
    pairs_t<float>(h, d, dt.n32, X, s0, mb, ldx, (const float*)Y, tri64, phi64,
                   tiles_per_chunk, s);
}

}  // namespace qts
