// Pairwise Shapley interaction indices (Theorem 1 with |S| = 2, Eq. 9-10,
// 8 nodes) and first-order values, per sample; third-order indices (|S| = 3)
// on the same row table further below (triples_lane_kernel, triples_kernel).
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
// Slot 0 is never divided by: with H0 = prod_{j >= 1} F_j,
//   g_0 = w val H0 c_0   and   g_i = w val H0 F_0 r_i  (i >= 1),
// which holds for any path.  It lets slot 0 carry the combined factor of a
// merged pair of sibling leaves A, B (split feature L):
//   vA F^A_L + vB F^B_L = bm + t c,  bm = vA b_A + vB b_B,
//   c = vA (1-b_A) - vB b_B (A followed), vB (1-b_B) - vA b_A (B followed),
//   else -bm,
// with the row's leaf value 1; that factor may vanish at a node, which the
// H0 form never divides by.  Slots 1.. are sorted by feature; slot 0 is any
// feature, so its pairs take the smaller/larger of the two features.
//
// Accumulation.  A workgroup owns one explained sample; the sample's pair
// triangle (pair i < k at k(k-1)/2 + i; features are sorted inside a path, so
// f_i < f_k) and its phi row accumulate in LDS in FP64 and are flushed with
// FP64 atomics to the global accumulators.  FP64 is the accumulation type
// for both kernel precisions: besides the precision, gfx950's LDS FP64 atomic
// add sustains about seven times the lane rate of its FP32 one.  When the
// triangle does not fit in LDS it is cut into ranges of rows k (the larger
// feature of the pair), one launch per range; a launch adds only the pairs
// whose larger feature falls in its range, and phi only in the first one.
#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

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
// FP64 reciprocal: the hardware estimate refined by two Newton steps
// (e = 1 - x r, r += r e; each squares the relative error), about five
// instructions where a correctly rounded division takes about eleven.  For
// the normal x in (0, 1] the factors take this is within about an ulp of 1/x.
__device__ __forceinline__ double rcpP(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int64_t tri_row(int64_t k) { return k * (k - 1) / 2; }

// Lane exchanges inside a quad of lanes (DPP quad_perm): partner lane ^ 1 and ^ 2.
constexpr int kQuadXor1 = 0xB1;  // [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // [2, 3, 0, 1]

template <int CTRL>
__device__ __forceinline__ float quad_swap(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the LS lanes that share a path (LS = 1, 2 or 4 consecutive lanes,
// all active together).
template <int LS, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if constexpr (LS >= 4) v += quad_swap<kQuadXor2>(v);
  if constexpr (LS >= 2) v += quad_swap<kQuadXor1>(v);
  return v;
}

// Add four pair values to the triangle with one atomic per pair.  With LS
// lanes per path each lane holds its nodes' part of the four sums; a
// reduce-scatter over the group leaves lane q with the totals of pairs
// u = q, q + LS, ..., which it adds.  idx/ok give each pair's triangle entry
// and whether it is stored.  The lane's choices are selects between scalars
// (a select between array elements can become a lane-dependent index, which
// puts the array in scratch memory).
template <int LS, typename T>
__device__ __forceinline__ void group_add(double* tris, const T (&pr)[4], const int (&idx)[4],
                                          const bool (&ok)[4], int q) {
  if constexpr (LS == 1) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ok[u]) lds_add(&tris[idx[u]], (double)pr[u]);
  } else if constexpr (LS == 2) {
    const bool h1 = (q & 1) != 0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const T a = pr[2 * t], b = pr[2 * t + 1];
      const int ea = idx[2 * t], eb = idx[2 * t + 1];
      const bool oa = ok[2 * t], ob = ok[2 * t + 1];
      const T sum = (h1 ? b : a) + quad_swap<kQuadXor1>(h1 ? a : b);
      if (h1 ? ob : oa) lds_add(&tris[h1 ? eb : ea], (double)sum);
    }
  } else {
    static_assert(LS == 4, "1, 2 or 4 lanes per path");
    const bool h2 = (q & 2) != 0, h1 = (q & 1) != 0;
    const T a0 = pr[0], a1 = pr[1], a2 = pr[2], a3 = pr[3];
    // lanes q and q ^ 2: keep pairs {2 h2, 2 h2 + 1}
    const T s0 = (h2 ? a2 : a0) + quad_swap<kQuadXor2>(h2 ? a0 : a2);
    const T s1 = (h2 ? a3 : a1) + quad_swap<kQuadXor2>(h2 ? a1 : a3);
    // lanes q and q ^ 1: keep pair 2 h2 + h1 = q
    const T sum = (h1 ? s1 : s0) + quad_swap<kQuadXor1>(h1 ? s0 : s1);
    const int e0 = idx[0], e1 = idx[1], e2 = idx[2], e3 = idx[3];
    const bool o0 = ok[0], o1 = ok[1], o2 = ok[2], o3 = ok[3];
    const int e = h2 ? (h1 ? e3 : e2) : (h1 ? e1 : e0);
    const bool o = h2 ? (h1 ? o3 : o2) : (h1 ? o1 : o0);
    if (o) lds_add(&tris[e], (double)sum);
  }
}

// group_add for LS > 1 where pair (i, k) sits at tris[rb[k] + f_i] (every
// pair but a merged slot 0's): lane q's offsets were chosen once per path
// (rbs[j] = rb[j + q], or -1 if not stored), so only the values need selects.
// The merged slot-0 pairs, whose entry depends on which feature is larger,
// take group_add.
template <int LS, int C, typename T>
__device__ __forceinline__ void group_add_own(double* tris, const T (&pr)[4], const int (&rbs)[C],
                                              int kb, int fi, int q) {
  if constexpr (LS == 2) {
    const bool h1 = (q & 1) != 0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (kb + 2 * t < C) {
        const T a = pr[2 * t], b = pr[2 * t + 1];
        const T sum = (h1 ? b : a) + quad_swap<kQuadXor1>(h1 ? a : b);
        const int e = rbs[kb + 2 * t];
        if (e >= 0) lds_add(&tris[e + fi], (double)sum);
      }
    }
  } else {
    static_assert(LS == 4, "2 or 4 lanes per path");
    const bool h2 = (q & 2) != 0, h1 = (q & 1) != 0;
    const T a0 = pr[0], a1 = pr[1], a2 = pr[2], a3 = pr[3];
    const T s0 = (h2 ? a2 : a0) + quad_swap<kQuadXor2>(h2 ? a0 : a2);
    const T s1 = (h2 ? a3 : a1) + quad_swap<kQuadXor2>(h2 ? a1 : a3);
    const T sum = (h1 ? s1 : s0) + quad_swap<kQuadXor1>(h1 ? s0 : s1);
    if (rbs[kb] >= 0) lds_add(&tris[rbs[kb] + fi], (double)sum);
  }
}

// Zero the LDS accumulators and stage the sample row.
__device__ __forceinline__ void pairs_prologue(double* phis, double* tris, int64_t ntri_r,
                                               float* xrow, const float* X, int64_t s,
                                               int64_t ldx, int F) {
  for (int i = threadIdx.x; i < F; i += blockDim.x) {
    xrow[i] = X[s * ldx + i];
    phis[i] = 0.0;
  }
  for (int64_t e = threadIdx.x; e < ntri_r; e += blockDim.x) tris[e] = 0.0;
  __syncthreads();
}

// Flush the LDS accumulators of output row s (sample, group) into the global
// FP64 ones.
__device__ __forceinline__ void pairs_epilogue(const double* phis, const double* tris,
                                               int64_t ntri_r, int64_t base, int64_t ntri,
                                               bool with_phi, int64_t s, int F,
                                               double* tri64, double* phi64) {
  __syncthreads();
  if (with_phi)
    for (int i = threadIdx.x; i < F; i += blockDim.x) {
      const double v = phis[i];
      if (v != 0.0) unsafeAtomicAdd(&phi64[s * F + i], v);
    }
  for (int64_t e = threadIdx.x; e < ntri_r; e += blockDim.x) {
    const double v = tris[e];
    if (v != 0.0) unsafeAtomicAdd(&tri64[s * ntri + base + e], v);
  }
}

}  // namespace

// Lane-per-path form for short paths (capacity C, register resident).  Each
// path of the class is taken by LS consecutive lanes (the table is slot-major,
// so a wave's 64 / LS paths load coalesced).  NN nodes (the rule's size, 8 or
// fewer where fewer are exact), NH per lane at a time, to bound the registers
// held by r (the node sum is additive): NN / (NH LS) passes, each adding its
// partial sums with its own atomics; with LS > 1 the group's lanes take
// different nodes in a pass and their partial sums are added across the group
// (DPP) before one atomic per pair and pass.
template <typename T, int C, int NH, bool MERGE, int NN, int LS>
__global__ void __launch_bounds__(512)
pairs_kernel(const int32_t* __restrict__ pd, const int32_t* __restrict__ pleaf,
             const SidePath* __restrict__ pside, const int32_t* __restrict__ feat,
             const float* __restrict__ lo, const float* __restrict__ hi,
             const T* __restrict__ bb, const T* __restrict__ cbb,
             int32_t np, int32_t chunk, const double* __restrict__ leaf_val,
             const float* __restrict__ X, int64_t M, int64_t ldx, int32_t F, int32_t r0,
             int32_t r1, int32_t with_phi, int32_t ng, int32_t grp,
             double* __restrict__ tri64, double* __restrict__ phi64, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t ntri = tri_row(F + 1) - F;         // F(F-1)/2
  const int64_t base0 = tri_row(r0);
  const int64_t ntri_r = tri_row(r1) - base0;      // rows [r0, r1)
  double* phis = reinterpret_cast<double*>(smem);  // [F]
  double* tris = phis + F;                         // [ntri_r]
  float* xrow = reinterpret_cast<float*>(tris + ntri_r);  // [F]

  const int64_t s = (int64_t)blockIdx.x % M;
  const int ch = (int)((int64_t)blockIdx.x / M);
  const int p0 = ch * chunk;
  const int p1 = min(np, p0 + chunk);
  pairs_prologue(phis, tris, ntri_r, xrow, X, s, ldx, F);

  constexpr int NP = NN / (NH * LS);  // node passes
  static_assert(NP * NH * LS == NN, "passes of NH nodes on each of LS lanes");
  constexpr int PW = 64 / LS;  // paths per wave
  const int lane = threadIdx.x & 63;
  const int q = lane % LS;     // pass P: the lane takes nodes P NH LS + q NH + [0, NH)
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  // LS > 1: the lane's nodes and weights per pass, selected with static indices
  T tq[NP * NH], wq[NP * NH];
#pragma unroll
  for (int e = 0; e < NP * NH; ++e) {
    const int n0 = (e / NH) * NH * LS + e % NH;
    tq[e] = nc.t[n0];
    wq[e] = nc.w[n0];
#pragma unroll
    for (int g = 1; g < LS; ++g) {
      tq[e] = q == g ? nc.t[n0 + g * NH] : tq[e];
      wq[e] = q == g ? nc.w[n0 + g * NH] : wq[e];
    }
  }
  for (int base = p0 + wave * PW; base < p1; base += nw * PW) {
    const int p = base + lane / LS;
    const bool valid = p < p1;
    const int pc = valid ? p : p1 - 1;  // clamped index for the loads
    // every table load of the path issues before the first use, and none is
    // conditional, so a wave waits for memory once per path instead of once
    // per slot
    int fm[C];
    float lov[C], hiv[C];
    T bv[C], cbv[C];
    const int d0 = pd[pc];
    const int leaf = pleaf[pc];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int64_t e = (int64_t)j * np + pc;
      fm[j] = feat[e];
      lov[j] = lo[e];
      hiv[j] = hi[e];
      bv[j] = bb[e];
      cbv[j] = cbb[e];
    }
    // MERGE: the class may hold merged rows (capacity <= kPairMergeMax)
    SidePath sp{};
    if (MERGE) sp = pside[pc];
    const bool merged = MERGE && valid && sp.leaf_b >= 0;
    const double va = leaf_val[leaf];
    const double vb = MERGE ? leaf_val[merged ? sp.leaf_b : leaf] : 0.0;
    const int d = valid ? d0 : 0;
    T val = valid ? (merged ? T(1) : (T)va) : T(0);
    // combined slot-0 factor of a merged row, in FP64, then rounded
    const T bm = MERGE ? (T)(va * sp.b_a + vb * sp.b_b) : T(0);
    const T cAm = MERGE ? (T)(va * sp.cb_a - vb * sp.b_b) : T(0);
    const T cBm = MERGE ? (T)(vb * sp.cb_b - va * sp.b_a) : T(0);
    // feature, row offset of its pairs in this launch's triangle rows, and
    // whether those rows are in range; then the slot's c = o - b and b (a
    // slot j >= 1 with b = 0 and o = 0 zeroes the path: its b is replaced by 1)
    int f[C], rb[C];
    bool inr[C];
    T cj[C], bj[C];
    bool dead = false;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      f[j] = fm[j] & kFeatureMask;
      rb[j] = (int)(tri_row(f[j]) - base0);
      inr[j] = (f[j] >= r0) & (f[j] < r1) & (j < d);
      const float x = xrow[f[j]];
      const bool miss = (fm[j] & kMissingOkBit) != 0;
      const bool lower = miss ? !(x < lov[j]) : (x >= lov[j]);
      const bool upper = !(x >= hiv[j]);
      const T b = bv[j];
      T c = (lower & upper) ? cbv[j] : -b;
      if (j == 0) {
        if (MERGE) {
          const bool lowerB = sp.mok_b ? !(x < sp.lo_b) : (x >= sp.lo_b);
          const bool upperB = !(x >= sp.hi_b);
          const T cm = (lower & upper) ? cAm : ((lowerB & upperB) ? cBm : -bm);
          cj[0] = merged ? cm : c;
          bj[0] = merged ? bm : b;
        } else {
          const bool z = (b == T(0)) & (c == T(0));
          dead |= z;
          cj[0] = c;
          bj[0] = z ? T(1) : b;
        }
      } else {
        const bool z = (b == T(0)) & (c == T(0));
        dead |= z;
        cj[j] = c;
        bj[j] = z ? T(1) : b;
      }
    }
    if (dead) val = T(0);
    // LS > 1: the triangle row offset of slot j + q (-1: its pairs are not
    // stored), where q is the lane's place in its group, chosen once per path
    // so that each lane reads its own pairs' entries with static indices
    // (lane q adds the pairs k = kb + q + LS v of each group of four)
    int rbs[C];
    if constexpr (LS > 1) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        rbs[j] = inr[j] ? rb[j] : -1;
#pragma unroll
        for (int g = 1; g < LS; ++g)
          rbs[j] = q == g ? (j + g < C && inr[j + g] ? rb[j + g] : -1) : rbs[j];
      }
    }
    const bool live = val != T(0);

    if constexpr (!MERGE) {
      // every slot sorted by feature and divided by: H = prod_j F_j,
      // g_i = w val H r_i
#pragma unroll
      for (int pass = 0; pass < NP; ++pass) {
        const int m0 = pass * NH;
        T H[NH];
#pragma unroll
        for (int m = 0; m < NH; ++m) H[m] = T(1);
        T r[C][NH];
#pragma unroll
        for (int j = 0; j < C; ++j) {
#pragma unroll
          for (int m = 0; m < NH; ++m) {
            const T Fv = fmaP(LS == 1 ? nc.t[m0 + m] : tq[m0 + m], cj[j], bj[j]);
            H[m] *= Fv;
            r[j][m] = cj[j] * rcpP(Fv);
          }
        }
        T G[NH];
#pragma unroll
        for (int m = 0; m < NH; ++m) G[m] = (LS == 1 ? nc.w[m0 + m] : wq[m0 + m]) * val * H[m];
#pragma unroll
        for (int i = 0; i < C; ++i) {
          if (i < d && live) {
            T g[NH];
            T ph = T(0);
#pragma unroll
            for (int m = 0; m < NH; ++m) {
              g[m] = G[m] * r[i][m];
              ph += g[m];
            }
            const int fi = f[i];
            ph = group_sum<LS>(ph);
            if (with_phi && q == 0) lds_add(&phis[fi], (double)ph);
            // pairs (i, k > i) in groups of four: the four values are
            // computed into separate registers before their atomics issue, so
            // the LDS queue sees back-to-back atomics instead of one per
            // dependency chain (inert slots k >= d are not stored)
#pragma unroll
            for (int kb = i + 1; kb < C; kb += 4) {
              T pr[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int k = kb + u < C ? kb + u : 0;
                pr[u] = g[0] * r[k][0];
#pragma unroll
                for (int m = 1; m < NH; ++m) pr[u] = fmaP(g[m], r[k][m], pr[u]);
              }
              if constexpr (LS == 1) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const int k = kb + u < C ? kb + u : 0;
                  if (kb + u < C && inr[k]) lds_add(&tris[rb[k] + fi], (double)pr[u]);
                }
              } else {
                group_add_own<LS, C>(tris, pr, rbs, kb, fi, q);
              }
            }
          }
        }
      }
      continue;
    }
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const int m0 = pass * NH;
      T H0[NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) H0[m] = T(1);
      T r[C][NH];
#pragma unroll
      for (int j = 1; j < C; ++j) {
#pragma unroll
        for (int m = 0; m < NH; ++m) {
          const T Fv = fmaP(LS == 1 ? nc.t[m0 + m] : tq[m0 + m], cj[j], bj[j]);
          H0[m] *= Fv;
          r[j][m] = cj[j] * rcpP(Fv);
        }
      }
      // G = w val H0; slot 0: g_0 = G c_0; slots i >= 1: g_i = (G F_0) r_i
      T G[NH], GF[NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) {
        G[m] = (LS == 1 ? nc.w[m0 + m] : wq[m0 + m]) * val * H0[m];
        GF[m] = G[m] * fmaP(LS == 1 ? nc.t[m0 + m] : tq[m0 + m], cj[0], bj[0]);
      }

      if (live) {
        // slot 0 and its pairs (0, k): the pair's larger feature gives the row
        {
          T g[NH];
          T ph = T(0);
#pragma unroll
          for (int m = 0; m < NH; ++m) {
            g[m] = G[m] * cj[0];
            ph += g[m];
          }
          const int f0 = f[0];
          const int rb0 = rb[0];
          ph = group_sum<LS>(ph);
          if (with_phi && q == 0) lds_add(&phis[f0], (double)ph);
#pragma unroll
          for (int kb = 1; kb < C; kb += 4) {
            T pr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k = kb + u < C ? kb + u : 1;
              pr[u] = g[0] * r[k][0];
#pragma unroll
              for (int m = 1; m < NH; ++m) pr[u] = fmaP(g[m], r[k][m], pr[u]);
            }
            int idx[4];
            bool ok[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k = kb + u < C ? kb + u : 1;
              // without merged rows every slot is sorted: f0 < f[k]
              const bool lo0 = MERGE ? f0 < f[k] : true;
              idx[u] = lo0 ? rb[k] + f0 : rb0 + f[k];
              const bool in = MERGE ? (((lo0 ? f[k] : f0) >= r0) & ((lo0 ? f[k] : f0) < r1) &
                                       (k < d))
                                    : inr[k];
              ok[u] = kb + u < C && in;
            }
            group_add<LS>(tris, pr, idx, ok, q);
          }
        }
#pragma unroll
        for (int i = 1; i < C; ++i) {
          if (i < d) {
            T g[NH];
            T ph = T(0);
#pragma unroll
            for (int m = 0; m < NH; ++m) {
              g[m] = GF[m] * r[i][m];
              ph += g[m];
            }
            const int fi = f[i];
            ph = group_sum<LS>(ph);
            if (with_phi && q == 0) lds_add(&phis[fi], (double)ph);
            // pairs (i, k > i) in groups of four: the four values are
            // computed into separate registers before their atomics issue, so
            // the LDS queue sees back-to-back atomics instead of one per
            // dependency chain (inert slots k >= d are not stored)
#pragma unroll
            for (int kb = i + 1; kb < C; kb += 4) {
              T pr[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int k = kb + u < C ? kb + u : 1;
                pr[u] = g[0] * r[k][0];
#pragma unroll
                for (int m = 1; m < NH; ++m) pr[u] = fmaP(g[m], r[k][m], pr[u]);
              }
              if constexpr (LS == 1) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const int k = kb + u < C ? kb + u : 1;
                  if (kb + u < C && inr[k]) lds_add(&tris[rb[k] + fi], (double)pr[u]);
                }
              } else {
                int idx[4];
                bool ok[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const int k = kb + u < C ? kb + u : 1;
                  idx[u] = rb[k] + fi;
                  ok[u] = kb + u < C && inr[k];
                }
                group_add<LS>(tris, pr, idx, ok, q);
              }
            }
          }
        }
      }
    }
  }
  // output row of (sample s, group grp): the accumulators are [M][ng][...]
  pairs_epilogue(phis, tris, ntri_r, base0, ntri, with_phi != 0, s * ng + grp, F, tri64, phi64);
}

// Generic form for long paths (any capacity up to 64): one wavefront per
// path.  Lane j owns slot j (o_j, c_j, F_j(m), r_j(m) = c_j / F_j(m)); the
// node products H(m) are reduced across lanes; each lane then leaves
// g_j(m) = w val H(m) r_j(m), r_j(m), its feature and its triangle row offset
// in the wave's LDS area, and the wave's lanes take the d(d-1)/2 pairs of the
// path in turn: pair q -> (i, k) from a table built once per workgroup, then
// SII_ik += sum_m g_i(m) r_k(m) from two 8-wide vector reads.
constexpr int kPairTable = kMaxUnique * (kMaxUnique - 1) / 2;  // 2016 pairs of <= 64 slots

template <typename T>
struct Vec2;
template <>
struct Vec2<float> { using type = float4; static constexpr int n = 4; };
template <>
struct Vec2<double> { using type = double2; static constexpr int n = 2; };

// Eight consecutive values from 16-byte aligned LDS.
template <typename T>
__device__ __forceinline__ void lds_load8(const T* p, T* out) {
  using V = typename Vec2<T>::type;
  constexpr int n = Vec2<T>::n;
  const V* v = reinterpret_cast<const V*>(p);
#pragma unroll
  for (int q = 0; q < 8 / n; ++q) {
    const V w = v[q];
    if constexpr (n == 4) {
      out[4 * q + 0] = w.x; out[4 * q + 1] = w.y; out[4 * q + 2] = w.z; out[4 * q + 3] = w.w;
    } else {
      out[2 * q + 0] = w.x; out[2 * q + 1] = w.y;
    }
  }
}

// LDS bytes of the generic kernel between the triangle and the sample row
// (pair table, padding to 16 bytes, per-wave slot areas), for nw waves.
__host__ __device__ constexpr size_t generic_mid_lds(int nw, size_t tsize) {
  return (size_t)kPairTable * 2 + 16 + (size_t)nw * 64 * (2 * kNodes * tsize + 2 * sizeof(int));
}

template <typename T>
__global__ void __launch_bounds__(256)
pairs_generic_kernel(const int32_t* __restrict__ pd, const int32_t* __restrict__ pleaf,
                     const int32_t* __restrict__ feat, const float* __restrict__ lo,
                     const float* __restrict__ hi, const T* __restrict__ bb,
                     const T* __restrict__ cbb, int32_t np, int32_t chunk,
                     const double* __restrict__ leaf_val, const float* __restrict__ X, int64_t M,
                     int64_t ldx, int32_t F, int32_t r0, int32_t r1, int32_t with_phi,
                     int32_t ng, int32_t grp, double* __restrict__ tri64,
                     double* __restrict__ phi64, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t ntri = tri_row(F + 1) - F;
  const int64_t base0 = tri_row(r0);
  const int64_t ntri_r = tri_row(r1) - base0;
  const int nw = blockDim.x >> 6;
  double* phis = reinterpret_cast<double*>(smem);  // [F]
  double* tris = phis + F;                         // [ntri_r]
  size_t off = (size_t)(F + ntri_r) * sizeof(double);
  uint16_t* ptab = reinterpret_cast<uint16_t*>(smem + off);  // [kPairTable]: k << 8 | i
  off = (off + (size_t)kPairTable * 2 + 15) & ~(size_t)15;
  T* gall = reinterpret_cast<T*>(smem + off);      // [nw][64][8]
  off += (size_t)nw * 64 * kNodes * sizeof(T);
  T* rall = reinterpret_cast<T*>(smem + off);      // [nw][64][8]
  off += (size_t)nw * 64 * kNodes * sizeof(T);
  int* fall = reinterpret_cast<int*>(smem + off);  // [nw][64] feature
  off += (size_t)nw * 64 * sizeof(int);
  int* rball = reinterpret_cast<int*>(smem + off); // [nw][64] row offset, -1: out of range
  off += (size_t)nw * 64 * sizeof(int);
  float* xrow = reinterpret_cast<float*>(smem + off);  // [F]

  const int64_t s = (int64_t)blockIdx.x % M;
  const int ch = (int)((int64_t)blockIdx.x / M);
  const int p0 = ch * chunk;
  const int p1 = min(np, p0 + chunk);
  // pair q -> (i < k) with k(k-1)/2 <= q < k(k+1)/2
  for (int q = threadIdx.x; q < kPairTable; q += blockDim.x) {
    int k = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
    while (k * (k - 1) / 2 > q) --k;
    while ((k + 1) * k / 2 <= q) ++k;
    ptab[q] = (uint16_t)((k << 8) | (q - k * (k - 1) / 2));
  }
  pairs_prologue(phis, tris, ntri_r, xrow, X, s, ldx, F);  // ends with a barrier

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  T* gw = gall + (size_t)wave * 64 * kNodes;
  T* rw = rall + (size_t)wave * 64 * kNodes;
  int* fw = fall + wave * 64;
  int* rbw = rball + wave * 64;
  for (int p = p0 + wave; p < p1; p += nw) {
    const int d = pd[p];
    const T val = (T)leaf_val[pleaf[p]];
    T Fv[kNodes], r[kNodes];
    bool z = false;
    int f = 0;
    if (lane < d) {
      const int64_t e = (int64_t)lane * np + p;
      const int fm = feat[e];
      const float lov = lo[e], hiv = hi[e];
      const T b = bb[e], cb = cbb[e];
      f = fm & kFeatureMask;
      const float x = xrow[f];
      const bool miss = (fm & kMissingOkBit) != 0;
      const bool lower = miss ? !(x < lov) : (x >= lov);
      const bool upper = !(x >= hiv);
      const T c = (lower & upper) ? cb : -b;
      z = (b == T(0)) & (c == T(0));
      const T bz = z ? T(1) : b;
#pragma unroll
      for (int m = 0; m < kNodes; ++m) {
        Fv[m] = fmaP(nc.t[m], c, bz);
        r[m] = c * rcpP(Fv[m]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < kNodes; ++m) {
        Fv[m] = T(1);
        r[m] = T(0);
      }
    }
    // a factor that vanishes at every node zeroes the whole path
    if (__any(z) || val == T(0)) continue;
    // H(m) = prod over the lanes' factors (lanes >= d hold 1)
#pragma unroll
    for (int m = 0; m < kNodes; ++m) Fv[m] = wave_prod(Fv[m]);
    T ph = T(0);
    if (lane < d) {
#pragma unroll
      for (int m = 0; m < kNodes; ++m) {
        const T g = nc.w[m] * val * Fv[m] * r[m];
        ph += g;
        gw[lane * kNodes + m] = g;
        rw[lane * kNodes + m] = r[m];
      }
      fw[lane] = f;
      rbw[lane] = (f >= r0 && f < r1) ? (int)(tri_row(f) - base0) : -1;
      if (with_phi) lds_add(&phis[f], (double)ph);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int npair = d * (d - 1) / 2;
    for (int q = lane; q < npair; q += 64) {
      const int e = ptab[q];
      const int i = e & 0xFF, k = e >> 8;
      const int rbk = rbw[k];
      if (rbk < 0) continue;
      T gi[kNodes], rk[kNodes];
      lds_load8(gw + i * kNodes, gi);
      lds_load8(rw + k * kNodes, rk);
      T pr = gi[0] * rk[0];
#pragma unroll
      for (int m = 1; m < kNodes; ++m) pr = fmaP(gi[m], rk[m], pr);
      lds_add(&tris[rbk + fw[i]], (double)pr);
    }
    // the next path overwrites this wave's slot areas
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  pairs_epilogue(phis, tris, ntri_r, base0, ntri, with_phi != 0, s * ng + grp, F, tri64, phi64);
}

// Third-order Shapley interaction indices (Theorem 1 with |S| = 3, Eq. 9-10,
// 8 nodes), per sample, into a packed tensor: the triple of features
// x < y < z sits at z(z-1)(z-2)/6 + y(y-1)/2 + x.
//
// A row of the pair table (slot 0 possibly the combined factor of a merged
// pair of sibling leaves, as above) with factors F_j(m) = b_j + t_m c_j and
// H0(m) = prod_{j >= 1} F_j(m), G(m) = w_m val H0(m):
//   g_0(m) = G(m) c_0,   g_j(m) = G(m) F_0(m) r_j(m),   r_j = c_j / F_j  (j >= 1)
//   SII_{abc} += sum_m g_a(m) r_b(m) r_c(m)   for slots a < b < c,
// so slot 0 is never divided by.  A slot j >= 1 with b_j = o_j = 0 zeroes the
// row, which is skipped.  One wavefront per row, lane j on slot j; for each
// largest slot c (uniform over the wave) the lanes take the pairs a < b < c
// from the pair table in LDS.  The sample's triples whose largest feature
// lies in [r0, r1) accumulate in LDS in FP64 and are flushed with FP64
// atomics into acc[M][F(F-1)(F-2)/6].
__host__ __device__ __forceinline__ int64_t tet_row(int64_t z) { return z * (z - 1) * (z - 2) / 6; }

template <typename T>
__device__ __forceinline__ T read_lane0(T v);
template <>
__device__ __forceinline__ float read_lane0<float>(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
}
template <>
__device__ __forceinline__ double read_lane0<double>(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 0);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 0);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// LDS bytes of the triples kernel besides the tensor range, for nw waves
// whose slot areas hold `cap` slots (the class capacity).
__host__ __device__ constexpr size_t triples_fixed_lds(int nw, int cap, size_t tsize, int F) {
  return (((size_t)cap * (cap - 1) + 15) & ~(size_t)15) +
         (size_t)nw * cap * (2 * kNodes * tsize + sizeof(int)) + (size_t)F * sizeof(float);
}

template <typename T>
__global__ void __launch_bounds__(1024)
triples_kernel(const int32_t* __restrict__ pd, const int32_t* __restrict__ pleaf,
               const SidePath* __restrict__ pside, const int32_t* __restrict__ feat,
               const float* __restrict__ lo, const float* __restrict__ hi,
               const T* __restrict__ bb, const T* __restrict__ cbb, int32_t np, int32_t cap,
               int32_t chunk,
               const double* __restrict__ leaf_val, const float* __restrict__ X, int64_t M,
               int64_t ldx, int32_t F, int32_t r0, int32_t r1, int32_t ng, int32_t grp,
               double* __restrict__ acc, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nw = blockDim.x >> 6;
  const int64_t nt = tet_row(F);
  const int64_t base0 = tet_row(r0);
  const int64_t nt_r = tet_row(r1) - base0;
  double* tets = reinterpret_cast<double*>(smem);  // [nt_r]
  size_t off = ((size_t)nt_r * sizeof(double) + 15) & ~(size_t)15;  // 16-byte areas follow
  // pairs of slots below the class capacity: cap(cap-1)/2 of them
  const int npt = cap * (cap - 1) / 2;
  uint16_t* ptab = reinterpret_cast<uint16_t*>(smem + off);  // [npt]: b << 8 | a
  off += ((size_t)npt * 2 + 15) & ~(size_t)15;
  T* gall = reinterpret_cast<T*>(smem + off);  // [nw][cap][8]
  off += (size_t)nw * cap * kNodes * sizeof(T);
  T* rall = reinterpret_cast<T*>(smem + off);  // [nw][cap][8]
  off += (size_t)nw * cap * kNodes * sizeof(T);
  int* fall = reinterpret_cast<int*>(smem + off);  // [nw][cap] feature
  off += (size_t)nw * cap * sizeof(int);
  float* xrow = reinterpret_cast<float*>(smem + off);  // [F]

  const int64_t s = (int64_t)blockIdx.x % M;
  const int ch = (int)((int64_t)blockIdx.x / M);
  const int p0 = ch * chunk;
  const int p1 = min(np, p0 + chunk);
  // pair q -> (a < b) with b(b-1)/2 <= q < b(b+1)/2
  for (int q = threadIdx.x; q < npt; q += blockDim.x) {
    int b = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
    while (b * (b - 1) / 2 > q) --b;
    while ((b + 1) * b / 2 <= q) ++b;
    ptab[q] = (uint16_t)((b << 8) | (q - b * (b - 1) / 2));
  }
  for (int i = threadIdx.x; i < F; i += blockDim.x) xrow[i] = X[s * ldx + i];
  for (int64_t e = threadIdx.x; e < nt_r; e += blockDim.x) tets[e] = 0.0;
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  T* gw = gall + (size_t)wave * cap * kNodes;
  T* rw = rall + (size_t)wave * cap * kNodes;
  int* fw = fall + wave * cap;
  for (int p = p0 + wave; p < p1; p += nw) {
    const int d = pd[p];  // <= cap
    if (d < 3) continue;
    const SidePath sp = pside[p];
    const bool merged = sp.leaf_b >= 0;
    const double va = leaf_val[pleaf[p]];
    const double vb = merged ? leaf_val[sp.leaf_b] : 0.0;
    const T val = merged ? T(1) : (T)va;
    T Fv[kNodes], r[kNodes];
    T c = T(0);
    bool z = false;
    int f = 0;
    if (lane < d) {
      const int64_t e = (int64_t)lane * np + p;
      const int fm = feat[e];
      const float lov = lo[e], hiv = hi[e];
      const T b = bb[e], cb = cbb[e];
      f = fm & kFeatureMask;
      const float x = xrow[f];
      const bool miss = (fm & kMissingOkBit) != 0;
      const bool lower = miss ? !(x < lov) : (x >= lov);
      const bool upper = !(x >= hiv);
      c = (lower & upper) ? cb : -b;
      T bz;
      if (lane == 0 && merged) {
        // combined slot-0 factor of the merged pair, in FP64, then rounded
        const T bm = (T)(va * sp.b_a + vb * sp.b_b);
        const T cAm = (T)(va * sp.cb_a - vb * sp.b_b);
        const T cBm = (T)(vb * sp.cb_b - va * sp.b_a);
        const bool lowerB = sp.mok_b ? !(x < sp.lo_b) : (x >= sp.lo_b);
        const bool upperB = !(x >= sp.hi_b);
        c = (lower & upper) ? cAm : ((lowerB & upperB) ? cBm : -bm);
        bz = bm;
      } else {
        z = (b == T(0)) & (c == T(0));
        bz = z ? T(1) : b;
      }
#pragma unroll
      for (int m = 0; m < kNodes; ++m) {
        Fv[m] = fmaP(nc.t[m], c, bz);
        r[m] = lane == 0 ? T(0) : c * rcpP(Fv[m]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < kNodes; ++m) {
        Fv[m] = T(1);
        r[m] = T(0);
      }
    }
    // a factor that vanishes at every node zeroes the whole row
    if (__any(z) || val == T(0)) continue;
    T H0[kNodes], F0[kNodes];
#pragma unroll
    for (int m = 0; m < kNodes; ++m) {
      F0[m] = read_lane0(Fv[m]);
      H0[m] = wave_prod(lane == 0 ? T(1) : Fv[m]);
    }
    if (lane < d) {
#pragma unroll
      for (int m = 0; m < kNodes; ++m) {
        const T G = nc.w[m] * val * H0[m];
        gw[lane * kNodes + m] = lane == 0 ? G * c : G * F0[m] * r[m];
        rw[lane * kNodes + m] = r[m];
      }
      fw[lane] = f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int cc = 2; cc < d; ++cc) {
      const int fc = fw[cc];
      // slots of an unmerged row are sorted by feature: the triples below
      // slot cc all have fc as their largest feature
      if (!merged && (fc < r0 || fc >= r1)) continue;
      T rc[kNodes];
      lds_load8(rw + cc * kNodes, rc);
      const int npair = cc * (cc - 1) / 2;
      for (int q = lane; q < npair; q += 64) {
        const int e = ptab[q];
        const int a = e & 0xFF, b = e >> 8;
        T ga[kNodes], rb[kNodes];
        lds_load8(gw + a * kNodes, ga);
        lds_load8(rw + b * kNodes, rb);
        T v = ga[0] * rb[0] * rc[0];
#pragma unroll
        for (int m = 1; m < kNodes; ++m) v = fmaP(ga[m] * rb[m], rc[m], v);
        // the three features in increasing order (slot 0 of a merged row can
        // hold any feature; the other slots are sorted)
        const int fa = fw[a], fb = fw[b];
        const int x0 = min(fa, fb), x1 = max(fa, fb);
        const int zf = max(x1, fc), y = max(x0, min(x1, fc)), x = min(x0, fc);
        if (x < y && y < zf && zf >= r0 && zf < r1)
          lds_add(&tets[tet_row(zf) - base0 + (int64_t)y * (y - 1) / 2 + x], (double)v);
      }
    }
    // the next row overwrites this wave's slot areas
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  const int64_t orow = s * ng + grp;  // acc is [M][ng][F(F-1)(F-2)/6]
  for (int64_t e = threadIdx.x; e < nt_r; e += blockDim.x) {
    const double v = tets[e];
    if (v != 0.0) unsafeAtomicAdd(&acc[orow * nt + base0 + e], v);
  }
}

// Lane-per-row form of triples_kernel for the short classes (capacity C <= 8):
// lane = row (slot-major table: a wave's 64 rows load coalesced), the row's
// factors and ratios in registers, its C(C,3) triples unrolled, with the same
// H0 form and the same LDS tensor range and flush.
template <typename T, int C>
__global__ void __launch_bounds__(512)
triples_lane_kernel(const int32_t* __restrict__ pd, const int32_t* __restrict__ pleaf,
                    const SidePath* __restrict__ pside, const int32_t* __restrict__ feat,
                    const float* __restrict__ lo, const float* __restrict__ hi,
                    const T* __restrict__ bb, const T* __restrict__ cbb, int32_t np,
                    int32_t chunk, const double* __restrict__ leaf_val, const float* __restrict__ X,
                    int64_t M, int64_t ldx, int32_t F, int32_t r0, int32_t r1, int32_t ng,
                    int32_t grp, double* __restrict__ acc, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t nt = tet_row(F);
  const int64_t base0 = tet_row(r0);
  const int64_t nt_r = tet_row(r1) - base0;
  double* tets = reinterpret_cast<double*>(smem);  // [nt_r]
  float* xrow = reinterpret_cast<float*>(smem + (((size_t)nt_r * sizeof(double) + 15) & ~(size_t)15));

  const int64_t s = (int64_t)blockIdx.x % M;
  const int ch = (int)((int64_t)blockIdx.x / M);
  const int p0 = ch * chunk;
  const int p1 = min(np, p0 + chunk);
  for (int i = threadIdx.x; i < F; i += blockDim.x) xrow[i] = X[s * ldx + i];
  for (int64_t e = threadIdx.x; e < nt_r; e += blockDim.x) tets[e] = 0.0;
  __syncthreads();

  for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
    const int d = pd[p];
    if (d < 3) continue;
    const SidePath sp = pside[p];
    const bool merged = sp.leaf_b >= 0;
    const double va = leaf_val[pleaf[p]];
    const double vb = merged ? leaf_val[sp.leaf_b] : 0.0;
    const T val = merged ? T(1) : (T)va;
    int f[C];
    T cj[C], bj[C];
    bool dead = false;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int64_t e = (int64_t)j * np + p;
      const int fm = feat[e];
      const T b = bb[e];
      f[j] = fm & kFeatureMask;
      const float x = xrow[f[j]];
      const bool miss = (fm & kMissingOkBit) != 0;
      const bool lower = miss ? !(x < lo[e]) : (x >= lo[e]);
      const bool upper = !(x >= hi[e]);
      T c = (lower & upper) ? cbb[e] : -b;
      if (j == 0 && merged) {
        const T bm = (T)(va * sp.b_a + vb * sp.b_b);
        const T cAm = (T)(va * sp.cb_a - vb * sp.b_b);
        const T cBm = (T)(vb * sp.cb_b - va * sp.b_a);
        const bool lowerB = sp.mok_b ? !(x < sp.lo_b) : (x >= sp.lo_b);
        const bool upperB = !(x >= sp.hi_b);
        cj[0] = (lower & upper) ? cAm : ((lowerB & upperB) ? cBm : -bm);
        bj[0] = bm;
      } else {
        // inert slots (j >= d) hold b = 1, c = 0: a factor of 1
        const bool z = (b == T(0)) & (c == T(0));
        dead |= z;
        cj[j] = c;
        bj[j] = z ? T(1) : b;
      }
    }
    if (dead || val == T(0)) continue;
    T GF[kNodes], G[kNodes], r[C][kNodes];
#pragma unroll
    for (int m = 0; m < kNodes; ++m) {
      T h = T(1);
#pragma unroll
      for (int j = 1; j < C; ++j) {
        const T Fv = fmaP(nc.t[m], cj[j], bj[j]);
        h *= Fv;
        r[j][m] = cj[j] * rcpP(Fv);
      }
      G[m] = nc.w[m] * val * h;
      GF[m] = G[m] * fmaP(nc.t[m], cj[0], bj[0]);
    }
#pragma unroll
    for (int c = 2; c < C; ++c) {
      // an unmerged row's slots are sorted: f[c] is the largest feature of
      // every triple below slot c
      if (c < d && (merged || (f[c] >= r0 && f[c] < r1))) {
#pragma unroll
        for (int b = 1; b < c; ++b) {
#pragma unroll
          for (int a = 0; a < b; ++a) {
            T v;
            if (a == 0) {
              T t = G[0] * r[b][0] * r[c][0];
#pragma unroll
              for (int m = 1; m < kNodes; ++m) t = fmaP(G[m] * r[b][m], r[c][m], t);
              v = cj[0] * t;
            } else {
              v = GF[0] * r[a][0] * r[b][0] * r[c][0];
#pragma unroll
              for (int m = 1; m < kNodes; ++m) v = fmaP(GF[m] * r[a][m] * r[b][m], r[c][m], v);
            }
            const int x0 = min(f[a], f[b]), x1 = max(f[a], f[b]);
            const int zf = max(x1, f[c]), y = max(x0, min(x1, f[c])), x = min(x0, f[c]);
            if (x < y && y < zf && zf >= r0 && zf < r1)
              lds_add(&tets[tet_row(zf) - base0 + (int64_t)y * (y - 1) / 2 + x], (double)v);
          }
        }
      }
    }
  }
  __syncthreads();
  const int64_t orow = s * ng + grp;
  for (int64_t e = threadIdx.x; e < nt_r; e += blockDim.x) {
    const double v = tets[e];
    if (v != 0.0) unsafeAtomicAdd(&acc[orow * nt + base0 + e], v);
  }
}

// out[i] = (float)acc[i]
__global__ void __launch_bounds__(256)
narrow_kernel(const double* __restrict__ acc, int64_t n, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)acc[i];
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

constexpr int kGenericThreads = 256;

// LDS bytes besides the triangle rows: the FP64 phi row, the sample row and,
// for the generic kernel, the pair table and each wave's slot areas.
size_t pairs_fixed_lds(int F, size_t tsize, bool generic) {
  size_t b = (size_t)F * sizeof(double) + (size_t)F * sizeof(float);
  if (generic) b += generic_mid_lds(kGenericThreads / 64, tsize);
  return b;
}

int64_t tri_row_h(int64_t k) { return k * (k - 1) / 2; }

// Cut the triangle rows [0, F) into ranges whose FP64 entries fit in
// `budget` bytes of LDS (row k holds k entries).
std::vector<std::pair<int, int>> row_ranges(int F, size_t budget) {
  std::vector<std::pair<int, int>> out;
  const int64_t cap = (int64_t)(budget / sizeof(double));
  if (cap < F) fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
  int r0 = 0;
  while (r0 < F) {
    int r1 = r0 + 1;
    while (r1 < F && tri_row_h(r1 + 1) - tri_row_h(r0) <= cap) ++r1;
    out.emplace_back(r0, r1);
    r0 = r1;
  }
  return out;
}

int pair_chunk(int np, int64_t M, const PairShape& shape, int64_t* n_chunks_out) {
  // chunks of at most max_chunk paths, and at least `fill` work items when
  // there are few samples (chunks of no fewer than 1024 paths)
  const int64_t max_chunk = std::max(1024, shape.max_chunk);
  int64_t n_chunks = (np + max_chunk - 1) / max_chunk;
  const int64_t fill = (std::max(1, shape.fill) + M - 1) / M;
  n_chunks = std::max<int64_t>(n_chunks, std::min<int64_t>(fill, (np + 1023) / 1024));
  n_chunks = std::max<int64_t>(1, n_chunks);
  *n_chunks_out = n_chunks;
  return (int)((np + n_chunks - 1) / n_chunks);
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
NodeConsts<T> node_consts(const DeviceTable& d, int n = 8) {
  if constexpr (std::is_same<T, float>::value)
    return n == 2 ? d.n32_2 : n == 4 ? d.n32_4 : n == 6 ? d.n32_6 : d.n32;
  else
    return n == 2 ? d.n64_2 : n == 4 ? d.n64_4 : n == 6 ? d.n64_6 : d.n64;
}

template <typename T, int C, int NH, bool MERGE, int NN = 8, int LS = 1>
void launch_pairs_fast(const HostTable& h, const DeviceTable& d, const PairClass& pc,
                       const float* X, int64_t M, int64_t ldx, const double* leaf_val,
                       double* tri64, double* phi64, const PairShape& shape, hipStream_t s) {
  const int F = h.F;
  int64_t n_chunks = 1;
  const int chunk = pair_chunk(pc.np, M, shape, &n_chunks);
  const int64_t grid = M * n_chunks;
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "interactions grid too large");
  const void* fn = (const void*)pairs_kernel<T, C, NH, MERGE, NN, LS>;
  const size_t limit = raise_lds_limit(fn);
  const size_t fixed = pairs_fixed_lds(F, sizeof(T), false);
  if (fixed >= limit) fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
  bool first = true;
  for (const auto& rg : row_ranges(F, limit - fixed)) {
    const size_t lds = fixed + (size_t)(tri_row_h(rg.second) - tri_row_h(rg.first)) * 8;
    hipLaunchKernelGGL((pairs_kernel<T, C, NH, MERGE, NN, LS>), dim3((unsigned)grid), dim3(512), lds, s,
                       d.pr_d + pc.pbase, d.pr_leaf + pc.pbase, d.pr_side + pc.pbase,
                       d.pr_feat + pc.base,
                       d.pr_lo + pc.base, d.pr_hi + pc.base, table_b<T>(d) + pc.base,
                       table_cb<T>(d) + pc.base, pc.np, chunk, leaf_val, X, M, ldx, F, rg.first,
                       rg.second, (int)first, h.n_groups, pc.group, tri64, phi64,
                       node_consts<T>(d, NN));
    check_hip(hipGetLastError(), "pairs_kernel launch");
    first = false;
  }
}

template <typename T>
void launch_pairs_generic(const HostTable& h, const DeviceTable& d, const PairClass& pc,
                          const float* X, int64_t M, int64_t ldx, const double* leaf_val,
                          double* tri64, double* phi64, const PairShape& shape, hipStream_t s) {
  const int F = h.F;
  int64_t n_chunks = 1;
  const int chunk = pair_chunk(pc.np, M, shape, &n_chunks);
  const int64_t grid = M * n_chunks;
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "interactions grid too large");
  const void* fn = (const void*)pairs_generic_kernel<T>;
  const size_t limit = raise_lds_limit(fn);
  const size_t fixed = pairs_fixed_lds(F, sizeof(T), true);
  if (fixed >= limit) fail(QTS_E_UNSUPPORTED, "n_features too large for the interactions kernel");
  bool first = true;
  for (const auto& rg : row_ranges(F, limit - fixed)) {
    const size_t lds = fixed + (size_t)(tri_row_h(rg.second) - tri_row_h(rg.first)) * 8;
    hipLaunchKernelGGL((pairs_generic_kernel<T>), dim3((unsigned)grid), dim3(kGenericThreads),
                       lds, s, d.pr_d + pc.pbase, d.pr_leaf + pc.pbase, d.pr_feat + pc.base,
                       d.pr_lo + pc.base, d.pr_hi + pc.base, table_b<T>(d) + pc.base,
                       table_cb<T>(d) + pc.base, pc.np, chunk, leaf_val, X, M, ldx, F, rg.first,
                       rg.second, (int)first, h.n_groups, pc.group, tri64, phi64,
                       node_consts<T>(d));
    check_hip(hipGetLastError(), "pairs_generic_kernel launch");
    first = false;
  }
}

template <typename T, int C>
void launch_triples_lane(const HostTable& h, const DeviceTable& d, const PairClass& pc,
                         const float* X, int64_t M, int64_t ldx, const double* leaf_val,
                         double* acc, hipStream_t s) {
  constexpr int kThreads = 512;
  const int F = h.F;
  const int64_t want = (2048 + M - 1) / M;
  const int64_t n_chunks = std::max<int64_t>(1, std::min<int64_t>(want, (pc.np + 511) / 512));
  const int chunk = (int)((pc.np + n_chunks - 1) / n_chunks);
  const int64_t grid = M * ((pc.np + chunk - 1) / chunk);
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "third-order grid too large");
  const void* fn = (const void*)triples_lane_kernel<T, C>;
  const size_t limit = raise_lds_limit(fn);
  const size_t fixed = (size_t)F * sizeof(float) + 16;  // the sample row and the alignment pad
  if (fixed >= limit) fail(QTS_E_UNSUPPORTED, "n_features too large for the third-order kernel");
  const int64_t cap = (int64_t)((limit - fixed) / sizeof(double));
  int r0 = 0;
  while (r0 < F) {
    int r1 = r0 + 1;
    if (tet_row(r1) - tet_row(r0) > cap)
      fail(QTS_E_UNSUPPORTED, "n_features too large for the third-order kernel");
    while (r1 < F && tet_row(r1 + 1) - tet_row(r0) <= cap) ++r1;
    const size_t lds =
        fixed + (((size_t)(tet_row(r1) - tet_row(r0)) * sizeof(double) + 15) & ~(size_t)15);
    hipLaunchKernelGGL((triples_lane_kernel<T, C>), dim3((unsigned)grid), dim3(kThreads), lds, s,
                       d.pr_d + pc.pbase, d.pr_leaf + pc.pbase, d.pr_side + pc.pbase,
                       d.pr_feat + pc.base, d.pr_lo + pc.base, d.pr_hi + pc.base,
                       table_b<T>(d) + pc.base, table_cb<T>(d) + pc.base, pc.np, chunk, leaf_val,
                       X, M, ldx, F, r0, r1, h.n_groups, pc.group, acc, node_consts<T>(d));
    check_hip(hipGetLastError(), "triples_lane_kernel launch");
    r0 = r1;
  }
}

template <typename T>
void launch_triples_t(const HostTable& h, const DeviceTable& d, const PairClass& pc,
                      const float* X, int64_t M, int64_t ldx, const double* leaf_val,
                      double* acc, hipStream_t s) {
  const int F = h.F;
  if (pc.np == 0) return;
  // short classes: one lane per row
  if (pc.cap == 4) return launch_triples_lane<T, 4>(h, d, pc, X, M, ldx, leaf_val, acc, s);
  if (pc.cap == 8) return launch_triples_lane<T, 8>(h, d, pc, X, M, ldx, leaf_val, acc, s);
  // slot areas sized by the class capacity: short classes take more waves,
  // but eight rather than sixteen where that lets the whole tensor fit in one
  // range (each range walks every row again; four waves measured slower than
  // two ranges)
  const size_t limit0 = raise_lds_limit((const void*)triples_kernel<T>);
  int threads = pc.cap <= 16 ? 1024 : pc.cap <= 32 ? 512 : 256;
  for (int t = threads; t >= 512; t /= 2) {
    const size_t fx = triples_fixed_lds(t / 64, pc.cap, sizeof(T), F);
    if (fx < limit0 && tet_row(F) <= (int64_t)((limit0 - fx) / sizeof(double)) - 1) {
      threads = t;
      break;
    }
  }
  // enough work items for the chip when there are few samples; chunks of no
  // fewer than 64 rows
  const int64_t want = (2048 + M - 1) / M;
  const int64_t n_chunks = std::max<int64_t>(1, std::min<int64_t>(want, (pc.np + 63) / 64));
  const int chunk = (int)((pc.np + n_chunks - 1) / n_chunks);
  const int64_t grid = M * ((pc.np + chunk - 1) / chunk);
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "third-order grid too large");
  const void* fn = (const void*)triples_kernel<T>;
  const size_t limit = raise_lds_limit(fn);
  const size_t fixed = triples_fixed_lds(threads / 64, pc.cap, sizeof(T), F);
  if (fixed >= limit) fail(QTS_E_UNSUPPORTED, "n_features too large for the third-order kernel");
  const int64_t cap = (int64_t)((limit - fixed) / sizeof(double)) - 1;  // less the alignment pad
  // ranges of the largest feature z; z holds z(z-1)/2 triples
  int r0 = 0;
  while (r0 < F) {
    int r1 = r0 + 1;
    if (tet_row(r1) - tet_row(r0) > cap)
      fail(QTS_E_UNSUPPORTED, "n_features too large for the third-order kernel");
    while (r1 < F && tet_row(r1 + 1) - tet_row(r0) <= cap) ++r1;
    const size_t lds =
        fixed + (((size_t)(tet_row(r1) - tet_row(r0)) * sizeof(double) + 15) & ~(size_t)15);
    hipLaunchKernelGGL((triples_kernel<T>), dim3((unsigned)grid), dim3(threads), lds, s,
                       d.pr_d + pc.pbase, d.pr_leaf + pc.pbase, d.pr_side + pc.pbase,
                       d.pr_feat + pc.base, d.pr_lo + pc.base, d.pr_hi + pc.base,
                       table_b<T>(d) + pc.base, table_cb<T>(d) + pc.base, pc.np, pc.cap, chunk,
                       leaf_val, X, M, ldx, F, r0, r1, h.n_groups, pc.group, acc,
                       node_consts<T>(d));
    check_hip(hipGetLastError(), "triples_kernel launch");
    r0 = r1;
  }
}

}  // namespace

void launch_pairs(const HostTable& h, const DeviceTable& d, const PairClass& pc, bool fp64,
                  const float* X, int64_t M, int64_t ldx, const double* lv, double* tri64,
                  double* phi64, const PairShape& sh, bool nodes_exact, hipStream_t s) {
  // the fewest nodes exact for the class (pair integrands of degree <= C - 2,
  // first-order ones of degree <= C - 1: n = C / 2)
  if (nodes_exact && pc.cap <= 12) {
    if (!fp64) {
      switch (pc.cap) {
        case 4: return launch_pairs_fast<float, 4, 2, true, 2>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
        case 8: return launch_pairs_fast<float, 8, 4, true, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
        default: return launch_pairs_fast<float, 12, 6, true, 6>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      }
    }
    switch (pc.cap) {
      case 4: return launch_pairs_fast<double, 4, 2, true, 2>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 8: return launch_pairs_fast<double, 8, 4, true, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      default: return launch_pairs_fast<double, 12, 3, true, 6>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    }
  }
  // register-resident instances exist where they do not spill.  Up to FP32
  // C = 20 and FP64 C = 8 a lane holds all eight nodes.  FP64 C = 12 and 16
  // take two node passes (one pass on two lanes measured slower: the FP64
  // selects and swaps cost more VALU time than the atomics they save), FP64
  // C = 20 two lanes and two passes (half the atomics of four passes on one
  // lane).  Longer classes take two or four lanes per path, which beats the
  // wave-per-path generic kernel; the longest (FP32 64, FP64 36 and up, which
  // would spill) run the generic kernel
  if (!fp64) {
    switch (pc.cap) {
      case 4: return launch_pairs_fast<float, 4, 8, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 8: return launch_pairs_fast<float, 8, 8, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 12: return launch_pairs_fast<float, 12, 8, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 16: return launch_pairs_fast<float, 16, 8, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 20: return launch_pairs_fast<float, 20, 8, false>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 24: return launch_pairs_fast<float, 24, 4, false, 8, 2>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 28: return launch_pairs_fast<float, 28, 4, false, 8, 2>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 32: return launch_pairs_fast<float, 32, 2, false, 8, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 36: return launch_pairs_fast<float, 36, 2, false, 8, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 40: return launch_pairs_fast<float, 40, 2, false, 8, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      case 48: return launch_pairs_fast<float, 48, 2, false, 8, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
      default: return launch_pairs_generic<float>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    }
  }
  switch (pc.cap) {
    case 4: return launch_pairs_fast<double, 4, 8, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    case 8: return launch_pairs_fast<double, 8, 8, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    case 12: return launch_pairs_fast<double, 12, 4, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    case 16: return launch_pairs_fast<double, 16, 4, true>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    case 20: return launch_pairs_fast<double, 20, 2, false, 8, 2>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    case 24: return launch_pairs_fast<double, 24, 2, false, 8, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    case 28: return launch_pairs_fast<double, 28, 2, false, 8, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    case 32: return launch_pairs_fast<double, 32, 2, false, 8, 4>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
    default: return launch_pairs_generic<double>(h, d, pc, X, M, ldx, lv, tri64, phi64, sh, s);
  }
}

void launch_triples(const HostTable& h, const DeviceTable& d, const PairClass& pc, bool fp64,
                    const float* X, int64_t M, int64_t ldx, const double* lv, double* acc,
                    hipStream_t s) {
  if (fp64) launch_triples_t<double>(h, d, pc, X, M, ldx, lv, acc, s);
  else launch_triples_t<float>(h, d, pc, X, M, ldx, lv, acc, s);
}

void launch_narrow_f64_f32(const double* acc, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(narrow_kernel, dim3(grid), dim3(256), 0, s, acc, n, out);
  check_hip(hipGetLastError(), "narrow_kernel launch");
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
