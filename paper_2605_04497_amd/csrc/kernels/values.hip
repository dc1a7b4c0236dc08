// First-order Shapley values: phi[s, f] accumulated over every root-to-leaf
// path of the ensemble (Theorem 1 with |S| = 1, Eq. 9-10, 8 nodes), and the
// adjoint of phi with respect to the leaf values.
//
// Work mapping (gfx950, wave64):
//   * a workgroup owns a tile of 64 explained samples (one per lane) and a
//     contiguous chunk of rows from one bucket; its wavefronts split the
//     chunk (rows of at most 8 features: one contiguous run per wavefront;
//     longer rows: row by row in turn);
//   * a wavefront processes one row at a time for all 64 samples, so every
//     row quantity (features, bounds, b_j, 1-b_j, slot-0 factor) is uniform
//     across the wave and is fetched with scalar loads;
//   * the sample tile is staged transposed in LDS ([F][65] floats), so the
//     per-lane gather x[s, f_j] is a conflict-free LDS read;
//   * contributions are added into an FP64 LDS accumulator ([F][65] doubles,
//     shared by the workgroup's waves) and flushed to the FP64 global
//     accumulator with one atomic per (sample, feature) at the end.
//
// Per (sample, row) with unique features j = 0..d-1 and nodes m:
//   o_j    = x in [lo_j, hi_j) ? 1 : 0   (NaN: missing_ok_j)            (Eq. 2)
//   c_j    = o_j - b_j, taken as the stored FP64-derived 1 - b_j or as -b_j
//   F_j(m) = b_j (1 - t_m) + o_j t_m = b_j + t_m c_j      (one FMA per node)
//   LOO_j  = sum_m w_m prod_{k != j} F_k(m)    by prefix x suffix products
//   phi[s, f_j] += val c_j LOO_j
// The leaf value is folded into slot 0 (Slot0: F_0 scaled by val, built per
// call in FP64), so a row needs no multiply by val; a merged sibling pair is
// the same form with a combined slot-0 factor.
// Rows of at most 8 features reuse the factors and prefix products of the
// slots they share with the previous row (values_rows_shared,
// adjoint_rows_shared).  Longer rows (values_rows_long, values_paths) run in
// batches of eight slots: slots past the end of a row get c = 0 and b = 1, a
// factor of exactly 1, so whole batches run without
// branches; the prefix products are kept only at batch checkpoints and
// rebuilt batch by batch in the backward sweep, which bounds the registers;
// NH < NN splits the nodes over several passes (the node sum is additive).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "../qts_device.h"

namespace qts {

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// Copy a wave-uniform value into a VGPR the compiler cannot fold back.
__device__ __forceinline__ float to_vgpr(float v) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
  return r;
}
__device__ __forceinline__ double to_vgpr(double v) {
  double r;
  asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "s"(v));
  return r;
}

// Node m and weight m of the 8-node rule in the walks that hold all 8 nodes
// in one pass: FP32 takes them as instruction literals, FP64 from the kernel
// argument (an FP32 FMA or multiply reading a scalar register issues at about
// half the rate of one with a literal or vector operands; FP64 shows no such
// difference).
template <typename T>
__device__ __forceinline__ T node8_t(const NodeConsts<T>& nc, int m) {
  if constexpr (sizeof(T) == 4) return rule8_t32(m);
  else return nc.t[m];
}
template <typename T>
__device__ __forceinline__ T node8_w(const NodeConsts<T>& nc, int m) {
  if constexpr (sizeof(T) == 4) return rule8_w32(m);
  else return nc.w[m];
}

// Add a row's leaf-value gradient, summed over the wave's 64 samples.  det:
// grad_leaf is this sample block's own row of partial sums, and every leaf
// belongs to one row, so a plain store suffices (and keeps the result
// independent of scheduling).
__device__ __forceinline__ void leaf_add(double* grad_leaf, int leaf, double v, bool det) {
  if (det) grad_leaf[leaf] = v;
  else if (v != 0.0) unsafeAtomicAdd(&grad_leaf[leaf], v);
}

// The path loop of one workgroup.  NANS: the tile holds a NaN, so the
// missing-value rule is evaluated; otherwise plain interval tests suffice.
// ADJ: adjoint mode.  phi is linear in the leaf value, so d phi[s, f_j] /
// d val = c_j LOO_j; instead of scattering val c_j LOO_j into the phi tile,
// each lane gathers g[s, f_j] c_j LOO_j from the upstream-gradient tile gs,
// the wave sums its 64 samples in FP64 (DPP reduction into lane 63) and adds
// the result to grad_leaf.
template <typename T, int DMAX, int NH, bool STORE_G, bool NANS, bool ADJ, int NN>
__device__ __forceinline__ void values_paths(
    const PathHdr* __restrict__ hdr, const int32_t* __restrict__ feat,
    const float* __restrict__ lo, const float* __restrict__ hi, const T* __restrict__ bb,
    const T* __restrict__ cbb, const SidePath* __restrict__ side,
    const Slot0<T>* __restrict__ z0, const float* xs, double* as, const T* gs,
    double* __restrict__ grad_leaf, int pb, int pe, int wave, int nw, int lane, const T* tv,
    const NodeConsts<T>& nc, bool det = false) {
  constexpr int NB = DMAX / 8;  // feature batches
  for (int p = pb + wave; p < pe; p += nw) {
    const int d = ldu(&hdr[p].d);
    const int off = ldu(&hdr[p].off);
    const int leaf = ldu(&hdr[p].leaf);
    // First order: slot 0 comes from Slot0 (leaf value folded in; the row's
    // own b_0, 1 - b_0 are not read).  Adjoint of a merged sibling pair:
    // slot 0 is the parent's split feature L, made inert in the products
    // (b = 1, c = 0), so the sweep yields w Q_j(m) = w prod_{k >= 1, k != j} F_k(m);
    // then
    //   d/dvA = sum_m F_A(m) R(m) + g_L c_A sum_m w Q_0(m),
    //   R(m) = sum_{j >= 1} g_j c_j w Q_j(m)   (shared by A and B),
    // and likewise for B with F_B and c_B.
    const int sidx = (!ADJ || side == nullptr) ? -1 : ldu(&hdr[p].tree);
    const bool merged = sidx >= 0;  // adjoint only
    const bool own0 = !ADJ || merged;  // slot 0 not taken from the row's elements
    T bm = T(0), cA = T(0), cB = T(0);
    T ba = T(0), cba = T(0), bb2 = T(0), cbb2 = T(0);
    float loB = 0.f, hiB = 0.f;
    bool mokB = false;
    int leafB = 0;
    if (!ADJ) {
      const Slot0<T>* z = z0 + p;
      bm = ldu(&z->bm);
      cA = ldu(&z->ca);
      cB = ldu(&z->cb);
      loB = ldu(&z->lo_b);
      hiB = ldu(&z->hi_b);
      mokB = ldu(&z->mok_b) != 0;
    } else if (merged) {
      const SidePath* sp = side + sidx;
      leafB = ldu(&sp->leaf_b);
      loB = ldu(&sp->lo_b);
      hiB = ldu(&sp->hi_b);
      mokB = ldu(&sp->mok_b) != 0;
      ba = (T)ldu(&sp->b_a);
      cba = (T)ldu(&sp->cb_a);
      bb2 = (T)ldu(&sp->b_b);
      cbb2 = (T)ldu(&sp->cb_b);
      bm = T(1);
    }
    // b_j of slot j (slot 0 of a merged path: bm)
    auto bload = [&](int j) -> T { return (j == 0 && own0) ? bm : ldu(bb + off + j); };
    double gacc = 0.0;
    double gaccB = 0.0;          // adjoint of a merged path: B's gradient
    T oc0A = T(0), oc0B = T(0);  // adjoint of a merged path: c_A and c_B
    T q0 = T(0);                 // adjoint of a merged path: sum_m w Q_0(m)
    const int nb = (d + 7) >> 3;  // batches in use; slots [d, 8 nb) are inert

    // c_j per slot, eight slots per batch
    T cf[DMAX];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < nb) {
        const int jb = 8 * b;
        int fm[8];
        float l[8], u[8], x[8];
        T bl[8], cbl[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          fm[k] = ldu(feat + off + jb + k);
          l[k] = ldu(lo + off + jb + k);
          u[k] = ldu(hi + off + jb + k);
          bl[k] = ldu(bb + off + jb + k);
          cbl[k] = ldu(cbb + off + jb + k);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = xs[(fm[k] & kFeatureMask) * kTileStride + lane];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          // hi = NaN (no upper bound) makes the upper compare true; a NaN x
          // passes the unordered lower compare iff missing_ok
          bool lower;
          if (NANS) {
            const bool miss = (fm[k] & kMissingOkBit) != 0;
            lower = miss ? !(x[k] < l[k]) : (x[k] >= l[k]);
          } else {
            lower = x[k] >= l[k];
          }
          const bool upper = !(x[k] >= u[k]);
          cf[jb + k] = (lower & upper) ? cbl[k] : -bl[k];
          if (b == 0 && k == 0 && own0) {
            bool lowerB;
            if (NANS) lowerB = mokB ? !(x[0] < loB) : (x[0] >= loB);
            else lowerB = x[0] >= loB;
            const bool upperB = !(x[0] >= hiB);
            if (ADJ) {
              oc0A = (lower & upper) ? cba : -ba;
              oc0B = (lowerB & upperB) ? cbb2 : -bb2;
              cf[0] = T(0);
            } else {
              cf[0] = (lower & upper) ? cA : ((lowerB & upperB) ? cB : -bm);
            }
          }
        }
      }
    }

#pragma unroll
    for (int pass = 0; pass < NN / NH; ++pass) {
      const int m0 = pass * NH;
      // checkpoints: ck[b][m] = w_m prod_{k < 8b} F_k(m)
      T ck[NB][NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) ck[0][m] = nc.w[m0 + m];
#pragma unroll
      for (int b = 1; b < NB; ++b) {
        if (b < nb) {
#pragma unroll
          for (int m = 0; m < NH; ++m) ck[b][m] = ck[b - 1][m];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int j = 8 * (b - 1) + k;
            const T bj = bload(j);
#pragma unroll
            for (int m = 0; m < NH; ++m) ck[b][m] *= fmaT(tv[m0 + m], cf[j], bj);
          }
        }
      }
      // backward sweep, last batch first: rebuild the batch's prefixes from
      // its checkpoint, then suffix products and leave-one-out sums
      T S[NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) S[m] = T(1);
      T R[ADJ ? NH : 1];
#pragma unroll
      for (int m = 0; m < (ADJ ? NH : 1); ++m) R[m] = T(0);
#pragma unroll
      for (int b = NB - 1; b >= 0; --b) {
        if (b < nb) {
          const int jb = 8 * b;
          T bj[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) bj[k] = bload(jb + k);
          T Pb[8][NH];
          T Gb[STORE_G ? 8 : 1][NH];
          T run[NH];
#pragma unroll
          for (int m = 0; m < NH; ++m) run[m] = ck[b][m];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int m = 0; m < NH; ++m) {
              const T g = fmaT(tv[m0 + m], cf[jb + k], bj[k]);
              Pb[k][m] = run[m];
              if (STORE_G) Gb[STORE_G ? k : 0][m] = g;
              run[m] *= g;
            }
          }
#pragma unroll
          for (int k = 7; k >= 0; --k) {
            const int j = jb + k;
            if (j < d) {
              const int f = ldu(feat + off + j) & kFeatureMask;
              if (ADJ && merged) {
                if (j > 0) {
                  const T gc = gs[f * kTileStride + lane] * cf[j];
#pragma unroll
                  for (int m = 0; m < NH; ++m)
                    R[ADJ ? m : 0] = fmaT(gc, Pb[k][m] * S[m], R[ADJ ? m : 0]);
                } else {
#pragma unroll
                  for (int m = 0; m < NH; ++m) q0 = fmaT(Pb[k][m], S[m], q0);
                }
              } else {
                T dot = Pb[k][0] * S[0];
#pragma unroll
                for (int m = 1; m < NH; ++m) dot = fmaT(Pb[k][m], S[m], dot);
                if (ADJ) {
                  gacc += (double)(gs[f * kTileStride + lane] * cf[j] * dot);
                } else {
                  const double c = (double)(cf[j] * dot);
                  __hip_atomic_fetch_add(&as[f * kTileStride + lane], c, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                }
              }
            }
            if (j > 0) {
#pragma unroll
              for (int m = 0; m < NH; ++m) {
                const T g = STORE_G ? Gb[STORE_G ? k : 0][m] : fmaT(tv[m0 + m], cf[j], bj[k]);
                S[m] *= g;
              }
            }
          }
        }
      }
      if (ADJ && merged) {
        T sa = T(0), sb = T(0);
#pragma unroll
        for (int m = 0; m < NH; ++m) {
          sa = fmaT(fmaT(tv[m0 + m], oc0A, ba), R[ADJ ? m : 0], sa);
          sb = fmaT(fmaT(tv[m0 + m], oc0B, bb2), R[ADJ ? m : 0], sb);
        }
        gacc += (double)sa;
        gaccB += (double)sb;
      }
    }
    if (ADJ) {
      if (merged) {
        const T gL = gs[(ldu(feat + off) & kFeatureMask) * kTileStride + lane];
        gacc += (double)(gL * oc0A * q0);
        gaccB += (double)(gL * oc0B * q0);
        gaccB = wave_sum_last(gaccB);
        if (lane == 63) leaf_add(grad_leaf, leafB, gaccB, det);
      }
      gacc = wave_sum_last(gacc);
      if (lane == 63) leaf_add(grad_leaf, leaf, gacc, det);
    }
  }
}


// Wide scalar loads of a ShortRow (dword-aligned vectors of 4 and 16 words).
typedef int32_t row_v4 __attribute__((ext_vector_type(4), aligned(4)));
typedef int32_t row_v8 __attribute__((ext_vector_type(8), aligned(4)));
typedef int32_t row_v16 __attribute__((ext_vector_type(16), aligned(4)));
static_assert(offsetof(ShortRow<float>, xoff) == 16 && offsetof(ShortRow<float>, lo) == 80 &&
                  offsetof(ShortRow<float>, b) == 144 && offsetof(ShortRow<float>, cb) == 176 &&
                  offsetof(ShortRow<double>, b) == 144 && offsetof(ShortRow<double>, cb) == 208,
              "ShortRow layout");

// A short row in registers (SGPRs: every field is wave-uniform).
template <typename T>
struct ShortRowRegs {
  int d, share, mok;
  int xo[8], ao[8];
  float l[8], u[8];
  T bl[8], cbl[8];
};

// The record of row p in four wide scalar loads, all issued before any is
// used.  AO = false leaves out the accumulator offsets (twice the sample
// tile's: the caller derives them where it adds, which saves 8 SGPRs).
template <typename T, bool AO = true>
__device__ __forceinline__ ShortRowRegs<T> load_short_row(const ShortRow<T>* rows, int row0,
                                                          int p) {
  ShortRowRegs<T> r;
  const int32_t* rw = reinterpret_cast<const int32_t*>(rows + (p - row0));
  const row_v4 hd = ldu(reinterpret_cast<const row_v4*>(rw));
  row_v16 of;
  if constexpr (AO) {
    of = ldu(reinterpret_cast<const row_v16*>(rw + 4));
  } else {
    const row_v8 o8 = ldu(reinterpret_cast<const row_v8*>(rw + 4));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      of[k] = o8[k];
      of[8 + k] = 2 * o8[k];
    }
  }
  const row_v16 bd = ldu(reinterpret_cast<const row_v16*>(rw + 20));
  if constexpr (sizeof(T) == 4) {
    const row_v16 bc = ldu(reinterpret_cast<const row_v16*>(rw + 36));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      r.bl[k] = __int_as_float(bc[k]);
      r.cbl[k] = __int_as_float(bc[8 + k]);
    }
  } else {
    const row_v16 b2 = ldu(reinterpret_cast<const row_v16*>(rw + 36));
    const row_v16 c2 = ldu(reinterpret_cast<const row_v16*>(rw + 52));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      r.bl[k] = __hiloint2double(b2[2 * k + 1], b2[2 * k]);
      r.cbl[k] = __hiloint2double(c2[2 * k + 1], c2[2 * k]);
    }
  }
  r.d = hd[0];
  r.share = hd[1];
  r.mok = hd[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    r.xo[k] = of[k];
    r.ao[k] = of[8 + k];
    r.l[k] = __int_as_float(bd[k]);
    r.u[k] = __int_as_float(bd[8 + k]);
  }
  return r;
}

// First order over rows of at most 8 features with all NH nodes in one pass,
// reusing work between consecutive rows.  Each wave walks a contiguous run of
// rows.  The products are taken over the slots in the order 1, 2, ..., 7, 0,
// so the prefix products and the factors F_j(m) of slots 1..s depend only on
// those slots; when slots 1..s of a row equal the previous row's (share[p] =
// s, from the host), their c_j, F_j(m) and prefix products are still in
// registers and only their suffix products and dot products are formed
// again.  Slot 0 (the row's own factor, from Slot0) and slots past s are
// evaluated as usual, each with the prefix product through it in the same
// step, so the shared count picks one entry into a single straight run of
// code; inert padding slots (b = 1, c = 0) give a factor of exactly 1.
template <typename T, int NH, bool NANS, bool KEEP = true>
__device__ __forceinline__ void values_rows_shared(
    const ShortRow<T>* __restrict__ rows, int row0, const Slot0<T>* __restrict__ z0,
    const float* xs, double* as, int pb, int pe, int wave, int nw, int lane, const T* tv,
    const NodeConsts<T>& nc) {
  constexpr bool kScalarT = NH == 8;
  const int run = (pe - pb + nw - 1) / nw;
  const int p_first = pb + wave * run;
  const int p_last = min(pe, p_first + run);
  T cf[8];       // c_j of the current row
  T G[8][NH];    // F_j(m) of the current row
  // prefix products in the order 1..7, 0: P[q] = w prod over the first q
  // slots of that order (slot q + 1 at position q); P[1..s] depend only on
  // shared slots and are kept from the previous row
  T P[7][NH];
#pragma unroll
  for (int m = 0; m < NH; ++m) P[0][m] = kScalarT ? node8_w(nc, m) : nc.w[m];
  const char* xl = reinterpret_cast<const char*>(xs + lane);
  char* al = reinterpret_cast<char*>(as + lane);
  for (int p = p_first; p < p_last; ++p) {
    // the record and slot 0, all loads issued before any is used.  An empty
    // row (d = 0) is walked too: its slots are inert and its Slot0 factor
    // is 0, so it adds exact zeros.
    // the 8-node FP64 walk derives the accumulator offsets (SGPR room)
    const ShortRowRegs<T> r = load_short_row<T, !(sizeof(T) == 8 && !KEEP)>(rows, row0, p);
    const Slot0<T>* z = z0 + p;
    const T bm = ldu(&z->bm);
    const T cA = ldu(&z->ca);
    const T cB = ldu(&z->cb);
    const float loB = ldu(&z->lo_b);
    const float hiB = ldu(&z->hi_b);
    const bool mokB = ldu(&z->mok_b) != 0;
    const int d = r.d;
    const int s = (KEEP && p != p_first) ? r.share : 0;
    const int mok = r.mok;
    const auto& xo = r.xo;
    const auto& ao = r.ao;
    const auto& l = r.l;
    const auto& u = r.u;
    const auto& bl = r.bl;
    const auto& cbl = r.cbl;
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = *reinterpret_cast<const float*>(xl + xo[k]);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k == 0 || k > s) {
        bool lower;
        if (NANS) {
          const bool miss = ((mok >> k) & 1) != 0;
          lower = miss ? !(x[k] < l[k]) : (x[k] >= l[k]);
        } else {
          lower = x[k] >= l[k];
        }
        const bool in = lower & !(x[k] >= u[k]);
        // b in a VGPR once: the select's -b and the factor FMAs read it
        // there (a VALU op reads one SGPR, and the select's mask is one)
        const T b = k == 0 ? bm : bl[k];
        const T bv = kScalarT ? to_vgpr(b) : b;
        T c;
        if (k == 0) {
          bool lowerB;
          if (NANS) lowerB = mokB ? !(x[0] < loB) : (x[0] >= loB);
          else lowerB = x[0] >= loB;
          const bool inB = lowerB & !(x[0] >= hiB);
          c = in ? cA : (inB ? cB : -bv);
        } else {
          c = in ? cbl[k] : -bv;
        }
        cf[k] = c;
        if (kScalarT) {
          // t as FP32 literals, or from SGPRs (FP64)
#pragma unroll
          for (int m = 0; m < NH; ++m) G[k][m] = fmaT(node8_t(nc, m), c, bv);
        } else {
#pragma unroll
          for (int m = 0; m < NH; ++m) G[k][m] = fmaT(tv[m], c, b);
        }
        // the prefix through this slot (every later slot is evaluated too)
        if (k >= 1 && k <= 6) {
#pragma unroll
          for (int m = 0; m < NH; ++m) P[k][m] = P[k - 1][m] * G[k][m];
        }
      }
    }
    // slot 0, last in the order: its leave-one-out product is P[6] F_7
    {
      T dot = P[6][0] * G[7][0];
#pragma unroll
      for (int m = 1; m < NH; ++m) dot = fmaT(P[6][m], G[7][m], dot);
      __hip_atomic_fetch_add(reinterpret_cast<double*>(al + ao[0]), (double)(cf[0] * dot),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    // slots 7..1: suffix products, starting from slot 0's factor.  A full
    // row (d = 8, most rows of depth-8 trees) takes a sweep without the
    // per-slot test of j < d.
    T S[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) S[m] = G[0][m];
    auto sweep = [&](auto full) __attribute__((always_inline)) {
#pragma unroll
      for (int q = 6; q >= 0; --q) {
        const int j = q + 1;
        if (decltype(full)::value || j < d) {
          T dot = P[q][0] * S[0];
#pragma unroll
          for (int m = 1; m < NH; ++m) dot = fmaT(P[q][m], S[m], dot);
          const double c = (double)(cf[j] * dot);
          __hip_atomic_fetch_add(reinterpret_cast<double*>(al + ao[j]), c, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (q > 0) {
#pragma unroll
          for (int m = 0; m < NH; ++m) S[m] *= G[j][m];
        }
      }
    };
    if (d == 8) sweep(std::true_type{});
    else sweep(std::false_type{});
  }
}

// First order over rows of more than 8 features, reusing work between
// consecutive rows.  Each wave walks a contiguous run of rows.  The products
// are taken over the slots in the order 1, 2, ..., d - 1, 0: slot 0 (the
// row's own factor, from Slot0) comes last, so the prefix products over slots
// 1..j-1 depend only on those slots.  When slots 1..s equal the previous
// row's (share[p] = s, from the host), the c_j of the batches of 8 slots that
// lie within them are still in registers, and so are the prefix checkpoints
// ck[b] = w prod_{1 <= k < 8b} F_k(m) of the batches b with 8b - 1 <= s (kept
// across rows when all nodes run in one pass).  The backward sweep is that of values_paths with the suffix
// products started from slot 0's factor; slot 0's own leave-one-out product
// is the full prefix over slots 1..d-1 (inert padding slots are factors 1).
template <typename T, int DMAX, int NH, bool STORE_G, bool NANS, int NN>
__device__ __forceinline__ void values_rows_long(
    const PathHdr* __restrict__ hdr, const int32_t* __restrict__ feat,
    const float* __restrict__ lo, const float* __restrict__ hi, const T* __restrict__ bb,
    const T* __restrict__ cbb, const Slot0<T>* __restrict__ z0,
    const int32_t* __restrict__ share, const float* xs, double* as, int pb, int pe, int wave,
    int nw, int lane, const T* tv, const NodeConsts<T>& nc) {
  constexpr int NB = DMAX / 8;
  constexpr bool kKeep = NH == NN;
  const int run = (pe - pb + nw - 1) / nw;
  const int p_first = pb + wave * run;
  const int p_last = min(pe, p_first + run);
  T cf[DMAX];     // c_j of the current row
  T ck[NB][NH];   // prefix checkpoints
  int ckv = 0;    // ck[1 .. ckv - 1] are the previous row's
  for (int p = p_first; p < p_last; ++p) {
    const int d = ldu(&hdr[p].d);
    if (d == 0) {
      ckv = 0;
      continue;
    }
    const int off = ldu(&hdr[p].off);
    const int s = p == p_first ? 0 : ldu(share + p);
    const int nb = (d + 7) >> 3;
    const Slot0<T>* z = z0 + p;
    const T bm = ldu(&z->bm);
    const T cA = ldu(&z->ca);
    const T cB = ldu(&z->cb);
    const float loB = ldu(&z->lo_b);
    const float hiB = ldu(&z->hi_b);
    const bool mokB = ldu(&z->mok_b) != 0;

    // c_j of every batch with a slot past s (a batch's shared slots are
    // evaluated again with it, to the same values: one branch per batch)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b < nb && (b == 0 || 8 * b + 7 > s)) {
        const int jb = 8 * b;
        int fm[8];
        float l[8], u[8], x[8];
        T bl[8], cbl[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          fm[k] = ldu(feat + off + jb + k);
          l[k] = ldu(lo + off + jb + k);
          u[k] = ldu(hi + off + jb + k);
          bl[k] = ldu(bb + off + jb + k);
          cbl[k] = ldu(cbb + off + jb + k);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = xs[(fm[k] & kFeatureMask) * kTileStride + lane];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int j = jb + k;
          bool lower;
          if (NANS) {
            const bool miss = (fm[k] & kMissingOkBit) != 0;
            lower = miss ? !(x[k] < l[k]) : (x[k] >= l[k]);
          } else {
            lower = x[k] >= l[k];
          }
          const bool in = lower & !(x[k] >= u[k]);
          if (j == 0) {
            bool lowerB;
            if (NANS) lowerB = mokB ? !(x[0] < loB) : (x[0] >= loB);
            else lowerB = x[0] >= loB;
            const bool inB = lowerB & !(x[0] >= hiB);
            cf[0] = in ? cA : (inB ? cB : -bm);
          } else {
            cf[j] = in ? cbl[k] : -bl[k];
          }
        }
      }
    }
    const int f0 = ldu(feat + off) & kFeatureMask;

#pragma unroll
    for (int pass = 0; pass < NN / NH; ++pass) {
      const int m0 = pass * NH;
      // checkpoints, recomputed from the first batch whose slots are not all
      // shared with the previous row
#pragma unroll
      for (int m = 0; m < NH; ++m) ck[0][m] = nc.w[m0 + m];
      bool fresh = !kKeep;
#pragma unroll
      for (int b = 1; b < NB; ++b) {
        if (b < nb) {
          fresh = fresh || b >= ckv || 8 * b - 1 > s;
          if (fresh) {
#pragma unroll
            for (int m = 0; m < NH; ++m) ck[b][m] = ck[b - 1][m];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int j = 8 * (b - 1) + k;
              if (j > 0) {
                const T bj = ldu(bb + off + j);
#pragma unroll
                for (int m = 0; m < NH; ++m) ck[b][m] *= fmaT(tv[m0 + m], cf[j], bj);
              }
            }
          }
        }
      }
      // backward sweep, last batch first; S starts from slot 0's factor
      T S[NH];
#pragma unroll
      for (int m = 0; m < NH; ++m) S[m] = fmaT(tv[m0 + m], cf[0], bm);
#pragma unroll
      for (int b = NB - 1; b >= 0; --b) {
        if (b < nb) {
          const int jb = 8 * b;
          T bj[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) bj[k] = jb + k == 0 ? T(1) : ldu(bb + off + jb + k);
          T Pb[8][NH];
          T Gb[STORE_G ? 8 : 1][NH];
          T run[NH];
#pragma unroll
          for (int m = 0; m < NH; ++m) run[m] = ck[b][m];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
#pragma unroll
            for (int m = 0; m < NH; ++m) {
              Pb[k][m] = run[m];
              if (jb + k > 0) {
                const T g = fmaT(tv[m0 + m], cf[jb + k], bj[k]);
                if (STORE_G) Gb[STORE_G ? k : 0][m] = g;
                run[m] *= g;
              }
            }
          }
          if (b == nb - 1) {
            // slot 0: w prod_{k >= 1} F_k(m), the full prefix
            T dot = run[0];
#pragma unroll
            for (int m = 1; m < NH; ++m) dot += run[m];
            __hip_atomic_fetch_add(&as[f0 * kTileStride + lane], (double)(cf[0] * dot),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
#pragma unroll
          for (int k = 7; k >= 0; --k) {
            const int j = jb + k;
            if (j > 0) {
              if (j < d) {
                const int f = ldu(feat + off + j) & kFeatureMask;
                T dot = Pb[k][0] * S[0];
#pragma unroll
                for (int m = 1; m < NH; ++m) dot = fmaT(Pb[k][m], S[m], dot);
                __hip_atomic_fetch_add(&as[f * kTileStride + lane], (double)(cf[j] * dot),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              }
#pragma unroll
              for (int m = 0; m < NH; ++m) {
                const T g = STORE_G ? Gb[STORE_G ? k : 0][m] : fmaT(tv[m0 + m], cf[j], bj[k]);
                S[m] *= g;
              }
            }
          }
        }
      }
    }
    ckv = kKeep ? nb : 0;
  }
}

// The rows and tile features of one work item.  Work item b is (sample block
// b mod nsb, row chunk b div nsb).  Ordinarily a chunk is `chunk` consecutive
// rows of the bucket and the tile holds every feature; with segments (wide
// feature spaces) chunk c is segment c, whose tile holds its own feature
// list, which the rows' elements index (lfeat).
struct ItemRows {
  int p0, p1;            // rows [p0, p1)
  int nf;                // tile features
  const int32_t* fmap;   // tile feature -> global feature (null: identity)
};

__device__ __forceinline__ ItemRows item_rows(const Segment* segs, const int32_t* seg_feat,
                                              int ch, int32_t path_begin, int32_t path_end,
                                              int32_t chunk, int32_t F) {
  ItemRows ir;
  if (segs != nullptr) {
    ir.p0 = ldu(&segs[ch].row_begin);
    ir.p1 = ldu(&segs[ch].row_end);
    ir.nf = ldu(&segs[ch].nfeat);
    ir.fmap = seg_feat + ldu(&segs[ch].feat_begin);
  } else {
    ir.p0 = path_begin + ch * chunk;
    ir.p1 = min(path_end, ir.p0 + chunk);
    ir.nf = F;
    ir.fmap = nullptr;
  }
  return ir;
}

// tile_f: the features the LDS layout is sized for (F, or kSegFeatures with
// segments); F: phi's row length.
template <typename T, int DMAX, int NH, bool STORE_G, int NN>
__global__ void __launch_bounds__(512)
values_kernel(const PathHdr* __restrict__ hdr, const int32_t* __restrict__ feat,
              const float* __restrict__ lo, const float* __restrict__ hi,
              const T* __restrict__ bb, const T* __restrict__ cbb,
              const Slot0<T>* __restrict__ z0, const int32_t* __restrict__ share,
              const float* __restrict__ X, int64_t M, int64_t ldx, int32_t F, int32_t tile_f,
              int32_t path_begin, int32_t path_end, int32_t chunk, int32_t nsb,
              const Segment* __restrict__ segs, const int32_t* __restrict__ seg_feat,
              int32_t ng, int32_t grp, double* __restrict__ acc, void* __restrict__ direct,
              int32_t direct_fp64, int32_t plain_add, const ShortRow<T>* __restrict__ srows,
              NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* xs = reinterpret_cast<float*>(smem);
  size_t xs_bytes = ((size_t)tile_f * kTileStride * sizeof(float) + 15) & ~(size_t)15;
  double* as = reinterpret_cast<double*>(smem + xs_bytes);

  // The dispatcher deals workgroups to the 8 XCDs in turn: XCD x gets the
  // workgroups b = x mod 8.  They take the x-th eighth of the work items in
  // order, so each XCD's L2 holds the rows of its own chunks only.
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const int sb = item % nsb;
  const int ch = item / nsb;
  const int64_t s0 = (int64_t)sb * kSamplesPerBlock;
  const ItemRows ir = item_rows(segs, seg_feat, ch, path_begin, path_end, chunk, F);
  const int nf = ir.nf;

  // stage the sample tile transposed; zero the accumulator; note any NaN.
  // With segments (wide feature spaces) X is feature-major [F][ldx] and acc
  // [ng][F][M], so consecutive threads take consecutive samples of a feature.
  const bool fmajor = segs != nullptr;
  const int tile = kSamplesPerBlock * nf;
  int nan_seen = 0;
  if (fmajor) {
    for (int i = threadIdx.x; i < tile; i += blockDim.x) {
      const int k = i >> 6, r = i & 63;
      const int64_t s = s0 + r;
      const float v = (s < M) ? X[(int64_t)ir.fmap[k] * ldx + s] : 0.0f;
      nan_seen |= (v != v);
      xs[k * kTileStride + r] = v;
      as[k * kTileStride + r] = 0.0;
    }
  } else {
    for (int i = threadIdx.x; i < tile; i += blockDim.x) {
      const int r = i / nf;
      const int k = i - r * nf;
      const int64_t s = s0 + r;
      const float v = (s < M) ? X[s * ldx + k] : 0.0f;
      nan_seen |= (v != v);
      xs[k * kTileStride + r] = v;
      as[k * kTileStride + r] = 0.0;
    }
  }
  const bool any_nan = __syncthreads_or(nan_seen) != 0;

  const int lane = threadIdx.x & 63;
  // wave-uniform loop bounds (kept in SGPRs so the path loads are scalar)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
  const int pb = __builtin_amdgcn_readfirstlane(ir.p0);
  const int pe = __builtin_amdgcn_readfirstlane(ir.p1);

  // nodes pinned in VGPRs: a VALU op may read only one SGPR on gfx9-class
  // hardware, and b_j arrives in an SGPR
  T tv[NN];
#pragma unroll
  for (int m = 0; m < NN; ++m) tv[m] = to_vgpr(nc.t[m]);

  // the shared-prefix walk keeps c_j and F_j(m) of all eight slots live
  // across rows: FP32 within 128 VGPRs (four waves per SIMD); FP64 only with
  // the 4-node rule (the 8-node FP64 instance has no registers to spare)
  constexpr bool kShared = DMAX == 8 && NH == NN && (STORE_G || NN == 4);
  // the 8-node FP64 instance walks the same records without keeping a row's
  // factors or prefix products for the next (no registers for them)
  constexpr bool kShortPlain = DMAX == 8 && NH == NN && !kShared;
  if (DMAX > 8 && any_nan)
    values_rows_long<T, DMAX, NH, STORE_G, true, NN>(hdr, feat, lo, hi, bb, cbb, z0, share, xs,
                                                     as, pb, pe, wave, nw, lane, tv, nc);
  else if (DMAX > 8)
    values_rows_long<T, DMAX, NH, STORE_G, false, NN>(hdr, feat, lo, hi, bb, cbb, z0, share, xs,
                                                      as, pb, pe, wave, nw, lane, tv, nc);
  else if (kShared && any_nan)
    values_rows_shared<T, NH, true>(srows, path_begin, z0, xs, as, pb, pe, wave, nw, lane, tv,
                                    nc);
  else if (kShared)
    values_rows_shared<T, NH, false>(srows, path_begin, z0, xs, as, pb, pe, wave, nw, lane, tv,
                                     nc);
  else if (kShortPlain && any_nan)
    values_rows_shared<T, NH, true, false>(srows, path_begin, z0, xs, as, pb, pe, wave, nw, lane,
                                           tv, nc);
  else if (kShortPlain)
    values_rows_shared<T, NH, false, false>(srows, path_begin, z0, xs, as, pb, pe, wave, nw,
                                            lane, tv, nc);
  else if (any_nan)
    values_paths<T, DMAX, NH, STORE_G, true, false, NN>(hdr, feat, lo, hi, bb, cbb, nullptr,
                                                        z0, xs, as, nullptr, nullptr, pb,
                                                        pe, wave, nw, lane, tv, nc);
  else
    values_paths<T, DMAX, NH, STORE_G, false, false, NN>(hdr, feat, lo, hi, bb, cbb, nullptr,
                                                         z0, xs, as, nullptr, nullptr, pb,
                                                         pe, wave, nw, lane, tv, nc);
  __syncthreads();

  // flush: consecutive threads take consecutive features of one sample.
  // direct: this workgroup is the only one of its sample block (one bucket,
  // one chunk), so it writes phi rows outright, in the output precision.
  if (fmajor) {
    // acc[grp, f, s] (segments never write phi directly)
    for (int i = threadIdx.x; i < tile; i += blockDim.x) {
      const int k = i >> 6, r = i & 63;
      const int64_t s = s0 + r;
      if (s < M) {
        const double v = as[k * kTileStride + r];
        const int64_t o = ((int64_t)grp * F + ir.fmap[k]) * M + s;
        if (v != 0.0) {
          if (plain_add) acc[o] += v;
          else unsafeAtomicAdd(&acc[o], v);
        }
      }
    }
    return;
  }
  for (int i = threadIdx.x; i < tile; i += blockDim.x) {
    const int r = i / nf;
    const int k = i - r * nf;
    const int64_t s = s0 + r;
    if (s < M) {
      const double v = as[k * kTileStride + r];
      const int64_t o = (s * ng + grp) * F + k;  // phi[s, grp, f]
      if (direct != nullptr) {
        if (direct_fp64) static_cast<double*>(direct)[o] = v;
        else static_cast<float*>(direct)[o] = (float)v;
      } else if (v != 0.0) {
        // plain_add: the only workgroup of this launch that holds (s, f)
        if (plain_add) acc[o] += v;
        else unsafeAtomicAdd(&acc[o], v);
      }
    }
  }
}


// Adjoint over rows of at most 8 features with all NH nodes in one pass,
// with the reuse of values_rows_shared (contiguous runs, slots 1..s of the
// previous row kept in registers: c_j, F_j(m) and g_j c_j).  Slot 0 (a merged
// pair's split feature, or any one feature of a single path) stays out of the
// products; with Q_j(m) = prod_{k >= 1, k != j} F_k(m), Q_0 = prod_{k >= 1} F_k,
//   R(m) = sum_{j >= 1} g_j c_j w_m Q_j(m),
//   d phi . g / d v_A = sum_m F_A(m) R(m) + g_0 c_A sum_m w_m Q_0(m),
// where F_A = b_A + t c_A is slot 0's factor of leaf A (a single path: its
// own), and likewise for leaf B of a merged pair.  The sum over m of
// F_A(m) R(m) is b_A sum_m R(m) + c_A sum_m t_m R(m).
template <typename T, int NH, bool NANS>
__device__ __forceinline__ void adjoint_rows_shared(
    const ShortRow<T>* __restrict__ rows, int row0, const PathHdr* __restrict__ hdr,
    const SidePath* __restrict__ side, const float* xs, const T* gs,
    double* __restrict__ grad_leaf, int pb, int pe, int wave, int nw, int lane, const T* tv,
    const NodeConsts<T>& nc, bool det) {
  constexpr bool kScalarT = NH == 8;
  const int run = (pe - pb + nw - 1) / nw;
  const int p_first = pb + wave * run;
  const int p_last = min(pe, p_first + run);
  T cf[8], gc[8];  // slots 1..7: c_j and g_j c_j of the current row
  T G[8][NH];      // slots 1..7: F_j(m)
  // prefix products over slots 1..q (P[q], q = 0..6; w folded in); P[1..s]
  // depend only on shared slots and are kept from the previous row
  T P[7][NH];
#pragma unroll
  for (int m = 0; m < NH; ++m) P[0][m] = kScalarT ? node8_w(nc, m) : nc.w[m];
  const char* xl = reinterpret_cast<const char*>(xs + lane);
  const char* gl = reinterpret_cast<const char*>(gs + lane);
  for (int p = p_first; p < p_last; ++p) {
    // the record and the row's leaf and side record, all loads issued
    // before any is used.  An empty row (d = 0) is walked too: its slots are
    // inert, so its leaf's gradient comes out exactly 0.
    const ShortRowRegs<T> r = load_short_row(rows, row0, p);
    const int leaf = ldu(&hdr[p].leaf);
    const int sidx = side == nullptr ? -1 : ldu(&hdr[p].tree);
    const bool merged = sidx >= 0;
    const int d = r.d;
    const int s = p == p_first ? 0 : r.share;
    // the tile row of slot k's feature: the sample tile is FP32 and the
    // gradient tile T
    const auto& xo = r.xo;
    const auto& go = sizeof(T) == 4 ? r.xo : r.ao;
    const auto& l = r.l;
    const auto& u = r.u;
    const auto& bl = r.bl;
    const auto& cbl = r.cbl;
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = *reinterpret_cast<const float*>(xl + xo[k]);
    auto follows = [&](float xv, float lv, float uv, bool miss) -> bool {
      bool lower;
      if (NANS) lower = miss ? !(xv < lv) : (xv >= lv);
      else lower = xv >= lv;
      return lower & !(xv >= uv);
    };
    // slot 0: leaf A's factor (and B's for a merged pair)
    T bA = bl[0], cbA = cbl[0], bB = T(0), cbB = T(0);
    float loB = 0.f, hiB = 0.f;
    bool mokB = false;
    int leafB = 0;
    if (merged) {
      const SidePath* sp = side + sidx;
      leafB = ldu(&sp->leaf_b);
      loB = ldu(&sp->lo_b);
      hiB = ldu(&sp->hi_b);
      mokB = ldu(&sp->mok_b) != 0;
      bA = (T)ldu(&sp->b_a);
      cbA = (T)ldu(&sp->cb_a);
      bB = (T)ldu(&sp->b_b);
      cbB = (T)ldu(&sp->cb_b);
    }
    const T cA = follows(x[0], l[0], u[0], (r.mok & 1) != 0) ? cbA : -bA;
    const T cB = follows(x[0], loB, hiB, mokB) ? cbB : -bB;
    const T g0 = *reinterpret_cast<const T*>(gl + go[0]);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      if (k > s) {
        // b in a VGPR once, for the select's -b and the factor FMAs
        const T bv = kScalarT ? to_vgpr(bl[k]) : bl[k];
        const T c = follows(x[k], l[k], u[k], ((r.mok >> k) & 1) != 0) ? cbl[k] : -bv;
        cf[k] = c;
        gc[k] = *reinterpret_cast<const T*>(gl + go[k]) * c;
        if (kScalarT) {
#pragma unroll
          for (int m = 0; m < NH; ++m) G[k][m] = fmaT(node8_t(nc, m), c, bv);
        } else {
#pragma unroll
          for (int m = 0; m < NH; ++m) G[k][m] = fmaT(tv[m], c, bl[k]);
        }
        // the prefix through this slot (every later slot is evaluated too)
        if (k <= 6) {
#pragma unroll
          for (int m = 0; m < NH; ++m) P[k][m] = P[k - 1][m] * G[k][m];
        }
      }
    }
    // sum_m w_m Q_0(m)
    T q0 = P[6][0] * G[7][0];
#pragma unroll
    for (int m = 1; m < NH; ++m) q0 = fmaT(P[6][m], G[7][m], q0);
    // R(m), slots 7..1
    T S[NH], R[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) {
      S[m] = T(1);
      R[m] = T(0);
    }
#pragma unroll
    for (int q = 6; q >= 0; --q) {
      const int j = q + 1;
      if (j < d) {
#pragma unroll
        for (int m = 0; m < NH; ++m) R[m] = fmaT(gc[j], P[q][m] * S[m], R[m]);
      }
      if (q > 0) {
#pragma unroll
        for (int m = 0; m < NH; ++m) S[m] *= G[j][m];
      }
    }
    T sR = R[0], stR = (kScalarT ? node8_t(nc, 0) : tv[0]) * R[0];
#pragma unroll
    for (int m = 1; m < NH; ++m) {
      sR += R[m];
      stR = fmaT(kScalarT ? node8_t(nc, m) : tv[m], R[m], stR);
    }
    const T gq = g0 * q0;
    double gA = (double)fmaT(bA, sR, cA * (stR + gq));
    gA = wave_sum_last(gA);
    if (lane == 63) leaf_add(grad_leaf, leaf, gA, det);
    if (merged) {
      double gB = (double)fmaT(bB, sR, cB * (stR + gq));
      gB = wave_sum_last(gB);
      if (lane == 63) leaf_add(grad_leaf, leafB, gB, det);
    }
  }
}

// Adjoint to the leaf values (same tiling as values_kernel): the tile holds
// the samples' rows and their upstream gradient rows g[s, :].
template <typename T, int DMAX, int NH, bool STORE_G, int NN>
__global__ void __launch_bounds__(512)
adjoint_kernel(const PathHdr* __restrict__ hdr, const int32_t* __restrict__ feat,
               const float* __restrict__ lo, const float* __restrict__ hi,
               const T* __restrict__ bb, const T* __restrict__ cbb,
               const SidePath* __restrict__ side, const int32_t* __restrict__ share,
               const float* __restrict__ X, const T* __restrict__ G, int64_t M, int64_t ldx,
               int32_t F, int32_t tile_f, int32_t path_begin, int32_t path_end, int32_t chunk,
               int32_t nsb, const Segment* __restrict__ segs,
               const int32_t* __restrict__ seg_feat, int32_t ng, int32_t grp,
               double* __restrict__ grad_leaf, int64_t part_stride,
               const ShortRow<T>* __restrict__ srows, NodeConsts<T> nc) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* xs = reinterpret_cast<float*>(smem);
  size_t xs_bytes = ((size_t)tile_f * kTileStride * sizeof(float) + 15) & ~(size_t)15;
  T* gs = reinterpret_cast<T*>(smem + xs_bytes);

  // work items dealt to the XCDs in contiguous eighths (xcd_item)
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const int sb = item % nsb;
  const int ch = item / nsb;
  const int64_t s0 = (int64_t)sb * kSamplesPerBlock;
  const ItemRows ir = item_rows(segs, seg_feat, ch, path_begin, path_end, chunk, F);
  const int nf = ir.nf;

  // stage the sample rows and gradient rows transposed (padding rows get a
  // zero gradient, so they add nothing); note any NaN.  With segments (wide
  // feature spaces) X is feature-major [F][ldx] and G [ng][F][M].
  const bool fmajor = segs != nullptr;
  const int tile = kSamplesPerBlock * nf;
  int nan_seen = 0;
  if (fmajor) {
    for (int i = threadIdx.x; i < tile; i += blockDim.x) {
      const int k = i >> 6, r = i & 63;
      const int f = ir.fmap[k];
      const int64_t s = s0 + r;
      const float v = (s < M) ? X[(int64_t)f * ldx + s] : 0.0f;
      nan_seen |= (v != v);
      xs[k * kTileStride + r] = v;
      gs[k * kTileStride + r] = (s < M) ? G[((int64_t)grp * F + f) * M + s] : T(0);  // G[grp, f, s]
    }
  } else {
    for (int i = threadIdx.x; i < tile; i += blockDim.x) {
      const int r = i / nf;
      const int k = i - r * nf;
      const int64_t s = s0 + r;
      const float v = (s < M) ? X[s * ldx + k] : 0.0f;
      nan_seen |= (v != v);
      xs[k * kTileStride + r] = v;
      gs[k * kTileStride + r] = (s < M) ? G[(s * ng + grp) * F + k] : T(0);  // G[s, grp, f]
    }
  }
  const bool any_nan = __syncthreads_or(nan_seen) != 0;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
  const int pb = __builtin_amdgcn_readfirstlane(ir.p0);
  const int pe = __builtin_amdgcn_readfirstlane(ir.p1);
  T tv[NN];
#pragma unroll
  for (int m = 0; m < NN; ++m) tv[m] = to_vgpr(nc.t[m]);
  // deterministic: this sample block's own row of partial sums
  const bool det = part_stride > 0;
  double* gl = det ? grad_leaf + (int64_t)sb * part_stride : grad_leaf;
  constexpr bool kShared = DMAX == 8 && NH == NN && (STORE_G || NN == 4);
  if (kShared && any_nan)
    adjoint_rows_shared<T, NH, true>(srows, path_begin, hdr, side, xs, gs, gl, pb, pe, wave, nw,
                                     lane, tv, nc, det);
  else if (kShared)
    adjoint_rows_shared<T, NH, false>(srows, path_begin, hdr, side, xs, gs, gl, pb, pe, wave, nw,
                                      lane, tv, nc, det);
  else if (any_nan)
    values_paths<T, DMAX, NH, STORE_G, true, true, NN>(hdr, feat, lo, hi, bb, cbb, side, nullptr,
                                                       xs, nullptr, gs, gl, pb, pe, wave, nw,
                                                       lane, tv, nc, det);
  else
    values_paths<T, DMAX, NH, STORE_G, false, true, NN>(hdr, feat, lo, hi, bb, cbb, side, nullptr,
                                                        xs, nullptr, gs, gl, pb, pe, wave, nw,
                                                        lane, tv, nc, det);
}

namespace {

// Paths per work item: about 32 rounds of the ~512 resident workgroups
// (small tail), chunks of at least 256 paths so the per-item tile load and
// flush stay small next to the path work.
int values_chunk(int n_paths, int nsb, int items) {
  const int64_t want_items = items > 0 ? items : 16384;
  int64_t n_chunks = (want_items + nsb - 1) / nsb;
  n_chunks = std::max<int64_t>(1, std::min<int64_t>(n_chunks, (n_paths + 255) / 256));
  return (int)((n_paths + n_chunks - 1) / n_chunks);
}

}  // namespace

bool values_direct(const std::vector<Bucket>& bks, int64_t M, const ValuesShape& shape) {
  if (bks.size() != 1 || M <= 0) return false;
  const int nsb = (int)((M + kSamplesPerBlock - 1) / kSamplesPerBlock);
  const int n_paths = bks[0].path_end - bks[0].path_begin;
  return values_chunk(n_paths, nsb, shape.items) >= n_paths;
}

namespace {


// The short-row records of a capacity-8 bucket from its first row (null for
// other buckets).
template <typename T>
const ShortRow<T>* short_rows_of(const PathArrays& a, const Bucket& bk) {
  if (bk.dmax != 8 || bk.srow_begin < 0) return nullptr;
  const ShortRow<T>* r;
  if constexpr (std::is_same<T, float>::value) r = a.srow32;
  else r = a.srow64;
  if (r == nullptr) fail(QTS_E_INVALID_ARG, "internal: no short-row records");
  return r + bk.srow_begin;
}

// How one launch over a bucket splits its rows: chunks of `chunk` rows with
// the full feature tile, or (wide feature spaces) the bucket's segments with
// their own tiles, the rows' elements read through lfeat.
struct RowSplit {
  const int32_t* feat;   // element features as the kernel indexes its tile
  const Segment* segs;   // null: plain chunks
  int chunk;
  int n_chunks;
  int tile_f;            // features the LDS tile is laid out for
};

RowSplit row_split(const HostTable& h, const PathArrays& a, const Bucket& bk, int nsb,
                   const ValuesShape& shape) {
  RowSplit r{a.feat, nullptr, 0, 0, h.F};
  if (a.compact == nullptr) {
    const int n_paths = bk.path_end - bk.path_begin;
    r.chunk = values_chunk(n_paths, nsb, shape.items);
    r.n_chunks = (n_paths + r.chunk - 1) / r.chunk;
    return r;
  }
  const CompactTable& c = *a.compact;
  for (size_t i = 0; i + 1 < c.bucket_seg.size(); ++i) {
    const int s0 = c.bucket_seg[i], s1 = c.bucket_seg[i + 1];
    if (s1 > s0 && c.segs[(size_t)s0].row_begin == bk.path_begin) {
      r.feat = a.lfeat;
      r.segs = a.segs + s0;
      r.n_chunks = s1 - s0;
      r.tile_f = kSegFeatures;
      return r;
    }
  }
  fail(QTS_E_INVALID_ARG, "internal: bucket without segments");
}

template <typename T, int DMAX, int NH, bool STORE_G, int NN>
void launch_one(const HostTable& h, const DeviceTable& d, const PathArrays& a, const Bucket& bk,
                const float* X, int64_t M, int64_t ldx, const void* slot0, double* acc,
                void* direct, const ValuesShape& shape, hipStream_t s, bool det) {
  const int F = h.F;
  const int nsb = (int)((M + kSamplesPerBlock - 1) / kSamplesPerBlock);
  const RowSplit rs = row_split(h, a, bk, nsb, shape);
  const int64_t grid = (int64_t)nsb * rs.n_chunks;
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "grid too large");
  const size_t lds = values_lds_bytes(rs.tile_f);
  // deterministic: one wave per workgroup (no LDS atomics between waves), and
  // one launch per chunk, so each launch has one workgroup per (sample, feature)
  const int threads = det ? 64 : 64 * shape.waves_per_block;
  const T* b = std::is_same<T, float>::value ? (const T*)a.b32 : (const T*)a.b64;
  const T* cb = std::is_same<T, float>::value ? (const T*)a.cb32 : (const T*)a.cb64;
  NodeConsts<T> nc;
  if constexpr (std::is_same<T, float>::value) nc = NN == 8 ? d.n32 : d.n32_4;
  else nc = NN == 8 ? d.n64 : d.n64_4;
  if (lds > raise_lds_limit((const void*)values_kernel<T, DMAX, NH, STORE_G, NN>))
    fail(QTS_E_UNSUPPORTED, "internal: the sample tile does not fit in LDS");
  const ShortRow<T>* srows = short_rows_of<T>(a, bk);
  if (!det) {
    hipLaunchKernelGGL((values_kernel<T, DMAX, NH, STORE_G, NN>), dim3((unsigned)grid),
                       dim3(threads), lds, s, a.hdr, rs.feat, a.lo, a.hi, b, cb,
                       (const Slot0<T>*)slot0, a.share, X, M, ldx, F, rs.tile_f, bk.path_begin,
                       bk.path_end, rs.chunk, nsb, rs.segs, a.seg_feat, h.n_groups, bk.group,
                       acc, rs.segs ? nullptr : direct,
                       (int32_t)(std::is_same<T, double>::value ? 1 : 0), 0, srows, nc);
    check_hip(hipGetLastError(), "values_kernel launch");
    return;
  }
  for (int c = 0; c < rs.n_chunks; ++c) {
    const int p0 = rs.segs ? bk.path_begin : bk.path_begin + c * rs.chunk;
    const int p1 = rs.segs ? bk.path_end : std::min(bk.path_end, p0 + rs.chunk);
    hipLaunchKernelGGL((values_kernel<T, DMAX, NH, STORE_G, NN>), dim3((unsigned)nsb),
                       dim3(threads), lds, s, a.hdr, rs.feat, a.lo, a.hi, b, cb,
                       (const Slot0<T>*)slot0, a.share, X, M, ldx, F, rs.tile_f, p0, p1,
                       rs.chunk, nsb, rs.segs ? rs.segs + c : nullptr, a.seg_feat, h.n_groups,
                       bk.group, acc, nullptr, (int32_t)(std::is_same<T, double>::value ? 1 : 0),
                       1, srows ? srows + (p0 - bk.path_begin) : nullptr, nc);
    check_hip(hipGetLastError(), "values_kernel launch");
  }
}

template <typename T, int DMAX, int NH, bool STORE_G, int NN>
void launch_adj_one(const HostTable& h, const DeviceTable& d, const PathArrays& a,
                    const Bucket& bk, const float* X, const void* G, int64_t M, int64_t ldx,
                    double* grad_leaf, const ValuesShape& shape, hipStream_t s,
                    int64_t part_stride) {
  const int F = h.F;
  const int nsb = (int)((M + kSamplesPerBlock - 1) / kSamplesPerBlock);
  const RowSplit rs = row_split(h, a, bk, nsb, shape);
  const int64_t grid = (int64_t)nsb * rs.n_chunks;
  if (grid > 0x7fffffff) fail(QTS_E_UNSUPPORTED, "grid too large");
  size_t xs = ((size_t)rs.tile_f * kTileStride * sizeof(float) + 15) & ~(size_t)15;
  const size_t lds = xs + (size_t)rs.tile_f * kTileStride * sizeof(T);
  const int threads = 64 * shape.waves_per_block;
  const T* b = std::is_same<T, float>::value ? (const T*)a.b32 : (const T*)a.b64;
  const T* cb = std::is_same<T, float>::value ? (const T*)a.cb32 : (const T*)a.cb64;
  NodeConsts<T> nc;
  if constexpr (std::is_same<T, float>::value) nc = NN == 8 ? d.n32 : d.n32_4;
  else nc = NN == 8 ? d.n64 : d.n64_4;
  if (lds > raise_lds_limit((const void*)adjoint_kernel<T, DMAX, NH, STORE_G, NN>))
    fail(QTS_E_UNSUPPORTED, "internal: the sample tile does not fit in LDS");
  hipLaunchKernelGGL((adjoint_kernel<T, DMAX, NH, STORE_G, NN>), dim3((unsigned)grid),
                     dim3(threads), lds, s, a.hdr, rs.feat, a.lo, a.hi, b, cb, a.side, a.share,
                     X, (const T*)G, M, ldx, F, rs.tile_f, bk.path_begin, bk.path_end, rs.chunk,
                     nsb, rs.segs, a.seg_feat, h.n_groups, bk.group, grad_leaf, part_stride,
                     short_rows_of<T>(a, bk), nc);
  check_hip(hipGetLastError(), "adjoint_kernel launch");
}

}  // namespace

void launch_adjoint(const HostTable& h, const DeviceTable& d, const PathArrays& a,
                    const Bucket& bk, bool fp64, const float* X, const void* G, int64_t M,
                    int64_t ldx, double* grad_leaf, const ValuesShape& shape, int nodes,
                    hipStream_t s, int64_t part_stride) {
  if (nodes == 4 && bk.dmax == 8) {
    if (!fp64) launch_adj_one<float, 8, 4, true, 4>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride);
    else launch_adj_one<double, 8, 4, false, 4>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride);
    return;
  }
  if (!fp64) {
    switch (bk.dmax) {
      case 8: launch_adj_one<float, 8, 8, true, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
      case 16: launch_adj_one<float, 16, 8, true, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
      case 32: launch_adj_one<float, 32, 8, false, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
      default: launch_adj_one<float, 64, 4, false, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
    }
  } else {
    switch (bk.dmax) {
      case 8: launch_adj_one<double, 8, 4, false, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
      case 16: launch_adj_one<double, 16, 4, false, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
      case 32: launch_adj_one<double, 32, 4, false, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
      default: launch_adj_one<double, 64, 1, false, 8>(h, d, a, bk, X, G, M, ldx, grad_leaf, shape, s, part_stride); break;
    }
  }
}

// Slot 0 of every first-order row with the current leaf values folded in.
template <typename T>
__global__ void __launch_bounds__(256)
slot0_kernel(const PathHdr* __restrict__ hdr, const int32_t* __restrict__ feat,
             const float* __restrict__ lo, const float* __restrict__ hi,
             const double* __restrict__ b64, const double* __restrict__ cb64,
             const SidePath* __restrict__ side, const double* __restrict__ leaf_val, int32_t n,
             Slot0<T>* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const PathHdr h = hdr[r];
  Slot0<T> z{T(0), T(0), T(0), 0.f, 0.f, 0};
  const int sidx = side == nullptr ? -1 : h.tree;
  if (h.d > 0 && sidx >= 0) {
    const SidePath sp = side[sidx];
    const double va = leaf_val[h.leaf];
    const double vb = leaf_val[sp.leaf_b];
    z.bm = (T)(va * sp.b_a + vb * sp.b_b);
    z.ca = (T)(va * sp.cb_a - vb * sp.b_b);
    z.cb = (T)(vb * sp.cb_b - va * sp.b_a);
    z.lo_b = sp.lo_b;
    z.hi_b = sp.hi_b;
    z.mok_b = sp.mok_b;
  } else if (h.d > 0) {
    const double v = leaf_val[h.leaf];
    const double bm = v * b64[h.off];
    z.bm = (T)bm;
    z.ca = (T)(v * cb64[h.off]);
    z.cb = (T)(-bm);
    z.lo_b = lo[h.off];
    z.hi_b = hi[h.off];
    z.mok_b = (feat[h.off] & kMissingOkBit) != 0 ? 1 : 0;
  }
  out[r] = z;
}

size_t slot0_bytes(int32_t n_rows, bool fp64) {
  return (size_t)n_rows * (fp64 ? sizeof(Slot0<double>) : sizeof(Slot0<float>));
}

void launch_slot0(const PathArrays& a, int32_t n_rows, const double* leaf_val, bool fp64,
                  void* out, hipStream_t s) {
  if (n_rows <= 0) return;
  const unsigned grid = (unsigned)((n_rows + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(slot0_kernel<double>, dim3(grid), dim3(256), 0, s, a.hdr, a.feat, a.lo,
                       a.hi, a.b64, a.cb64, a.side, leaf_val, n_rows, (Slot0<double>*)out);
  else
    hipLaunchKernelGGL(slot0_kernel<float>, dim3(grid), dim3(256), 0, s, a.hdr, a.feat, a.lo,
                       a.hi, a.b64, a.cb64, a.side, leaf_val, n_rows, (Slot0<float>*)out);
  check_hip(hipGetLastError(), "slot0_kernel launch");
}

void launch_values(const HostTable& h, const DeviceTable& d, const PathArrays& a,
                   const Bucket& bk, bool fp64, const float* X, int64_t M, int64_t ldx,
                   const void* slot0, double* acc, void* direct, const ValuesShape& shape,
                   int nodes, hipStream_t s, bool deterministic) {
  if (nodes == 4 && bk.dmax == 8) {
    if (!fp64) launch_one<float, 8, 4, true, 4>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic);
    else launch_one<double, 8, 4, false, 4>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic);
    return;
  }
  if (!fp64) {
    switch (bk.dmax) {
      case 8: launch_one<float, 8, 8, true, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
      case 16: launch_one<float, 16, 8, true, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
      case 32: launch_one<float, 32, 8, false, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
      default: launch_one<float, 64, 4, false, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
    }
  } else {
    switch (bk.dmax) {
      case 8: launch_one<double, 8, 8, false, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
      case 16: launch_one<double, 16, 4, false, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
      case 32: launch_one<double, 32, 4, false, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
      default: launch_one<double, 64, 2, false, 8>(h, d, a, bk, X, M, ldx, slot0, acc, direct, shape, s, deterministic); break;
    }
  }
}

}  // namespace qts
