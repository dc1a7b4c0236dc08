// Device-side tables and kernel launchers (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "qts_internal.h"

namespace qts {

// The 8-node rule on [0,1] in the two precisions used by the kernels.
template <typename T>
struct NodeConsts {
  T t[kNodes];
  T w[kNodes];
};

constexpr int kTileStride = kSamplesPerBlock + 1;  // padded LDS row (bank spread)

// The 8-node rule on [0,1] rounded to FP32, as constants: the FP32 walks that
// hold all 8 nodes in one pass take its nodes and weights as instruction
// literals (an FP32 FMA or multiply with a literal operand issues at about
// twice the rate of one reading a scalar register).  build_nodes checks that
// they equal the FP32 rounding of the rule it computes (Eq. 10).
__host__ __device__ constexpr float rule8_t32(int m) {
  constexpr float t[kNodes] = {0x1.454e34p-6f, 0x1.a06d54p-4f, 0x1.e5dad4p-3f, 0x1.a214dap-2f,
                               0x1.2ef592p-1f, 0x1.86894ap-1f, 0x1.cbf256p-1f, 0x1.f5d58ep-1f};
  return t[m];
}
__host__ __device__ constexpr float rule8_w32(int m) {
  constexpr float w[kNodes] = {0x1.9ea1dp-5f, 0x1.c76fb6p-4f, 0x1.413c5p-3f, 0x1.73636p-3f,
                               0x1.73636p-3f, 0x1.413c5p-3f, 0x1.c76fb6p-4f, 0x1.9ea1dp-5f};
  return w[m];
}

// A first-order row of a capacity-8 bucket as the walk over short rows reads
// it: every field of the row in one record, so a wave fetches the row with a
// few wide scalar loads from one address, and the LDS byte offsets of the
// slots' features precomputed (xoff into the FP32 sample tile, aoff into the
// FP64 accumulator tile; both tiles are [feature][kTileStride]).  Slots past
// d are inert (offset 0, lo = -inf, hi = NaN, missing_ok, b = 1, 1 - b = 0).
// Slot 0's factor comes from Slot0 (built per call); its lo/hi here are A's.
template <typename T>
struct alignas(16) ShortRow {
  int32_t d;        // features of the row (0: an empty path)
  int32_t share;    // slots 1..share equal to the previous row's
  int32_t mok;      // bit k: a missing value follows slot k's splits
  int32_t pad;
  int32_t xoff[8];  // feature * kTileStride * 4
  int32_t aoff[8];  // feature * kTileStride * 8
  float lo[8], hi[8];
  T b[8], cb[8];    // b_j and 1 - b_j (FP64-derived), rounded to T
};

// Device copy of the path table.  Element arrays are shared by all buckets.
struct DeviceTable {
  int device = -1;
  PathHdr* hdr = nullptr;
  int32_t* feat = nullptr;
  float* lo = nullptr;
  float* hi = nullptr;
  float* b32 = nullptr;
  float* cb32 = nullptr;
  double* b64 = nullptr;
  double* cb64 = nullptr;
  double* leaf_val = nullptr;  // the model's own leaf values
  int32_t* share = nullptr;    // HostTable::share
  // slot-major pair table (interactions)
  int32_t* pr_d = nullptr;
  int32_t* pr_leaf = nullptr;
  SidePath* pr_side = nullptr;  // per row; leaf_b = -1 for a single path
  int32_t* pr_feat = nullptr;
  float* pr_lo = nullptr;
  float* pr_hi = nullptr;
  float* pr_b32 = nullptr;
  float* pr_cb32 = nullptr;
  double* pr_b64 = nullptr;
  double* pr_cb64 = nullptr;
  // first-order table with sibling leaves merged (same element layout)
  PathHdr* mhdr = nullptr;
  int32_t* mfeat = nullptr;
  float* mlo = nullptr;
  float* mhi = nullptr;
  float* mb32 = nullptr;
  float* mcb32 = nullptr;
  double* mb64 = nullptr;
  double* mcb64 = nullptr;
  SidePath* side = nullptr;
  int32_t* mshare = nullptr;
  // short-row records of the capacity-8 buckets (Bucket::srow_begin), plain
  // and merged tables
  ShortRow<float>* srow32 = nullptr;
  ShortRow<double>* srow64 = nullptr;
  ShortRow<float>* msrow32 = nullptr;
  ShortRow<double>* msrow64 = nullptr;
  // feature-compacted segments (wide_features only), plain and merged tables
  int32_t* lfeat = nullptr;
  Segment* segs = nullptr;
  int32_t* seg_feat = nullptr;
  int32_t* mlfeat = nullptr;
  Segment* msegs = nullptr;
  int32_t* mseg_feat = nullptr;
  NodeConsts<float> n32;     // the 8-node rule
  NodeConsts<double> n64;
  NodeConsts<float> n32_4;   // the 4-node rule (first 4 entries)
  NodeConsts<double> n64_4;
  NodeConsts<float> n32_2, n32_6;   // the 2- and 6-node rules (interactions)
  NodeConsts<double> n64_2, n64_6;
};

// Device copy of the depth-first tables (DfsTable).
struct DeviceDfs {
  bool built = false;
  DfsNode* nodes = nullptr;
  float* coef32 = nullptr;
  double* coef64 = nullptr;
  int32_t* events = nullptr;       // DfsTable::events
  int32_t* tree_first = nullptr;
  int32_t* tree_nodes = nullptr;
  int32_t n_trees = 0;
  int32_t max_level = 0;
  int32_t n_rows = 0;
  int32_t* row_f = nullptr;
  int32_t* row_d = nullptr;
  int32_t* tile_base = nullptr;
  int32_t* tile_d = nullptr;
  int32_t* feat = nullptr;
  float* lo = nullptr;
  float* hi = nullptr;
  float* b32 = nullptr;
  float* cb32 = nullptr;
  double* b64 = nullptr;
  double* cb64 = nullptr;
  std::vector<int32_t> group_tile;  // host copy: tiles of each output group
  int64_t n_updates = 0;            // pair updates per sample
  int64_t n_updates3 = 0;           // third-order updates per sample
  int32_t max_row_d = 0;            // most features split above one node (other than its own)
  int64_t n_nodes = 0;              // internal nodes
};
// The depth-first third-order pass keeps a row's ratios in registers: rows of
// at most this many features.
constexpr int32_t kDfsTriplesMaxRow = 32;

// The arrays one first-order (or adjoint) launch walks.
struct PathArrays {
  const PathHdr* hdr;
  const int32_t* feat;
  const float* lo;
  const float* hi;
  const float* b32;
  const float* cb32;
  const double* b64;
  const double* cb64;
  const SidePath* side;  // null: no merged paths (hdr.tree is then ignored)
  const int32_t* share;  // per row: slots 1..share equal to the previous row's
  // wide_features: the table's segments (host copy) and their device arrays;
  // null otherwise
  const CompactTable* compact;
  const int32_t* lfeat;
  const Segment* segs;
  const int32_t* seg_feat;
  const ShortRow<float>* srow32;  // capacity-8 rows (features as the kernel indexes its tile)
  const ShortRow<double>* srow64;
};

inline PathArrays plain_arrays(const DeviceTable& d, const HostTable& h) {
  const bool w = !h.compact.segs.empty();
  return PathArrays{d.hdr, d.feat, d.lo, d.hi, d.b32, d.cb32, d.b64, d.cb64, nullptr, d.share,
                    w ? &h.compact : nullptr, d.lfeat, d.segs, d.seg_feat, d.srow32, d.srow64};
}
inline PathArrays merged_arrays(const DeviceTable& d, const HostTable& h) {
  const bool w = !h.mcompact.segs.empty();
  return PathArrays{d.mhdr, d.mfeat, d.mlo, d.mhi, d.mb32, d.mcb32, d.mb64, d.mcb64, d.side,
                    d.mshare, w ? &h.mcompact : nullptr, d.mlfeat, d.msegs, d.mseg_feat,
                    d.msrow32, d.msrow64};
}

// Slot 0 of a first-order row with its leaf value folded in, built per call
// from the current leaf values (launch_slot0).  The row's polynomial is
//   F_0(t) prod_{j >= 1} F_j(t),  F_0(t) = bm + t c,
// c = ca when the sample is in A's interval on slot 0's feature, else cb when
// it is in B's, else -bm.  A merged sibling pair: bm = vA b_A + vB b_B,
// ca = vA (1 - b_A) - vB b_B, cb = vB (1 - b_B) - vA b_A.  A single path with
// value v: bm = v b_0, ca = v (1 - b_0), cb = -bm (B's interval is A's).  The
// products are taken in FP64 and rounded once to T.
template <typename T>
struct Slot0 {
  T bm, ca, cb;
  float lo_b, hi_b;  // B's interval on slot 0's feature (hi = NaN: no bound)
  int32_t mok_b;     // 1: a NaN follows B's splits there
};

// Launch shape of the first-order (and adjoint) kernel for one bucket.
struct ValuesShape {
  int waves_per_block = 8;  // wavefronts sharing one 64-sample tile
  int items = 16384;        // target number of (sample block, path chunk) work items
};

// Launch shape of the interactions kernel for one capacity class.
struct PairShape {
  int max_chunk = 65536;  // most paths per (sample, chunk) work item
  int fill = 2048;        // least work items when there are few samples
};

inline size_t values_lds_bytes(int F) {
  size_t xs = (size_t)F * kTileStride * sizeof(float);
  xs = (xs + 15) & ~(size_t)15;
  return xs + (size_t)F * kTileStride * sizeof(double);
}

// Largest F whose tile + FP64 accumulator fit in one workgroup's LDS.
constexpr int kMaxLdsBytes = 160 * 1024;

// Work item of workgroup b of n.  The dispatcher deals workgroups to the 8
// XCDs in turn (b goes to XCD b mod 8); the workgroups of one XCD take one
// contiguous eighth of the items, so its L2 serves the data of neighbouring
// items (the last n mod 8 workgroups keep their own index).
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int kXcds = 8;
  const int per = n / kXcds;
  if (b >= per * kXcds) return b;
  return (b % kXcds) * per + b / kXcds;
}

// Wave-uniform load through the scalar data cache: reading through the
// constant address space lets the compiler emit s_load for an address that is
// uniform across the wave (path data read by every lane of a wavefront).
template <class T>
__device__ __forceinline__ T ldu(const T* p) {
  return *reinterpret_cast<const __attribute__((address_space(4))) T*>(
      reinterpret_cast<const __attribute__((address_space(4))) char*>(
          (const __attribute__((address_space(4))) void*)p));
}

// Wavefront reductions with DPP (no LDS): inclusive steps inside each row of
// 16 lanes (row_shr 1, 2, 4, 8; a lane with no source takes `old`, the
// identity), then across rows (row_bcast 15 into rows 1 and 3, row_bcast 31
// into rows 2 and 3).  Lane 63 then holds the reduction of all 64 lanes.
// Every lane of the wavefront must be active.
__device__ __forceinline__ int dpp_step(int old, int v, int st) {
  switch (st) {
    case 0: return __builtin_amdgcn_update_dpp(old, v, 0x111, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_update_dpp(old, v, 0x112, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_update_dpp(old, v, 0x114, 0xf, 0xf, false);
    case 3: return __builtin_amdgcn_update_dpp(old, v, 0x118, 0xf, 0xf, false);
    case 4: return __builtin_amdgcn_update_dpp(old, v, 0x142, 0xa, 0xf, false);
    default: return __builtin_amdgcn_update_dpp(old, v, 0x143, 0xc, 0xf, false);
  }
}

__device__ __forceinline__ double dpp_step(double old, double v, int st) {
  const long long o = __double_as_longlong(old), b = __double_as_longlong(v);
  const int lo = dpp_step((int)(o & 0xffffffffLL), (int)(b & 0xffffffffLL), st);
  const int hi = dpp_step((int)(o >> 32), (int)(b >> 32), st);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float dpp_step(float old, float v, int st) {
  return __int_as_float(dpp_step(__float_as_int(old), __float_as_int(v), st));
}

__device__ __forceinline__ float read_lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double read_lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Product over the wavefront, returned to every lane.
template <typename T>
__device__ __forceinline__ T wave_prod(T v) {
#pragma unroll
  for (int st = 0; st < 6; ++st) v *= dpp_step(T(1), v, st);
  return read_lane63(v);
}

// Sum over the wavefront, valid in lane 63 only.
__device__ __forceinline__ double wave_sum_last(double v) {
#pragma unroll
  for (int st = 0; st < 6; ++st) v += dpp_step(0.0, v, st);
  return v;
}

// Raise a kernel's dynamic-LDS limit on the current device (once per kernel
// and device; thread-safe); returns the usable dynamic LDS bytes.
size_t raise_lds_limit(const void* fn);

void launch_fill_zero(double* p, int64_t n, hipStream_t s);
// Seeded uniform values in [-3, 3) (inputs for timing launch shapes).
void launch_fill_uniform(float* p, int64_t n, uint32_t seed, hipStream_t s);
void launch_cast_f64_f32(const double* src, float* dst, int64_t n, hipStream_t s);
void launch_widen_f32_f64(const float* src, double* dst, int64_t n, hipStream_t s);
// Batched transposes: dst[b][c][r] = src[b][r][c], r < R, c < C (row strides
// lds and ldd, batch strides sbs and dbs, nbatch batches), with a cast.
void launch_transpose(const float* src, int64_t R, int64_t C, int64_t lds, int64_t sbs,
                      float* dst, int64_t ldd, int64_t dbs, int32_t nbatch, hipStream_t s);
void launch_transpose(const double* src, int64_t R, int64_t C, int64_t lds, int64_t sbs,
                      double* dst, int64_t ldd, int64_t dbs, int32_t nbatch, hipStream_t s);
void launch_transpose(const double* src, int64_t R, int64_t C, int64_t lds, int64_t sbs,
                      float* dst, int64_t ldd, int64_t dbs, int32_t nbatch, hipStream_t s);
// out[i] = sum_r part[r * n + i] over r = 0 .. nrows-1, in that order.
void launch_sum_rows(const double* part, int64_t nrows, int64_t n, double* out, hipStream_t s);

// Fill Slot0<float> (fp64 = false) or Slot0<double> for the n_rows rows of `a`
// from leaf_val; `out` holds n_rows records.
void launch_slot0(const PathArrays& a, int32_t n_rows, const double* leaf_val, bool fp64,
                  void* out, hipStream_t s);
size_t slot0_bytes(int32_t n_rows, bool fp64);

// Accumulate phi (FP64, [M,F], pre-zeroed) over the paths of one bucket.
// `a` is plain_arrays() or, with `bk` from HostTable::mbuckets, merged_arrays();
// slot0 is launch_slot0's output for the same arrays and precision.  With
// `direct` non-null (see values_direct) phi is written there instead.
// nodes = 4 runs the d <= 8 bucket with the 4-node rule (exact there for
// first order, Theorem 2); every other bucket, and nodes = 8, use 8 nodes.
// deterministic: one wavefront per workgroup and one launch per row chunk,
// in chunk order, each adding its tiles to acc without atomics (each (sample,
// feature) has one owner per launch), so phi does not depend on scheduling.
// Wide feature spaces (wide_features(F): the table's work items are
// segments) take feature-major layouts: X is [F][ldx] (ldx >= M) and acc
// [n_groups][F][M]; `direct` is not used there.
void launch_values(const HostTable& h, const DeviceTable& d, const PathArrays& a,
                   const Bucket& bk, bool fp64, const float* X, int64_t M, int64_t ldx,
                   const void* slot0, double* acc, void* direct, const ValuesShape& shape,
                   int nodes, hipStream_t s, bool deterministic = false);
// True when a first-order call over `bks` (the table in use) with M samples
// and this launch shape is one bucket walked as one chunk: each sample block
// has a single workgroup, which may then write phi itself (launch_values with
// `direct` = phi, float or double by precision; acc unused, no zero fill and
// no cast).
bool values_direct(const std::vector<Bucket>& bks, int64_t M, const ValuesShape& shape);

// Adjoint: add J^T G over the rows of one bucket into grad_leaf (pre-zeroed);
// a merged row adds to both of its leaves.
// G is [M, F] float (fp64 = false) or double; wide feature spaces take X as
// [F][ldx] and G as [n_groups][F][M] (feature-major, as launch_values).
// part_stride > 0 (deterministic): grad_leaf is [sample blocks][part_stride],
// zeroed by the caller; each sample block stores its rows' leaf sums there
// without atomics (every leaf belongs to one row), and the caller adds the
// blocks in order (launch_sum_rows).
void launch_adjoint(const HostTable& h, const DeviceTable& d, const PathArrays& a,
                    const Bucket& bk, bool fp64, const float* X, const void* G, int64_t M,
                    int64_t ldx, double* grad_leaf, const ValuesShape& shape, int nodes,
                    hipStream_t s, int64_t part_stride = 0);

// Interactions: accumulate the FP64 pair triangle [M][F(F-1)/2] and phi [M][F]
// (both pre-zeroed) over the paths of one capacity class.
// nodes_exact: the class uses the fewest nodes exact for its capacity C
// (pair integrands have degree <= C - 2: 2 nodes for C <= 4, 4 for C <= 8,
// 6 for C <= 12, else 8), instead of the 8-node rule.
void launch_pairs(const HostTable& h, const DeviceTable& d, const PairClass& pc, bool fp64,
                  const float* X, int64_t M, int64_t ldx, const double* leaf_val, double* tri64,
                  double* phi64, const PairShape& shape, bool nodes_exact, hipStream_t s);
// Phi[M][F][F] (and phi[M][F] when non-null) in FP32 or FP64 from the accumulators.
// Third-order indices of one capacity class added into acc[M][F(F-1)(F-2)/6]
// (FP64, zeroed by the caller); acc cast to float32.
void launch_triples(const HostTable& h, const DeviceTable& d, const PairClass& pc, bool fp64,
                    const float* X, int64_t M, int64_t ldx, const double* lv, double* acc,
                    hipStream_t s);
void launch_narrow_f64_f32(const double* acc, int64_t n, float* out, hipStream_t s);

// Depth-first interactions (DfsTable): the walk writes y_v(t_m) of samples
// [s0, s0 + mb) to Y[mb][n_rows][8] (T by precision); the pair pass adds their
// pair and first-order updates into the FP64 accumulators of those samples.
size_t dfs_walk_lds_bytes(int F, int max_level, bool fp64);
// lvals: 2 values per record (T), filled from leaf_val by the launch with s0 = 0.
void launch_dfs_walk(const HostTable& h, const DeviceDfs& d, const DeviceTable& dt, bool fp64,
                     const double* leaf_val, const float* X, int64_t s0, int32_t mb,
                     int64_t ldx, void* Y, void* lvals, hipStream_t s);
// Third order (packed tensor acc[M][n_groups][F(F-1)(F-2)/6], FP64, zeroed by
// the caller) from the walk's y_v of samples [s0, s0 + mb); needs
// dfs_triples_supported(d).
bool dfs_triples_supported(const DeviceDfs& d);
void launch_dfs_triples(const HostTable& h, const DeviceDfs& d, const DeviceTable& dt, bool fp64,
                        const float* X, int64_t s0, int32_t mb, int64_t ldx, const void* Y,
                        double* acc, int32_t tiles_per_chunk, hipStream_t s);
void launch_dfs_pairs(const HostTable& h, const DeviceDfs& d, const DeviceTable& dt, bool fp64,
                      const float* X, int64_t s0, int32_t mb, int64_t ldx, const void* Y,
                      double* tri64, double* phi64, int32_t tiles_per_chunk, hipStream_t s);
void launch_pairs_finalize(const double* tri64, const double* phi64, int64_t M, int F, bool fp64,
                           void* Phi, void* phi, hipStream_t s);

void check_hip(hipError_t e, const char* what);

}  // namespace qts
