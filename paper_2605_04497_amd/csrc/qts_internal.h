// Internal structures shared by the host library and the kernel launchers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "qtreeshap.h"

namespace qts {

constexpr int kNodes = 8;          // fixed Gauss-Legendre node count (section 5)
constexpr int kMaxDepth = 128;     // deeper trees are rejected (QTS_E_UNSUPPORTED)
constexpr int kMaxUnique = 64;     // longer collapsed paths are rejected
constexpr int kSamplesPerBlock = 64;  // one explained sample per wavefront lane

// Error raised inside the library; converted to a return code at the C-ABI.
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

// Per-path header, 16 bytes so one scalar load fetches it.
struct alignas(16) PathHdr {
  int32_t off;   // first element of the path in the element arrays
  int32_t d;     // unique features on the path
  int32_t leaf;  // leaf ordinal (tree-major, node-id order)
  int32_t tree;
};

// Element flag: bit 30 of the packed feature word marks "a NaN follows every
// split of this feature on the path" (missing_ok).
constexpr int32_t kMissingOkBit = 1 << 30;
constexpr int32_t kFeatureMask = kMissingOkBit - 1;

// Paths with the same unique-feature capacity are stored contiguously.
// With several outputs (tree groups), a bucket holds one group's paths.
struct Bucket {
  int32_t dmax;        // capacity of the kernel instance (8, 16, 32 or 64)
  int32_t path_begin;  // [path_begin, path_end) in path order
  int32_t path_end;
  int64_t elems;       // sum of d over the bucket's paths
  int32_t group = 0;   // output group of the bucket's trees
  int32_t srow_begin = -1;  // capacity 8: index of its first row in the short-row records
};

// Sibling record of a merged path.  Two leaves A (left) and B (right) of one
// parent have the same collapsed feature set and the same elements except the
// one of the parent's split feature L; the val-weighted sum of their
// polynomials is one polynomial whose L factor is vA F_A + vB F_B (linear in
// p, like any factor).  The merged path keeps A's elements with L moved to
// slot 0 (A's interval there) and this record holds B's side of slot 0.
struct alignas(16) SidePath {
  float lo_b, hi_b;  // B's interval on L (hi = NaN: no upper bound)
  int32_t leaf_b;    // B's leaf ordinal
  int32_t mok_b;     // 1: a NaN follows B's splits on L
  double b_a, cb_a;  // A's b_L and 1 - b_L (FP64)
  double b_b, cb_b;  // B's b_L and 1 - b_L (FP64)
};

// Feature-compacted segments of a first-order table.  The first-order and
// adjoint kernels stage a workgroup's 64 samples transposed in LDS, F floats
// plus F doubles of accumulator per sample; when that tile does not fit
// (wide_features), each work item takes instead a segment: consecutive rows
// of one bucket whose elements use at most kSegFeatures distinct features.
// The kernel stages only those features and addresses them by their index in
// the segment's feature list (lfeat), then adds its accumulators to phi at
// the features' global ids.
constexpr int kSegFeatures = 96;   // tile features per segment (75 KB of LDS)
constexpr int kSegMaxRows = 2048;  // rows per segment at most
constexpr int kTileLdsBudget = 160 * 1024;
inline bool wide_features(int F) {
  const size_t xs = ((size_t)F * 65 * sizeof(float) + 15) & ~(size_t)15;
  return xs + (size_t)F * 65 * sizeof(double) > (size_t)kTileLdsBudget;
}
struct Segment {
  int32_t row_begin, row_end;  // rows [row_begin, row_end) of the table
  int32_t feat_begin;          // first entry of the segment's list in seg_feat
  int32_t nfeat;               // distinct features of its rows (<= kSegFeatures)
};
struct CompactTable {
  std::vector<Segment> segs;        // every bucket's segments, in row order
  std::vector<int32_t> bucket_seg;  // [n_buckets + 1]: segments of bucket i
  std::vector<int32_t> seg_feat;    // global feature ids, per segment
  std::vector<int32_t> lfeat;       // per element: index in its segment's list | missing_ok
};
CompactTable build_compact(const std::vector<PathHdr>& hdr,
                           const std::vector<int32_t>& feat,
                           const std::vector<Bucket>& bks, int32_t F);

// Collapsed path table in host memory (built once per model).
struct HostTable {
  int32_t F = 0;
  int32_t n_groups = 1;  // outputs: every tree adds to the output of its group
  int32_t n_trees = 0;
  int32_t max_depth = 0;
  int32_t max_unique = 0;
  double base_score = 0.0;
  double expected = 0.0;  // sum_T E_T[f] + base_score (group 0)
  std::vector<double> expected_g;  // per group: sum over its trees of E_T[f] + its base score
  std::vector<PathHdr> hdr;
  std::vector<int32_t> feat;  // packed: feature | missing_ok bit
  std::vector<float> lo, hi;
  std::vector<double> b, cb;  // b_j and 1 - b_j, FP64
  std::vector<double> leaf_value;
  std::vector<int32_t> tree_group;  // [n_trees]
  std::vector<Bucket> buckets;
  // per row of a table with at most 8 features: the number s of slots
  // 1..s equal to the previous row's (0 for other rows); see prefix_share
  std::vector<int32_t> share;
  // The first-order table with sibling leaves merged: same layout; a merged
  // path has hdr.tree = its SidePath index (-1 for an unmerged path).
  std::vector<PathHdr> mhdr;
  std::vector<int32_t> mfeat;
  std::vector<float> mlo, mhi;
  std::vector<double> mb, mcb;
  std::vector<Bucket> mbuckets;
  std::vector<SidePath> side;
  std::vector<int32_t> mshare;
  // wide_features(F): the segments of both first-order tables
  CompactTable compact, mcompact;
};

// tree_group: [n_trees] output group of each tree (null: all in group 0);
// base_scores: [n_groups].
HostTable build_host_table(const qts_tree_arrays& t, int32_t n_features, int32_t n_groups,
                           const int32_t* tree_group, const double* base_scores);

// Path table for the interactions kernel: rows grouped by capacity class
// (4, 8, ..., 40, 48, 64 slots: the kernel instances), sorted by length
// inside a class with neighbouring rows taken from different trees, stored
// slot-major ([slot][row] within a class) so one lane per row reads
// coalesced.  A row is a path, or a merged pair of sibling leaves of at most
// kPairMergeMax features (SidePath in `side`, the combined split feature in
// slot 0); the remaining slots are sorted by feature (a single path: all of
// them).  Slots past a row's end are inert (feature 0, no bounds,
// missing_ok, b = 1, 1-b = 0).
constexpr int kPairMergeMax = 16;
struct PairClass {
  int32_t cap;    // slots per path
  int32_t np;     // paths in the class
  int64_t base;   // first element of the class (slot-major block of cap * np)
  int32_t pbase;  // first path of the class in the per-path arrays
  int32_t group = 0;  // output group of the class's rows
};

struct PairTable {
  std::vector<PairClass> classes;
  std::vector<int32_t> d, leaf;          // per row
  std::vector<SidePath> side;            // per row (leaf_b = -1: a single path)
  std::vector<int32_t> feat;             // packed: feature | missing_ok bit
  std::vector<float> lo, hi;
  std::vector<double> b, cb;
};

PairTable build_pair_table(const HostTable& h);

// Tables of the depth-first form of the interactions (section 5, Algorithm 1
// at order 2, with the telescoping update of Eq. 11).  For an internal node v
// with split feature f and children u, let (b_j, o_j) be feature j's cover
// product and follow indicator over the splits on j above v (b = o = 1 when
// j is not split there), F_j = b_j + t (o_j - b_j), r_j = (o_j - b_j) / F_j,
// and H_u(t) the sum over the leaves below u of val * prod F (the leaf's own
// factors).  Summing the change of r_f across the edge v -> u over the
// subtree, with every other feature at its value at v, gives
//   y_v(t_m) = w_m sum_u H_u(t_m) (r_f^u - r_f^v)(t_m),
//   phi_f   += sum_m y_v(t_m),
//   SII_fj  += sum_m y_v(t_m) r_j^v(t_m)   for the features j != f split above v,
// and the telescoping sum over a path's edges reproduces Theorem 1's
// products.  The change of r is taken without cancellation as
//   r_f^u - r_f^v = (o^u b^v - o^v b^u) / (F^u F^v),
// and o^u b^v - o^v b^u is b^v - b^u (FP64 from the covers), -b^u or 0.
// The tree walk (one wavefront per tree and group of samples) forms y_v for
// every internal node; the pair pass (lane per node) adds the updates.
struct alignas(16) DfsNode {
  int32_t f;        // split feature
  int32_t level;    // depth of the node (root 0)
  int32_t parent;   // record of the parent node, -1 at the root
  int32_t flags;    // kDfs* bits
  int32_t left, right;      // records of internal children, -1 for a leaf
  int32_t leaf_l, leaf_r;   // leaf ordinals of leaf children, -1 otherwise
  int32_t row;      // the node's row of the pair pass (where y_v is stored)
  float lo_v, hi_v;         // the interval of f's splits above v (no bound: -inf / NaN)
  float lo_l, hi_l, lo_r, hi_r;  // the same including the edge to each child
  int32_t pad;
};
constexpr int32_t kDfsLeftChild = 1;  // the node is its parent's left child
constexpr int32_t kDfsFresh = 2;      // f is not split above the node
constexpr int32_t kDfsMokV = 4;       // a NaN follows every split on f above the node
constexpr int32_t kDfsMokL = 8;       // ... and the edge to the left child
constexpr int32_t kDfsMokR = 16;      // ... and the edge to the right child
// Per node, FP64: b^v, 1 - b^v, b^L, 1 - b^L, b^R, 1 - b^R, b^v - b^L, b^v - b^R.
constexpr int kDfsCoef = 8;

// The walk of a tree as a linear stream of events, in the order a depth-first
// walk meets them: per internal node, enter (go down the left edge), middle
// (left subtree done, go down the right edge) and exit (both done).  An event
// is record << 2 | kind, so the walk reads its control in order instead of
// following child and parent links.
constexpr int32_t kDfsEnter = 0, kDfsMiddle = 1, kDfsExit = 2;

struct DfsTable {
  std::vector<DfsNode> nodes;    // per tree, internal nodes in preorder
  std::vector<double> coef;      // kDfsCoef per node
  std::vector<int32_t> events;   // per tree, 3 per internal node
  std::vector<int32_t> tree_first, tree_nodes;  // trees with a split, largest first
                                               // (first record; events start at 3 x it)
  int32_t max_level = 0;
  // pair pass: one row per internal node, rows of a group sorted by length
  // and padded to whole tiles of 64 rows; element (slot k, lane i) of tile t
  // at tile_base[t] + 64 k + i (slot-major inside the tile)
  int32_t n_rows = 0;
  std::vector<int32_t> row_f;    // split feature (-1: padding row)
  std::vector<int32_t> row_d;    // features split above the node, other than f
  std::vector<int32_t> tile_base, tile_d;
  std::vector<int32_t> group_tile;  // [n_groups + 1]: tiles of each group
  std::vector<int32_t> feat;     // feature | missing_ok; a row's features ascending
  std::vector<float> lo, hi;
  std::vector<double> b, cb;
  int64_t n_updates = 0;         // sum of row_d: pair updates per sample
  int64_t n_updates3 = 0;        // sum of row_d (row_d - 1) / 2: third-order updates
  int32_t max_row_d = 0;
};

DfsTable build_dfs_table(const qts_tree_arrays& t, const HostTable& h);

// Golub-Welsch: n-node Gauss-Legendre rule on [0,1] in FP64.
void gauss_legendre(int n, double* t, double* one_minus_t, double* w);

}  // namespace qts
