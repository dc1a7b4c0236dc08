// Model validation and the collapsed, bucketed path table (host side).
//
// For each leaf the root-to-leaf path is collapsed to its unique features, in
// order of first appearance.  For feature j (Eq. 2 and section 2):
//   b_j        = product of w_e = cover(child)/cover(parent) over the path's
//                splits on j (w_e = 0 when the parent cover is 0), in FP64;
//   1 - b_j    computed in FP64 (not from a rounded b_j);
//   [lo, hi)   the x values that satisfy every split on j: a left edge needs
//              x < threshold, a right edge x >= threshold (hi = NaN: no bound);
//   missing_ok a NaN value follows every split on j (all default directions
//              along the path agree with the path).
// E[f] = sum over leaves of val * prod_j b_j  (Eq. 1, the game at S = empty).
// Paths with the same unique-feature capacity (8, 16, 32, 64) are stored
// contiguously so one kernel instance with a fixed register budget serves them.
//
// A second table serves the first-order kernel: there, two leaves that are
// the children of one node are one merged path (see SidePath).  Their
// polynomials differ only in the factor of the parent's split feature L, and
// phi is linear in each leaf's polynomial, so
//   vA prod_j F^A_j + vB prod_j F^B_j = prod_{j != L} F_j * (vA F^A_L + vB F^B_L)
// exactly: the merged path carries the combined factor in slot 0 and a leaf
// value of 1.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "../qts_internal.h"

namespace qts {

namespace {

struct Edge {
  int32_t f;
  bool left;
  float thr;
  bool dleft;
  double w;
  int32_t parent;  // node the edge leaves
};

struct RawPath {
  int32_t leaf;
  int32_t tree;
  int32_t group = 0;  // output group of the tree
  int32_t parent = -1;     // parent node of the leaf (-1: the root is the leaf)
  bool left_child = false;
  std::vector<int32_t> feat;
  std::vector<float> lo, hi;
  std::vector<uint8_t> mok;
  std::vector<double> b;
};

int bucket_capacity(int d) {
  if (d <= 8) return 8;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  return 64;
}

class Builder {
 public:
  Builder(const qts_tree_arrays& t, int32_t F) : t_(t), F_(F) {}

  void tree(int32_t ti, int32_t group) {
    group_ = group;
    const int64_t a = t_.tree_offsets[ti], e = t_.tree_offsets[ti + 1];
    if (e <= a) fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(ti) + " has no nodes");
    if (e - a > (int64_t)std::numeric_limits<int32_t>::max())
      fail(QTS_E_UNSUPPORTED, "tree " + std::to_string(ti) + " is too large");
    base_ = a;
    n_ = (int32_t)(e - a);
    tree_ = ti;
    visited_.assign((size_t)n_, 0);
    // leaf ordinals in node-id order (every node with left < 0 is a leaf slot)
    leaf_ord_.assign((size_t)n_, -1);
    for (int32_t i = 0; i < n_; ++i)
      if (t_.left[a + i] < 0) leaf_ord_[(size_t)i] = (int32_t)(n_leaves_++);
    path_.clear();
    visit(0, 0);
  }

  std::vector<RawPath> paths;
  std::vector<double> leaf_value;
  std::vector<double> expected;  // per output group
  int32_t max_depth = 0;
  int32_t max_unique = 0;
  int64_t n_leaves_ = 0;

 private:
  void visit(int32_t node, int32_t depth) {
    if (node < 0 || node >= n_)
      fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(tree_) + ": child id out of range");
    if (visited_[(size_t)node])
      fail(QTS_E_INVALID_MODEL,
           "tree " + std::to_string(tree_) + ": node reached twice (cycle or shared child)");
    visited_[(size_t)node] = 1;
    if (depth > kMaxDepth)
      fail(QTS_E_UNSUPPORTED, "tree " + std::to_string(tree_) + " is deeper than 128");
    const int64_t g = base_ + node;
    const double cov = t_.cover[g];
    if (!(cov >= 0.0))
      fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(tree_) + ": negative or NaN cover");
    const int32_t l = t_.left[g], r = t_.right[g];
    if (l < 0 || r < 0) {
      if (l >= 0 || r >= 0)
        fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(tree_) + ": node with one child");
      leaf(node, depth);
      return;
    }
    const int32_t f = t_.feature[g];
    if (f < 0 || f >= F_)
      fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(tree_) + ": feature out of range");
    const float thr = t_.threshold[g];
    if (std::isnan(thr))
      fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(tree_) + ": NaN threshold");
    if (l >= n_ || r >= n_)
      fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(tree_) + ": child id out of range");
    const bool dl = t_.default_left ? (t_.default_left[g] != 0) : false;
    for (int c = 0; c < 2; ++c) {
      const int32_t child = c == 0 ? l : r;
      const double cc = t_.cover[base_ + child];
      const double w = cov == 0.0 ? 0.0 : cc / cov;
      path_.push_back(Edge{f, c == 0, thr, dl, w, node});
      visit(child, depth + 1);
      path_.pop_back();
    }
  }

  void leaf(int32_t node, int32_t depth) {
    const int64_t g = base_ + node;
    max_depth = std::max(max_depth, depth);
    RawPath p;
    p.leaf = leaf_ord_[(size_t)node];
    p.tree = tree_;
    p.group = group_;
    if (!path_.empty()) {
      p.parent = path_.back().parent;
      p.left_child = path_.back().left;
    }
    const float kNoBound = std::numeric_limits<float>::quiet_NaN();
    for (const Edge& e : path_) {
      size_t k = 0;
      while (k < p.feat.size() && p.feat[k] != e.f) ++k;
      if (k == p.feat.size()) {
        p.feat.push_back(e.f);
        p.lo.push_back(-std::numeric_limits<float>::infinity());
        p.hi.push_back(kNoBound);
        p.mok.push_back(1);
        p.b.push_back(1.0);
      }
      p.b[k] *= e.w;
      if (e.left) {
        p.hi[k] = std::isnan(p.hi[k]) ? e.thr : std::min(p.hi[k], e.thr);
        p.mok[k] &= (uint8_t)(e.dleft ? 1 : 0);
      } else {
        p.lo[k] = std::max(p.lo[k], e.thr);
        p.mok[k] &= (uint8_t)(e.dleft ? 0 : 1);
      }
    }
    const int d = (int)p.feat.size();
    if (d > kMaxUnique)
      fail(QTS_E_UNSUPPORTED, "a path has more than 64 unique features");
    max_unique = std::max(max_unique, d);
    const double val = t_.value[g];
    if (leaf_value.size() <= (size_t)p.leaf) leaf_value.resize((size_t)p.leaf + 1, 0.0);
    leaf_value[(size_t)p.leaf] = val;
    double prod = val;
    for (double bj : p.b) prod *= bj;
    expected[(size_t)group_] += prod;
    if (d > 0) paths.push_back(std::move(p));
  }

  const qts_tree_arrays& t_;
  int32_t F_;
  int32_t group_ = 0;
  int64_t base_ = 0;
  int32_t n_ = 0;
  int32_t tree_ = 0;
  std::vector<uint8_t> visited_;
  std::vector<int32_t> leaf_ord_;
  std::vector<Edge> path_;
};

}  // namespace

// Per row of a table: the number s of leading slots 1..s whose elements
// (feature, missing_ok, interval, b) are identical to the previous row's.
// Rows are in tree order with leaves left to right (stably grouped by
// length bucket), so neighbours share the root side of their paths; slot 0
// is each row's own factor and is never shared.
static std::vector<int32_t> prefix_share(const std::vector<PathHdr>& hdr,
                                         const std::vector<int32_t>& feat,
                                         const std::vector<float>& lo,
                                         const std::vector<float>& hi,
                                         const std::vector<double>& b) {
  auto same_bits = [](auto x, auto y) { return std::memcmp(&x, &y, sizeof(x)) == 0; };
  std::vector<int32_t> share(hdr.size(), 0);
  for (size_t r = 1; r < hdr.size(); ++r) {
    const PathHdr& a = hdr[r];
    const PathHdr& q = hdr[r - 1];
    const int n = std::min(a.d, q.d);
    int k = 1;
    for (; k < n; ++k) {
      const size_t i = (size_t)a.off + (size_t)k, j = (size_t)q.off + (size_t)k;
      if (feat[i] != feat[j] || !same_bits(lo[i], lo[j]) || !same_bits(hi[i], hi[j]) ||
          !same_bits(b[i], b[j]))
        break;
    }
    share[r] = k - 1;
  }
  return share;
}

CompactTable build_compact(const std::vector<PathHdr>& hdr, const std::vector<int32_t>& feat,
                           const std::vector<Bucket>& bks, int32_t F) {
  CompactTable c;
  c.lfeat.assign(feat.size(), 0);
  std::vector<int32_t> local((size_t)F, -1);  // feature -> index in the open segment
  std::vector<int32_t> open;                  // the open segment's features
  c.bucket_seg.push_back(0);
  for (const Bucket& bk : bks) {
    int32_t r = bk.path_begin;
    while (r < bk.path_end) {
      Segment sg{r, r, (int32_t)c.seg_feat.size(), 0};
      open.clear();
      while (r < bk.path_end && r - sg.row_begin < kSegMaxRows) {
        // the row joins if its new features still fit the tile
        const PathHdr& p = hdr[(size_t)r];
        int fresh = 0;
        for (int k = 0; k < p.d; ++k) {
          const int32_t f = feat[(size_t)p.off + (size_t)k] & kFeatureMask;
          if (local[(size_t)f] < 0) {
            local[(size_t)f] = -2;  // counted once
            ++fresh;
          }
        }
        for (int k = 0; k < p.d; ++k) {
          const int32_t f = feat[(size_t)p.off + (size_t)k] & kFeatureMask;
          if (local[(size_t)f] == -2) local[(size_t)f] = -1;
        }
        if ((int)open.size() + fresh > kSegFeatures) break;  // a row has <= 64 < kSegFeatures
        for (int k = 0; k < p.d; ++k) {
          const size_t e = (size_t)p.off + (size_t)k;
          const int32_t f = feat[e] & kFeatureMask;
          if (local[(size_t)f] < 0) {
            local[(size_t)f] = (int32_t)open.size();
            open.push_back(f);
          }
          c.lfeat[e] = local[(size_t)f] | (feat[e] & kMissingOkBit);
        }
        ++r;
      }
      sg.row_end = r;
      sg.nfeat = (int32_t)open.size();
      for (int32_t f : open) {
        c.seg_feat.push_back(f);
        local[(size_t)f] = -1;
      }
      c.segs.push_back(sg);
    }
    c.bucket_seg.push_back((int32_t)c.segs.size());
  }
  return c;
}

HostTable build_host_table(const qts_tree_arrays& t, int32_t F, int32_t n_groups,
                           const int32_t* tree_group, const double* base_scores) {
  if (F < 1) fail(QTS_E_INVALID_ARG, "n_features must be >= 1");
  if (n_groups < 1) fail(QTS_E_INVALID_ARG, "n_groups must be >= 1");
  if (!base_scores) fail(QTS_E_INVALID_ARG, "null base scores");
  if (t.n_trees < 0) fail(QTS_E_INVALID_ARG, "n_trees must be >= 0");
  if (t.n_trees > 0 && (!t.tree_offsets || !t.left || !t.right || !t.feature || !t.threshold ||
                        !t.cover || !t.value))
    fail(QTS_E_INVALID_ARG, "null tree array");
  if (t.n_trees > 0 && t.tree_offsets[0] != 0)
    fail(QTS_E_INVALID_MODEL, "tree_offsets[0] must be 0");
  Builder bld(t, F);
  bld.expected.assign((size_t)n_groups, 0.0);
  std::vector<int32_t> groups((size_t)std::max(0, t.n_trees), 0);
  for (int32_t ti = 0; ti < t.n_trees; ++ti) {
    const int32_t g = tree_group ? tree_group[ti] : 0;
    if (g < 0 || g >= n_groups)
      fail(QTS_E_INVALID_MODEL, "tree " + std::to_string(ti) + ": output group out of range");
    groups[(size_t)ti] = g;
    bld.tree(ti, g);
  }
  if (bld.n_leaves_ > (int64_t)std::numeric_limits<int32_t>::max() / 2)
    fail(QTS_E_UNSUPPORTED, "too many leaves");

  HostTable h;
  h.F = F;
  h.n_groups = n_groups;
  h.n_trees = t.n_trees;
  h.max_depth = bld.max_depth;
  h.max_unique = bld.max_unique;
  h.base_score = base_scores[0];
  h.expected_g.resize((size_t)n_groups);
  for (int32_t g = 0; g < n_groups; ++g)
    h.expected_g[(size_t)g] = bld.expected[(size_t)g] + base_scores[g];
  h.expected = h.expected_g[0];
  h.leaf_value = std::move(bld.leaf_value);
  h.leaf_value.resize((size_t)bld.n_leaves_, 0.0);

  // group paths by capacity, keeping tree-major order inside a group
  std::vector<size_t> order(bld.paths.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  // buckets: runs of equal (capacity, output group)
  auto bucket_key = [&](const RawPath& p) {
    return std::make_pair(bucket_capacity((int)p.feat.size()), p.group);
  };
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    return bucket_key(bld.paths[x]) < bucket_key(bld.paths[y]);
  });
  int64_t n_el = 0;
  for (const RawPath& p : bld.paths) n_el += (int64_t)p.feat.size();
  if (n_el > (int64_t)std::numeric_limits<int32_t>::max())
    fail(QTS_E_UNSUPPORTED, "path table too large");
  h.hdr.reserve(order.size());
  h.feat.reserve((size_t)n_el);
  h.lo.reserve((size_t)n_el);
  h.hi.reserve((size_t)n_el);
  h.b.reserve((size_t)n_el);
  h.cb.reserve((size_t)n_el);
  for (size_t idx : order) {
    const RawPath& p = bld.paths[idx];
    const int d = (int)p.feat.size();
    const int cap = bucket_capacity(d);
    const int32_t pi = (int32_t)h.hdr.size();
    if (h.buckets.empty() || h.buckets.back().dmax != cap || h.buckets.back().group != p.group)
      h.buckets.push_back(Bucket{cap, pi, pi, 0, p.group});
    h.buckets.back().path_end = pi + 1;
    h.buckets.back().elems += d;
    h.hdr.push_back(PathHdr{(int32_t)h.feat.size(), d, p.leaf, p.tree});
    for (int k = 0; k < d; ++k) {
      h.feat.push_back(p.feat[k] | (p.mok[k] ? kMissingOkBit : 0));
      h.lo.push_back(p.lo[k]);
      h.hi.push_back(p.hi[k]);
      h.b.push_back(p.b[k]);
      h.cb.push_back(1.0 - p.b[k]);
    }
  }

  // Merged first-order table.  Leaves are visited left child first, so two
  // leaf siblings are consecutive in bld.paths.
  struct Unit {
    size_t a;
    int side;  // -1: a single path
  };
  std::vector<Unit> units;
  std::vector<size_t> slot0;  // per unit: the element that goes to slot 0
  for (size_t i = 0; i < bld.paths.size(); ++i) {
    const RawPath& A = bld.paths[i];
    if (i + 1 < bld.paths.size()) {
      const RawPath& B = bld.paths[i + 1];
      if (A.parent >= 0 && B.parent == A.parent && B.tree == A.tree && A.left_child &&
          !B.left_child && A.feat.size() == B.feat.size()) {
        // the parent's split feature: the only element where A and B differ
        const int32_t L = t.feature[t.tree_offsets[A.tree] + A.parent];
        size_t kL = 0;
        while (kL < A.feat.size() && A.feat[kL] != L) ++kL;
        if (kL == A.feat.size()) fail(QTS_E_INVALID_MODEL, "internal: split feature not on path");
        SidePath sp;
        sp.lo_b = B.lo[kL];
        sp.hi_b = B.hi[kL];
        sp.leaf_b = B.leaf;
        sp.mok_b = B.mok[kL] ? 1 : 0;
        sp.b_a = A.b[kL];
        sp.cb_a = 1.0 - A.b[kL];
        sp.b_b = B.b[kL];
        sp.cb_b = 1.0 - B.b[kL];
        units.push_back(Unit{i, (int)h.side.size()});
        h.side.push_back(sp);
        slot0.push_back(kL);
        ++i;
        continue;
      }
    }
    // a single path: its deepest feature takes slot 0, so slots 1.. keep the
    // root-first order that merged neighbours have there
    units.push_back(Unit{i, -1});
    slot0.push_back(bld.paths[i].feat.empty() ? 0 : bld.paths[i].feat.size() - 1);
  }
  std::vector<size_t> morder(units.size());
  for (size_t i = 0; i < morder.size(); ++i) morder[i] = i;
  std::stable_sort(morder.begin(), morder.end(), [&](size_t x, size_t y) {
    return bucket_key(bld.paths[units[x].a]) < bucket_key(bld.paths[units[y].a]);
  });
  for (size_t ui : morder) {
    const RawPath& p = bld.paths[units[ui].a];
    const int d = (int)p.feat.size();
    const int cap = bucket_capacity(d);
    const int32_t pi = (int32_t)h.mhdr.size();
    if (h.mbuckets.empty() || h.mbuckets.back().dmax != cap ||
        h.mbuckets.back().group != p.group)
      h.mbuckets.push_back(Bucket{cap, pi, pi, 0, p.group});
    h.mbuckets.back().path_end = pi + 1;
    h.mbuckets.back().elems += d;
    h.mhdr.push_back(PathHdr{(int32_t)h.mfeat.size(), d, p.leaf, units[ui].side});
    // element order: the merged (or a single path's deepest) slot first, the
    // others in path order
    const size_t kL = slot0[ui];
    for (int r = 0; r < d; ++r) {
      const size_t k = r == 0 ? kL : ((size_t)r <= kL ? (size_t)r - 1 : (size_t)r);
      h.mfeat.push_back(p.feat[k] | (p.mok[k] ? kMissingOkBit : 0));
      h.mlo.push_back(p.lo[k]);
      h.mhi.push_back(p.hi[k]);
      h.mb.push_back(p.b[k]);
      h.mcb.push_back(1.0 - p.b[k]);
    }
  }
  h.tree_group = std::move(groups);
  h.share = prefix_share(h.hdr, h.feat, h.lo, h.hi, h.b);
  h.mshare = prefix_share(h.mhdr, h.mfeat, h.mlo, h.mhi, h.mb);
  // the rows of capacity-8 buckets, numbered in bucket order, index the
  // short-row records of each table
  for (std::vector<Bucket>* bks : {&h.buckets, &h.mbuckets}) {
    int32_t n = 0;
    for (Bucket& bk : *bks)
      if (bk.dmax == 8) {
        bk.srow_begin = n;
        n += bk.path_end - bk.path_begin;
      }
  }
  if (wide_features(F)) {
    h.compact = build_compact(h.hdr, h.feat, h.buckets, F);
    h.mcompact = build_compact(h.mhdr, h.mfeat, h.mbuckets, F);
  }
  return h;
}

}  // namespace qts

namespace qts {

PairTable build_pair_table(const HostTable& h) {
  PairTable pt;
  // capacities of the interactions kernel instances
  auto cap_of = [](int d) {
    static const int caps[] = {4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 48, 64};
    for (int c : caps)
      if (d <= c) return c;
    return 64;
  };
  // Rows: one per merged pair of sibling leaves of at most kPairMergeMax
  // features (the register-resident kernel instances take them), one per
  // other path.  A merged row of the first-order table that is longer is
  // split back into its two paths: A keeps the row's elements, B differs in
  // slot 0 (the parent's split feature) only.
  std::vector<int32_t> tree_of_leaf(h.leaf_value.size(), 0);
  for (const PathHdr& p : h.hdr) tree_of_leaf[(size_t)p.leaf] = p.tree;
  struct Row {
    int32_t m;     // row of the merged first-order table
    int32_t side;  // SidePath index of a merged row, else -1
    bool as_b;     // the B path of a split merged row
    int32_t d, leaf, tree;
  };
  std::vector<Row> rows;
  rows.reserve(h.mhdr.size() + h.side.size());
  for (size_t m = 0; m < h.mhdr.size(); ++m) {
    const PathHdr& p = h.mhdr[m];
    const int32_t tree = tree_of_leaf[(size_t)p.leaf];
    if (p.tree >= 0 && p.d > kPairMergeMax) {
      rows.push_back(Row{(int32_t)m, -1, false, p.d, p.leaf, tree});
      rows.push_back(Row{(int32_t)m, p.tree, true, p.d, h.side[(size_t)p.tree].leaf_b, tree});
    } else {
      rows.push_back(Row{(int32_t)m, p.tree, false, p.d, p.leaf, tree});
    }
  }
  const size_t n = rows.size();
  std::vector<size_t> order(n);
  for (size_t i = 0; i < n; ++i) order[i] = i;
  // Inside a class: by length, then by the row's rank among its tree's rows
  // of that length, then by tree.  Neighbouring rows (one per lane) then come
  // from different trees, so a wave's lanes rarely add into the same pair
  // entry at the same time (paths of one tree share most of their features).
  std::vector<int32_t> rank(n, 0);
  {
    std::vector<int32_t> count((size_t)h.n_trees * (kMaxUnique + 1), 0);
    for (size_t i = 0; i < n; ++i)
      rank[i] = count[(size_t)rows[i].tree * (kMaxUnique + 1) + (size_t)rows[i].d]++;
  }
  auto group_of = [&](const Row& r) { return h.tree_group[(size_t)r.tree]; };
  std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    const int cx = cap_of(rows[x].d), cy = cap_of(rows[y].d);
    if (cx != cy) return cx < cy;
    const int gx = group_of(rows[x]), gy = group_of(rows[y]);
    if (gx != gy) return gx < gy;
    if (rows[x].d != rows[y].d) return rows[x].d < rows[y].d;
    if (rank[x] != rank[y]) return rank[x] < rank[y];
    return rows[x].tree < rows[y].tree;
  });
  // class boundaries
  size_t i = 0;
  int64_t el = 0;
  while (i < n) {
    const int cap = cap_of(rows[order[i]].d);
    const int32_t g = group_of(rows[order[i]]);
    size_t j = i;
    while (j < n && cap_of(rows[order[j]].d) == cap && group_of(rows[order[j]]) == g) ++j;
    pt.classes.push_back(PairClass{cap, (int32_t)(j - i), el, (int32_t)i, g});
    el += (int64_t)cap * (int64_t)(j - i);
    i = j;
  }
  if (el > (int64_t)std::numeric_limits<int32_t>::max())
    fail(QTS_E_UNSUPPORTED, "pair table too large");
  pt.d.resize(n);
  pt.leaf.resize(n);
  SidePath none{};
  none.leaf_b = -1;
  none.hi_b = std::numeric_limits<float>::quiet_NaN();
  none.lo_b = -std::numeric_limits<float>::infinity();
  pt.side.assign(n, none);
  pt.feat.assign((size_t)el, kMissingOkBit);
  pt.lo.assign((size_t)el, -std::numeric_limits<float>::infinity());
  pt.hi.assign((size_t)el, std::numeric_limits<float>::quiet_NaN());
  pt.b.assign((size_t)el, 1.0);
  pt.cb.assign((size_t)el, 0.0);
  std::vector<int> idx;
  for (const PairClass& c : pt.classes) {
    for (int32_t q = 0; q < c.np; ++q) {
      const size_t r = (size_t)c.pbase + (size_t)q;
      const Row& row = rows[order[r]];
      const PathHdr& p = h.mhdr[(size_t)row.m];
      pt.d[r] = row.d;
      pt.leaf[r] = row.leaf;
      const bool merged = row.side >= 0 && !row.as_b;
      if (merged) pt.side[r] = h.side[(size_t)row.side];
      // element k of the merged first-order row, with B's slot 0 for as_b
      auto fe = [&](int k) {
        if (row.as_b && k == 0) {
          const SidePath& sp = h.side[(size_t)row.side];
          return (h.mfeat[(size_t)p.off] & kFeatureMask) | (sp.mok_b ? kMissingOkBit : 0);
        }
        return h.mfeat[(size_t)p.off + (size_t)k];
      };
      // slot order: a merged row keeps its combined element in slot 0;
      // every other slot is sorted by feature (a single path: all of them)
      const int first = merged ? 1 : 0;
      idx.resize((size_t)p.d);
      for (int k = 0; k < p.d; ++k) idx[(size_t)k] = k;
      std::sort(idx.begin() + first, idx.end(), [&](int x, int y) {
        return (fe(x) & kFeatureMask) < (fe(y) & kFeatureMask);
      });
      for (int k = 0; k < p.d; ++k) {
        const int e = idx[(size_t)k];
        const size_t src = (size_t)p.off + (size_t)e;
        const size_t dst = (size_t)c.base + (size_t)k * (size_t)c.np + (size_t)q;
        pt.feat[dst] = fe(e);
        if (row.as_b && e == 0) {
          const SidePath& sp = h.side[(size_t)row.side];
          pt.lo[dst] = sp.lo_b;
          pt.hi[dst] = sp.hi_b;
          pt.b[dst] = sp.b_b;
          pt.cb[dst] = sp.cb_b;
        } else {
          pt.lo[dst] = h.mlo[src];
          pt.hi[dst] = h.mhi[src];
          pt.b[dst] = h.mb[src];
          pt.cb[dst] = h.mcb[src];
        }
      }
    }
  }
  return pt;
}

}  // namespace qts
