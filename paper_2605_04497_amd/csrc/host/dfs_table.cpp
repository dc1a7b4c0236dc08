// Tables of the depth-first form of the pairwise interactions (section 5,
// Algorithm 1 at order 2): per tree, the internal nodes in preorder with what
// the tree walk needs at each (the split feature's interval and cover product
// above the node and on each child edge), and one pair-pass row per internal
// node holding the features split above it.  The model has been validated by
// build_host_table.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

#include "../qts_internal.h"

namespace qts {

namespace {

struct Edge {
  int32_t f;
  bool left;
  float thr;
  bool dleft;
  double w;
};

// The splits on one feature along a path, collapsed: cover product, the
// interval that follows them all ([lo, hi), hi = NaN: no upper bound) and
// whether a NaN follows them all.
struct Collapsed {
  double b = 1.0;
  float lo = -std::numeric_limits<float>::infinity();
  float hi = std::numeric_limits<float>::quiet_NaN();
  bool mok = true;
  bool seen = false;
};

void add_edge(Collapsed& c, bool left, float thr, bool dleft, double w) {
  c.seen = true;
  c.b *= w;
  if (left) {
    c.hi = std::isnan(c.hi) ? thr : std::min(c.hi, thr);
    c.mok = c.mok && dleft;
  } else {
    c.lo = std::max(c.lo, thr);
    c.mok = c.mok && !dleft;
  }
}

struct Row {
  int32_t group, node, f;
  std::vector<int32_t> feat;
  std::vector<float> lo, hi;
  std::vector<double> b;
};

class Walker {
 public:
  Walker(const qts_tree_arrays& t, DfsTable& out, std::vector<Row>& rows)
      : t_(t), out_(out), rows_(rows) {}

  void tree(int32_t ti, int32_t group, int32_t first_leaf) {
    base_ = t_.tree_offsets[ti];
    const int32_t n = (int32_t)(t_.tree_offsets[ti + 1] - base_);
    leaf_ord_.assign((size_t)n, -1);
    int32_t k = first_leaf;
    for (int32_t i = 0; i < n; ++i)
      if (t_.left[base_ + i] < 0) leaf_ord_[(size_t)i] = k++;
    group_ = group;
    path_.clear();
    const int32_t first = (int32_t)out_.nodes.size();
    if (t_.left[base_] >= 0) visit(0, 0, -1, false);
    const int32_t count = (int32_t)out_.nodes.size() - first;
    if (count > 0) {
      out_.tree_first.push_back(first);
      out_.tree_nodes.push_back(count);
    }
  }

 private:
  Collapsed collapse(int32_t f) const {
    Collapsed c;
    for (const Edge& e : path_)
      if (e.f == f) add_edge(c, e.left, e.thr, e.dleft, e.w);
    return c;
  }

  // Returns the record index of internal node `node`.
  int32_t visit(int32_t node, int32_t level, int32_t parent, bool is_left) {
    const int64_t g = base_ + node;
    const int32_t f = t_.feature[g];
    const float thr = t_.threshold[g];
    const bool dl = t_.default_left ? t_.default_left[g] != 0 : false;
    const double cov = t_.cover[g];
    const int32_t l = t_.left[g], r = t_.right[g];
    const double wl = cov == 0.0 ? 0.0 : t_.cover[base_ + l] / cov;
    const double wr = cov == 0.0 ? 0.0 : t_.cover[base_ + r] / cov;
    const Collapsed cv = collapse(f);
    Collapsed cl = cv, cr = cv;
    add_edge(cl, true, thr, dl, wl);
    add_edge(cr, false, thr, dl, wr);

    const int32_t rec = (int32_t)out_.nodes.size();
    DfsNode d{};
    d.f = f;
    d.level = level;
    d.parent = parent;
    d.flags = (is_left ? kDfsLeftChild : 0) | (cv.seen ? 0 : kDfsFresh) |
              (cv.mok ? kDfsMokV : 0) | (cl.mok ? kDfsMokL : 0) | (cr.mok ? kDfsMokR : 0);
    d.left = d.right = -1;
    d.leaf_l = t_.left[base_ + l] < 0 ? leaf_ord_[(size_t)l] : -1;
    d.leaf_r = t_.left[base_ + r] < 0 ? leaf_ord_[(size_t)r] : -1;
    d.row = (int32_t)rows_.size();
    d.lo_v = cv.lo;
    d.hi_v = cv.hi;
    d.lo_l = cl.lo;
    d.hi_l = cl.hi;
    d.lo_r = cr.lo;
    d.hi_r = cr.hi;
    out_.nodes.push_back(d);
    const double coef[kDfsCoef] = {cv.b, 1.0 - cv.b, cl.b, 1.0 - cl.b,
                                   cr.b, 1.0 - cr.b, cv.b - cl.b, cv.b - cr.b};
    out_.coef.insert(out_.coef.end(), coef, coef + kDfsCoef);
    out_.max_level = std::max(out_.max_level, level);

    // the pair-pass row: every feature split above the node except f, in
    // ascending feature order
    Row row;
    row.group = group_;
    row.node = rec;
    row.f = f;
    std::vector<int32_t> seen;
    for (const Edge& e : path_)
      if (e.f != f && std::find(seen.begin(), seen.end(), e.f) == seen.end()) seen.push_back(e.f);
    std::sort(seen.begin(), seen.end());
    for (const int32_t g : seen) {
      const Collapsed c = collapse(g);
      row.feat.push_back(g | (c.mok ? kMissingOkBit : 0));
      row.lo.push_back(c.lo);
      row.hi.push_back(c.hi);
      row.b.push_back(c.b);
    }
    rows_.push_back(std::move(row));

    out_.events.push_back(rec << 2 | kDfsEnter);
    if (t_.left[base_ + l] >= 0) {
      path_.push_back(Edge{f, true, thr, dl, wl});
      const int32_t cl_rec = visit(l, level + 1, rec, true);
      path_.pop_back();
      out_.nodes[(size_t)rec].left = cl_rec;
    }
    out_.events.push_back(rec << 2 | kDfsMiddle);
    if (t_.left[base_ + r] >= 0) {
      path_.push_back(Edge{f, false, thr, dl, wr});
      const int32_t cr_rec = visit(r, level + 1, rec, false);
      path_.pop_back();
      out_.nodes[(size_t)rec].right = cr_rec;
    }
    out_.events.push_back(rec << 2 | kDfsExit);
    return rec;
  }

  const qts_tree_arrays& t_;
  DfsTable& out_;
  std::vector<Row>& rows_;
  int64_t base_ = 0;
  int32_t group_ = 0;
  std::vector<int32_t> leaf_ord_;
  std::vector<Edge> path_;
};

}  // namespace

DfsTable build_dfs_table(const qts_tree_arrays& t, const HostTable& h) {
  DfsTable out;
  std::vector<Row> rows;
  Walker w(t, out, rows);
  int32_t first_leaf = 0;
  for (int32_t ti = 0; ti < t.n_trees; ++ti) {
    w.tree(ti, h.tree_group.empty() ? 0 : h.tree_group[(size_t)ti], first_leaf);
    for (int64_t i = t.tree_offsets[ti]; i < t.tree_offsets[ti + 1]; ++i)
      if (t.left[i] < 0) ++first_leaf;
  }
  // trees with the most nodes first (the walk's longest work items start early)
  std::vector<size_t> ord(out.tree_first.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](size_t a, size_t b) { return out.tree_nodes[a] > out.tree_nodes[b]; });
  std::vector<int32_t> tf, tn;
  for (size_t i : ord) {
    tf.push_back(out.tree_first[i]);
    tn.push_back(out.tree_nodes[i]);
  }
  out.tree_first.swap(tf);
  out.tree_nodes.swap(tn);

  // pair-pass rows: by group, then by length; each group padded to whole tiles
  std::vector<size_t> ro(rows.size());
  std::iota(ro.begin(), ro.end(), 0);
  // inside a group: by length, then by the row's rank among its tree's rows of
  // that length, then by tree, so that neighbouring lanes come from different
  // trees (rows of one tree share most features: their pair updates would
  // meet in the same triangle entries)
  std::vector<int32_t> rank(rows.size(), 0), tree_of(rows.size(), 0);
  {
    int32_t tr = -1;
    std::vector<int32_t> count(kMaxUnique + 2, 0);
    for (size_t i = 0; i < rows.size(); ++i) {
      if (out.nodes[(size_t)rows[i].node].parent < 0) {  // a new tree starts
        ++tr;
        std::fill(count.begin(), count.end(), 0);
      }
      tree_of[i] = tr;
      rank[i] = count[std::min<size_t>(rows[i].feat.size(), kMaxUnique + 1)]++;
    }
  }
  std::stable_sort(ro.begin(), ro.end(), [&](size_t a, size_t b) {
    if (rows[a].group != rows[b].group) return rows[a].group < rows[b].group;
    if (rows[a].feat.size() != rows[b].feat.size())
      return rows[a].feat.size() < rows[b].feat.size();
    if (rank[a] != rank[b]) return rank[a] < rank[b];
    return tree_of[a] < tree_of[b];
  });
  const int32_t K = h.n_groups;
  out.group_tile.assign((size_t)K + 1, 0);
  std::vector<int32_t> order;  // row position -> rows index, -1 for padding
  size_t i = 0;
  for (int32_t g = 0; g < K; ++g) {
    out.group_tile[(size_t)g] = (int32_t)(order.size() / 64);
    while (i < ro.size() && rows[ro[i]].group == g) order.push_back((int32_t)ro[i++]);
    while (order.size() % 64) order.push_back(-1);
  }
  out.group_tile[(size_t)K] = (int32_t)(order.size() / 64);
  if (order.size() > (size_t)std::numeric_limits<int32_t>::max() / 16)
    fail(QTS_E_UNSUPPORTED, "too many internal nodes for the depth-first form");
  out.n_rows = (int32_t)order.size();
  out.row_f.assign(order.size(), -1);
  out.row_d.assign(order.size(), 0);
  const size_t n_tiles = order.size() / 64;
  int64_t el = 0;
  for (size_t tt = 0; tt < n_tiles; ++tt) {
    int32_t dmax = 0;
    for (size_t q = 0; q < 64; ++q) {
      const int32_t ri = order[tt * 64 + q];
      if (ri >= 0) dmax = std::max(dmax, (int32_t)rows[(size_t)ri].feat.size());
    }
    out.tile_base.push_back((int32_t)el);
    out.tile_d.push_back(dmax);
    el += (int64_t)dmax * 64;
    if (el > std::numeric_limits<int32_t>::max())
      fail(QTS_E_UNSUPPORTED, "depth-first pair table too large");
  }
  out.feat.assign((size_t)el, kMissingOkBit);
  out.lo.assign((size_t)el, -std::numeric_limits<float>::infinity());
  out.hi.assign((size_t)el, std::numeric_limits<float>::quiet_NaN());
  out.b.assign((size_t)el, 1.0);
  out.cb.assign((size_t)el, 0.0);
  for (size_t pos = 0; pos < order.size(); ++pos) {
    const int32_t ri = order[pos];
    if (ri < 0) continue;
    const Row& r = rows[(size_t)ri];
    out.row_f[pos] = r.f;
    const int64_t rd = (int64_t)r.feat.size();
    out.row_d[pos] = (int32_t)rd;
    out.n_updates += rd;
    out.n_updates3 += rd * (rd - 1) / 2;
    out.max_row_d = std::max(out.max_row_d, (int32_t)rd);
    out.nodes[(size_t)r.node].row = (int32_t)pos;
    const size_t tt = pos / 64, lane = pos % 64;
    for (size_t k = 0; k < r.feat.size(); ++k) {
      const size_t e = (size_t)out.tile_base[tt] + 64 * k + lane;
      out.feat[e] = r.feat[k];
      out.lo[e] = r.lo[k];
      out.hi[e] = r.hi[k];
      out.b[e] = r.b[k];
      out.cb[e] = 1.0 - r.b[k];
    }
  }
  return out;
}

}  // namespace qts
