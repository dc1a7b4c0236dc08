// C-ABI entry points (declared in include/qtreeshap.h).
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "qts_device.h"
#include "qts_internal.h"
#include "qtreeshap.h"

namespace qts {

constexpr int kSideStreams = 3;  // extra branches of a captured graph
constexpr size_t kMaxGraphs = 16;

// One captured call: its launches depend only on these arguments.
struct GraphKey {
  int kind = 0;  // 0 values, 1 interactions, 2 adjoint, 3 third order
  int fp64 = 0;
  const void* X = nullptr;
  int64_t M = 0, ldx = 0;
  const void* in = nullptr;    // leaf-value override or grad_phi
  const void* out0 = nullptr;  // phi / Phi / grad_leaf
  const void* out1 = nullptr;  // phi of the interactions call
  hipStream_t stream = nullptr;
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && fp64 == o.fp64 && X == o.X && M == o.M && ldx == o.ldx &&
           in == o.in && out0 == o.out0 && out1 == o.out1 && stream == o.stream;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
  void* scratch = nullptr;  // the call's FP64 accumulators, owned by this graph
  hipEvent_t done = nullptr;  // recorded after each launch of the graph
  uint64_t stamp = 0;
};

// Per-ensemble cache of instantiated graphs (see qts_set_graph_replay).
struct GraphCache {
  std::mutex mu;
  bool on = false;
  hipStream_t cap = nullptr;  // capture stream
  hipStream_t side[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSideStreams] = {};
  std::vector<GraphEntry> entries;
  uint64_t clock = 0;
};

}  // namespace qts

struct qts_ensemble {
  qts::HostTable host;
  std::vector<qts::PairClass> pair_classes;
  qts::DeviceTable dev;
  bool on_device = false;
  // launch shapes per bucket capacity index (8, 16, 32, 64) and precision,
  // and per pair capacity class and precision (defaults until autotuned)
  // [node policy][precision][length bucket]; the adjoint's tuned separately
  qts::ValuesShape vshape[2][2][4];
  qts::ValuesShape ashape[2][2][4];
  std::vector<qts::PairShape> pshape[2][2];  // [node policy][precision]
  bool merge_siblings = true;  // first-order calls walk the merged table
  bool deterministic = false;  // first-order and adjoint results independent of scheduling
  int node_policy = QTS_NODES_FIXED8;
  int64_t pair_rows = 0, pair_elements = 0, pair_updates = 0;  // interactions table
  // depth-first form of the interactions (qts_set_pair_traversal): the tree
  // arrays are kept to build its tables on first use
  int pair_traversal = QTS_PAIRS_AUTO;
  bool dfs_faster[2] = {false, false};  // QTS_PAIRS_AUTO: qts_autotune's choice per precision
  bool dfs3_faster[2] = {false, false};  // the same for the third-order call
  struct Trees {
    std::vector<int64_t> off;
    std::vector<int32_t> left, right, feature;
    std::vector<float> threshold;
    std::vector<uint8_t> default_left;
    std::vector<double> cover, value;
  } trees;
  qts::DeviceDfs dfs;
  qts::GraphCache graphs;
};

namespace qts {

namespace {
thread_local std::string g_last_error;

int cap_index(int dmax) { return dmax <= 8 ? 0 : dmax <= 16 ? 1 : dmax <= 32 ? 2 : 3; }

// The bucket with the most rows of each capacity (launch shapes are kept per
// capacity; with output groups several buckets share one).
std::vector<Bucket> largest_per_capacity(const std::vector<Bucket>& bks) {
  std::vector<Bucket> out;
  for (const Bucket& bk : bks) {
    bool done = false;
    for (Bucket& o : out)
      if (o.dmax == bk.dmax) {
        if (bk.path_end - bk.path_begin > o.path_end - o.path_begin) o = bk;
        done = true;
      }
    if (!done) out.push_back(bk);
  }
  return out;
}

template <class Fn>
int guarded(Fn&& fn) {
  try {
    fn();
    return QTS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return QTS_E_OOM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return QTS_E_HIP;
  }
}

// Allocation-failure injection (qts_debug_fail_allocations): how many more
// device allocations may succeed, or -1 (no injection).
std::atomic<int64_t> g_alloc_budget{-1};

// Every device allocation of the library goes through here.
hipError_t device_alloc(void** p, size_t bytes, hipStream_t s, bool async) {
  int64_t b = g_alloc_budget.load();
  while (b >= 0) {
    if (b == 0) return hipErrorOutOfMemory;
    if (g_alloc_budget.compare_exchange_weak(b, b - 1)) break;
  }
  return async ? hipMallocAsync(p, bytes, s) : hipMalloc(p, bytes);
}

template <class T>
T* upload(const std::vector<T>& v, hipStream_t s) {
  if (v.empty()) return nullptr;
  T* p = nullptr;
  const hipError_t e = device_alloc(reinterpret_cast<void**>(&p), v.size() * sizeof(T), s, false);
  if (e != hipSuccess) {
    // earlier uploads may still read host vectors that the unwinding frees
    (void)hipStreamSynchronize(s);
    check_hip(e, "hipMalloc");
  }
  check_hip(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s),
            "hipMemcpyAsync");
  return p;
}

constexpr size_t kPad = 8;

template <class T>
std::vector<T> padded(const std::vector<T>& v, T fill) {
  std::vector<T> out(v);
  out.resize(v.size() + kPad, fill);
  return out;
}

template <class T>
std::vector<T> narrow(const std::vector<double>& v) {
  std::vector<T> out(v.size());
  for (size_t i = 0; i < v.size(); ++i) out[i] = (T)v[i];
  return out;
}

// Device layout of a first-order path table: every path is padded to whole
// batches of eight elements with inert slots (feature 0, no bounds,
// missing_ok, b = 1, 1-b = 0): their factor is exactly 1 and their
// contribution 0, so the kernels process whole batches without per-slot
// tests.  Eight more inert slots follow the last path.  Synchronous with
// respect to the host vectors (waits on the stream).
void upload_paths(const std::vector<PathHdr>& hdr_in, const std::vector<int32_t>& feat_in,
                  const std::vector<float>& lo_in, const std::vector<float>& hi_in,
                  const std::vector<double>& b_in, const std::vector<double>& cb_in,
                  const CompactTable& ct, hipStream_t s, PathHdr** o_hdr, int32_t** o_feat,
                  float** o_lo, float** o_hi, float** o_b32, float** o_cb32, double** o_b64,
                  double** o_cb64, int32_t** o_lfeat, Segment** o_segs, int32_t** o_seg_feat) {
  std::vector<PathHdr> hdr = hdr_in;
  const bool wide = !ct.segs.empty();
  std::vector<int32_t> feat, lfeat;
  std::vector<float> lo, hi;
  std::vector<double> b64, cb64;
  size_t n_pad = 0;
  for (const PathHdr& p : hdr_in) n_pad += (size_t)((p.d + 7) / 8) * 8;
  feat.reserve(n_pad + kPad);
  lo.reserve(n_pad + kPad);
  hi.reserve(n_pad + kPad);
  b64.reserve(n_pad + kPad);
  cb64.reserve(n_pad + kPad);
  for (size_t i = 0; i < hdr_in.size(); ++i) {
    const PathHdr& p = hdr_in[i];
    hdr[i].off = (int32_t)feat.size();
    const int padded_d = (p.d + 7) / 8 * 8;
    for (int k = 0; k < padded_d; ++k) {
      const bool real = k < p.d;
      const size_t e = (size_t)p.off + (size_t)k;
      feat.push_back(real ? feat_in[e] : kMissingOkBit);
      if (wide) lfeat.push_back(real ? ct.lfeat[e] : kMissingOkBit);
      lo.push_back(real ? lo_in[e] : -INFINITY);
      hi.push_back(real ? hi_in[e] : NAN);
      b64.push_back(real ? b_in[e] : 1.0);
      cb64.push_back(real ? cb_in[e] : 0.0);
    }
  }
  if (feat.size() > (size_t)0x7fffffff) fail(QTS_E_UNSUPPORTED, "path table too large");
  feat = padded(feat, (int32_t)kMissingOkBit);
  if (wide) lfeat = padded(lfeat, (int32_t)kMissingOkBit);
  lo = padded(lo, -INFINITY);
  hi = padded(hi, NAN);
  b64 = padded(b64, 1.0);
  cb64 = padded(cb64, 0.0);
  std::vector<float> b32 = narrow<float>(b64), cb32 = narrow<float>(cb64);
  *o_hdr = upload(hdr, s);
  *o_feat = upload(feat, s);
  *o_lo = upload(lo, s);
  *o_hi = upload(hi, s);
  *o_b32 = upload(b32, s);
  *o_cb32 = upload(cb32, s);
  *o_b64 = upload(b64, s);
  *o_cb64 = upload(cb64, s);
  if (wide) {
    *o_lfeat = upload(lfeat, s);
    *o_segs = upload(ct.segs, s);
    *o_seg_feat = upload(ct.seg_feat, s);
  }
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// The short-row records (ShortRow) of a table's capacity-8 buckets, in the
// order Bucket::srow_begin numbers them; the slots' features as the
// first-order kernel indexes its tile (the segment-local feature for wide
// feature spaces).
template <typename T>
std::vector<ShortRow<T>> short_rows(const std::vector<PathHdr>& hdr,
                                    const std::vector<int32_t>& feat, const CompactTable& ct,
                                    const std::vector<float>& lo, const std::vector<float>& hi,
                                    const std::vector<double>& b, const std::vector<double>& cb,
                                    const std::vector<int32_t>& share,
                                    const std::vector<Bucket>& bks) {
  const std::vector<int32_t>& tf = ct.segs.empty() ? feat : ct.lfeat;
  std::vector<ShortRow<T>> out;
  for (const Bucket& bk : bks) {
    if (bk.dmax != 8) continue;
    if ((size_t)bk.srow_begin != out.size()) fail(QTS_E_INVALID_ARG, "internal: short-row order");
    for (int32_t p = bk.path_begin; p < bk.path_end; ++p) {
      ShortRow<T> r{};
      r.d = hdr[(size_t)p].d;
      r.share = share[(size_t)p];
      for (int k = 0; k < 8; ++k) {
        if (k < r.d) {
          const size_t e = (size_t)hdr[(size_t)p].off + (size_t)k;
          const int32_t f = tf[e] & kFeatureMask;
          r.xoff[k] = f * kTileStride * (int32_t)sizeof(float);
          r.aoff[k] = f * kTileStride * (int32_t)sizeof(double);
          if (tf[e] & kMissingOkBit) r.mok |= 1 << k;
          r.lo[k] = lo[e];
          r.hi[k] = hi[e];
          r.b[k] = (T)b[e];
          r.cb[k] = (T)cb[e];
        } else {
          r.mok |= 1 << k;
          r.lo[k] = -INFINITY;
          r.hi[k] = NAN;
          r.b[k] = T(1);
          r.cb[k] = T(0);
        }
      }
      out.push_back(r);
    }
  }
  return out;
}

void keep_trees(const qts_tree_arrays& t, qts_ensemble::Trees& k) {
  const int64_t n = t.n_trees > 0 ? t.tree_offsets[t.n_trees] : 0;
  k.off.assign(t.tree_offsets, t.tree_offsets + (t.n_trees + 1));
  k.left.assign(t.left, t.left + n);
  k.right.assign(t.right, t.right + n);
  k.feature.assign(t.feature, t.feature + n);
  k.threshold.assign(t.threshold, t.threshold + n);
  if (t.default_left) k.default_left.assign(t.default_left, t.default_left + n);
  else k.default_left.assign((size_t)n, 0);
  k.cover.assign(t.cover, t.cover + n);
  k.value.assign(t.value, t.value + n);
}

void free_dfs(DeviceDfs& d) {
  void* ptrs[] = {d.nodes, d.coef32, d.coef64, d.events, d.tree_first, d.tree_nodes, d.row_f,
                  d.row_d, d.tile_base, d.tile_d, d.feat, d.lo, d.hi, d.b32, d.cb32, d.b64,
                  d.cb64};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  d = DeviceDfs{};
}

void build_dfs(qts_ensemble* e) {
  if (e->dfs.built) return;
  const qts_ensemble::Trees& k = e->trees;
  qts_tree_arrays ta{(int32_t)(k.off.size() - 1), k.off.data(), k.left.data(), k.right.data(),
                     k.feature.data(), k.threshold.data(), k.default_left.data(),
                     k.cover.data(), k.value.data()};
  const DfsTable t = build_dfs_table(ta, e->host);
  DeviceDfs& d = e->dfs;
  hipStream_t s = nullptr;
  try {
    d.nodes = upload(t.nodes, s);
    const std::vector<float> c32 = narrow<float>(t.coef);
    d.coef32 = upload(c32, s);
    d.coef64 = upload(t.coef, s);
    d.events = upload(t.events, s);
    d.tree_first = upload(t.tree_first, s);
    d.tree_nodes = upload(t.tree_nodes, s);
    d.n_trees = (int32_t)t.tree_first.size();
    d.max_level = t.max_level;
    d.n_rows = t.n_rows;
    d.row_f = upload(t.row_f, s);
    d.row_d = upload(t.row_d, s);
    d.tile_base = upload(t.tile_base, s);
    d.tile_d = upload(t.tile_d, s);
    d.feat = upload(t.feat, s);
    d.lo = upload(t.lo, s);
    d.hi = upload(t.hi, s);
    const std::vector<float> b32 = narrow<float>(t.b), cb32 = narrow<float>(t.cb);
    d.b32 = upload(b32, s);
    d.cb32 = upload(cb32, s);
    d.b64 = upload(t.b, s);
    d.cb64 = upload(t.cb, s);
    d.group_tile = t.group_tile;
    d.n_updates = t.n_updates;
    d.n_updates3 = t.n_updates3;
    d.max_row_d = t.max_row_d;
    d.n_nodes = (int64_t)t.nodes.size();
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    d.built = true;
  } catch (...) {
    (void)hipStreamSynchronize(s);
    free_dfs(d);
    throw;
  }
}

void free_device(DeviceTable& d) {
  void* ptrs[] = {d.hdr,    d.feat,    d.lo,      d.hi,      d.b32,     d.cb32,
                  d.b64,    d.cb64,    d.leaf_val, d.pr_d,   d.pr_leaf, d.pr_feat,
                  d.pr_lo,  d.pr_hi,   d.pr_b32,  d.pr_cb32, d.pr_b64,  d.pr_cb64,
                  d.mhdr,   d.mfeat,   d.mlo,     d.mhi,     d.mb32,    d.mcb32,
                  d.mb64,   d.mcb64,   d.side,    d.pr_side, d.share,   d.mshare,
                  d.lfeat,  d.segs,    d.seg_feat, d.mlfeat, d.msegs,  d.mseg_feat,
                  d.srow32, d.srow64,  d.msrow32, d.msrow64};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  d = DeviceTable{};
}

void build_nodes(DeviceTable& d) {
  double t[kNodes], s[kNodes], w[kNodes];
  gauss_legendre(kNodes, t, s, w);
  for (int m = 0; m < kNodes; ++m) {
    d.n32.t[m] = (float)t[m];
    d.n32.w[m] = (float)w[m];
    d.n64.t[m] = t[m];
    d.n64.w[m] = w[m];
    // the FP32 short-row walks take the rule as instruction literals
    if (d.n32.t[m] != rule8_t32(m) || d.n32.w[m] != rule8_w32(m))
      fail(QTS_E_UNSUPPORTED, "the FP32 8-node rule differs from the kernels' constants");
  }
  // fewer-node rules, padded with zero nodes and weights
  auto rule = [&](int n, NodeConsts<float>& f32, NodeConsts<double>& f64) {
    gauss_legendre(n, t, s, w);
    for (int m = 0; m < kNodes; ++m) {
      f32.t[m] = m < n ? (float)t[m] : 0.f;
      f32.w[m] = m < n ? (float)w[m] : 0.f;
      f64.t[m] = m < n ? t[m] : 0.0;
      f64.w[m] = m < n ? w[m] : 0.0;
    }
  };
  rule(4, d.n32_4, d.n64_4);
  rule(2, d.n32_2, d.n64_2);
  rule(6, d.n32_6, d.n64_6);
}

void require_device(const qts_ensemble* ens) {
  if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
  if (!ens->on_device) fail(QTS_E_INVALID_ARG, "ensemble was built host-only");
  int cur = -1;
  check_hip(hipGetDevice(&cur), "hipGetDevice");
  if (cur != ens->dev.device)
    fail(QTS_E_INVALID_ARG, "current HIP device differs from the ensemble's device");
}

void check_rows(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx) {
  if (M < 0) fail(QTS_E_INVALID_ARG, "M must be >= 0");
  if (ldx < ens->host.F) fail(QTS_E_INVALID_ARG, "ldx must be >= n_features");
  if (M > 0 && !X) fail(QTS_E_INVALID_ARG, "null X");
  if (M > (int64_t)1 << 40) fail(QTS_E_UNSUPPORTED, "M too large");
}

// Stream-ordered scratch; freed on the same stream when the call's work ends.
struct Scratch {
  void* p = nullptr;
  hipStream_t s = nullptr;
  Scratch(size_t bytes, hipStream_t st) : s(st) {
    if (bytes) check_hip(device_alloc(&p, bytes, s, true), "hipMallocAsync");
  }
  ~Scratch() {
    if (p) (void)hipFreeAsync(p, s);
  }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
};

// Optional event timing of the main kernels (see qts_set_kernel_timing).
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];
};
Timing& timing() {
  static Timing t;
  return t;
}

// Records an event pair around a scope when timing is enabled.
class TimedScope {
 public:
  TimedScope(int kind, hipStream_t s, bool enable = true) : kind_(kind), s_(s) {
    if (!enable) return;
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    if (!t.on) return;
    check_hip(hipEventCreate(&a_), "hipEventCreate");
    check_hip(hipEventCreate(&b_), "hipEventCreate");
    check_hip(hipEventRecord(a_, s_), "hipEventRecord");
    active_ = true;
  }
  void done() {
    if (!active_) return;
    check_hip(hipEventRecord(b_, s_), "hipEventRecord");
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.ev[kind_].emplace_back(a_, b_);
    active_ = false;
  }
  ~TimedScope() {
    if (active_) {
      (void)hipEventDestroy(a_);
      (void)hipEventDestroy(b_);
    }
  }

 private:
  int kind_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  bool active_ = false;
};

// Persistent autotune cache (qts_set_tune_cache): one line per tuned launch,
//   <key> -> a b
// where the key names everything the timing depended on: the build's kernel
// sources, the device (architecture and compute units), the kernel kind,
// precision and node policy, the features and outputs, the bucket or class
// (capacity, group, rows) and the size class of the tuning row count.
#ifndef QTS_KERNELS_SHA
#define QTS_KERNELS_SHA "unversioned"
#endif
struct TuneCache {
  std::mutex mu;
  std::string path;
  bool loaded = false;
  std::vector<std::pair<std::string, std::pair<int, int>>> entries;
  int64_t hits = 0, misses = 0;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

// Under the cache's lock.
void tune_cache_load(TuneCache& c) {
  if (c.loaded) return;
  c.loaded = true;
  c.entries.clear();
  FILE* f = std::fopen(c.path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    std::string ln(line);
    const size_t arrow = ln.find(" -> ");
    if (arrow == std::string::npos) continue;
    int a = 0, b = 0;
    if (std::sscanf(ln.c_str() + arrow + 4, "%d %d", &a, &b) != 2) continue;
    c.entries.emplace_back(ln.substr(0, arrow), std::make_pair(a, b));
  }
  std::fclose(f);
}

bool tune_cache_get(const std::string& key, int* a, int* b) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> g(c.mu);
  if (c.path.empty()) return false;
  tune_cache_load(c);
  for (auto it = c.entries.rbegin(); it != c.entries.rend(); ++it)
    if (it->first == key) {
      *a = it->second.first;
      *b = it->second.second;
      ++c.hits;
      return true;
    }
  ++c.misses;
  return false;
}

void tune_cache_put(const std::string& key, int a, int b) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> g(c.mu);
  if (c.path.empty()) return;
  c.entries.emplace_back(key, std::make_pair(a, b));
  FILE* f = std::fopen(c.path.c_str(), "a");
  if (!f) return;  // a read-only cache still serves hits
  std::fprintf(f, "%s -> %d %d\n", key.c_str(), a, b);
  std::fclose(f);
}

std::string tune_key(const std::string& device, const char* kind, bool fp64, int policy,
                     const HostTable& h, int cap, int group, int64_t rows, int64_t m_class) {
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "v1 kernels=%s device=%s kind=%s prec=%s policy=%d F=%d groups=%d cap=%d "
                "group=%d rows=%lld mclass=%lld",
                QTS_KERNELS_SHA, device.c_str(), kind, fp64 ? "fp64" : "fp32", policy, h.F,
                h.n_groups, cap, group, (long long)rows, (long long)m_class);
  return buf;
}

// The streams one call's launches go to: the call's own stream, plus, while
// a graph is captured, side streams forked from it so that the per-bucket
// (per-class) launches become parallel branches of the graph.  Buckets add
// into the same FP64 accumulators with atomics, so their order is free.
struct Lanes {
  hipStream_t main = nullptr;
  GraphCache* g = nullptr;  // non-null while capturing
  int n_side = 0;
  void fork(int n_launches) {
    n_side = g ? std::min(kSideStreams, n_launches - 1) : 0;
    if (n_side <= 0) return;
    check_hip(hipEventRecord(g->fork, main), "hipEventRecord");
    for (int k = 0; k < n_side; ++k)
      check_hip(hipStreamWaitEvent(g->side[k], g->fork, 0), "hipStreamWaitEvent");
  }
  hipStream_t pick(int i) const {
    const int k = n_side > 0 ? i % (n_side + 1) : 0;
    return k == 0 ? main : g->side[k - 1];
  }
  void join() {
    for (int k = 0; k < n_side; ++k) {
      check_hip(hipEventRecord(g->join[k], g->side[k]), "hipEventRecord");
      check_hip(hipStreamWaitEvent(main, g->join[k], 0), "hipStreamWaitEvent");
    }
    n_side = 0;
  }
};

int nodes_of(const qts_ensemble* ens) { return ens->node_policy == QTS_NODES_EXACT ? 4 : 8; }
int pol_index(const qts_ensemble* ens) { return ens->node_policy == QTS_NODES_EXACT ? 1 : 0; }

const PairShape& pair_shape(const qts_ensemble* ens, bool fp64, size_t i) {
  static const PairShape kDefault{};
  const auto& v = ens->pshape[ens->node_policy == QTS_NODES_EXACT ? 1 : 0][fp64 ? 1 : 0];
  return i < v.size() ? v[i] : kDefault;
}

// The launches of one call, on `ln` (acc: the FP64 accumulators of the call).
// Rows of the first-order table in use and the call's scratch: the Slot0
// records first, then (FP32) the FP64 accumulator at a 256-byte boundary.
int32_t value_rows(const qts_ensemble* ens) {
  return (int32_t)(ens->merge_siblings ? ens->host.mhdr.size() : ens->host.hdr.size());
}
size_t slot0_region(const qts_ensemble* ens, bool fp64) {
  return (slot0_bytes(value_rows(ens), fp64) + 255) & ~(size_t)255;
}
// A call whose rows form one bucket walked as one chunk writes phi from its
// workgroups directly (no FP64 accumulator, zero fill or cast).
bool direct_call(const qts_ensemble* ens, int64_t M, bool fp64) {
  const HostTable& h = ens->host;
  const std::vector<Bucket>& bks = ens->merge_siblings ? h.mbuckets : h.buckets;
  // segmented (wide feature space) tables split every sample block; with
  // several outputs each group has buckets of its own
  if (bks.size() != 1 || wide_features(h.F) || h.n_groups != 1) return false;
  return values_direct(bks, M,
                       ens->vshape[pol_index(ens)][fp64 ? 1 : 0][cap_index(bks[0].dmax)]);
}
// Output elements per sample: K groups of F features.
int64_t out_row(const qts_ensemble* ens) { return (int64_t)ens->host.n_groups * ens->host.F; }

// Wide feature spaces (wide_features): the first-order and adjoint kernels
// take X feature-major, [F][M], in the call's scratch.
size_t xt_region(const qts_ensemble* ens, int64_t M) {
  return (sizeof(float) * (size_t)(M * ens->host.F) + 255) & ~(size_t)255;
}

// Layout: Slot0 records | (wide: X feature-major | FP64 accumulator [K][F][M])
// | (otherwise, FP32 output: FP64 accumulator [M][K][F]).
size_t values_scratch_bytes(const qts_ensemble* ens, int64_t M, bool fp64) {
  if (wide_features(ens->host.F))
    return slot0_region(ens, fp64) + xt_region(ens, M) +
           sizeof(double) * (size_t)(M * out_row(ens));
  const bool acc = !fp64 && (ens->deterministic || !direct_call(ens, M, fp64));
  return slot0_region(ens, fp64) + (acc ? sizeof(double) * (size_t)(M * out_row(ens)) : 0);
}

void issue_values(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                  const double* leaf, void* phi, bool fp64, void* scratch, Lanes& ln,
                  bool timed) {
  const HostTable& h = ens->host;
  const int64_t n = M * out_row(ens);
  void* slot0 = scratch;
  const PathArrays arr = ens->merge_siblings ? merged_arrays(ens->dev, ens->host)
                                             : plain_arrays(ens->dev, ens->host);
  const std::vector<Bucket>& bks = ens->merge_siblings ? h.mbuckets : h.buckets;
  launch_slot0(arr, value_rows(ens), leaf, fp64, slot0, ln.main);
  // wide feature spaces: X transposed into the scratch, the accumulator
  // [K][F][M], transposed into phi at the end
  const bool fmajor = wide_features(h.F);
  const int64_t F = h.F, K = h.n_groups;
  const float* Xk = X;
  int64_t ldk = ldx;
  double* a;
  if (fmajor) {
    float* xt = (float*)((char*)scratch + slot0_region(ens, fp64));
    a = (double*)((char*)xt + xt_region(ens, M));
    launch_transpose(X, M, F, ldx, 0, xt, M, 0, 1, ln.main);
    Xk = xt;
    ldk = M;
  } else {
    a = fp64 ? (double*)phi : (double*)((char*)scratch + slot0_region(ens, fp64));
  }
  auto finish = [&] {
    if (fmajor) {
      if (fp64) launch_transpose(a, F, M, M, F * M, (double*)phi, K * F, F, (int32_t)K, ln.main);
      else launch_transpose(a, F, M, M, F * M, (float*)phi, K * F, F, (int32_t)K, ln.main);
    } else if (!fp64) {
      launch_cast_f64_f32(a, (float*)phi, n, ln.main);
    }
  };
  if (ens->deterministic) {
    // one stream, buckets and chunks in order, adds without atomics
    launch_fill_zero(a, n, ln.main);
    TimedScope ts(0, timed ? ln.main : nullptr, timed);
    for (const Bucket& bk : bks)
      launch_values(h, ens->dev, arr, bk, fp64, Xk, M, ldk, slot0, a, nullptr,
                    ens->vshape[pol_index(ens)][fp64 ? 1 : 0][cap_index(bk.dmax)],
                    nodes_of(ens), ln.main, true);
    ts.done();
    finish();
    return;
  }
  if (direct_call(ens, M, fp64)) {
    TimedScope ts(0, timed ? ln.main : nullptr, timed);
    launch_values(h, ens->dev, arr, bks[0], fp64, X, M, ldx, slot0, nullptr, phi,
                  ens->vshape[pol_index(ens)][fp64 ? 1 : 0][cap_index(bks[0].dmax)],
                  nodes_of(ens), ln.main);
    ts.done();
    return;
  }
  launch_fill_zero(a, n, ln.main);
  TimedScope ts(0, timed ? ln.main : nullptr, timed);
  ln.fork((int)bks.size());
  for (size_t i = 0; i < bks.size(); ++i) {
    const Bucket& bk = bks[i];
    launch_values(h, ens->dev, arr, bk, fp64, Xk, M, ldk, slot0, a, nullptr,
                  ens->vshape[pol_index(ens)][fp64 ? 1 : 0][cap_index(bk.dmax)], nodes_of(ens),
                  ln.pick((int)i));
  }
  ln.join();
  ts.done();
  finish();
}

// Whether an interactions call of this precision takes the depth-first form.
bool use_dfs(const qts_ensemble* ens, bool fp64) {
  return ens->pair_traversal == QTS_PAIRS_DFS ||
         (ens->pair_traversal == QTS_PAIRS_AUTO && ens->dfs_faster[fp64 ? 1 : 0]);
}

// Whether a third-order call takes the depth-first form (its pass keeps a
// row's ratios in registers: rows of at most kDfsTriplesMaxRow features).
bool use_dfs3(const qts_ensemble* ens, bool fp64) {
  if (!ens->dfs.built || !dfs_triples_supported(ens->dfs)) return false;
  return ens->pair_traversal == QTS_PAIRS_DFS ||
         (ens->pair_traversal == QTS_PAIRS_AUTO && ens->dfs3_faster[fp64 ? 1 : 0]);
}

// The depth-first form takes the samples in batches whose y_v values (8 per
// sample and internal node) fit this much scratch.
constexpr size_t kDfsScratchBytes = (size_t)4 << 30;

int32_t dfs_batch(const qts_ensemble* ens, int64_t M, bool fp64) {
  const size_t per = (size_t)ens->dfs.n_rows * kNodes * (fp64 ? sizeof(double) : sizeof(float));
  int64_t mb = per == 0 ? M : (int64_t)(kDfsScratchBytes / per);
  mb = std::max<int64_t>(8, mb / 8 * 8);
  return (int32_t)std::min<int64_t>(mb, std::max<int64_t>(M, 1));
}

// Bytes of an interactions call's scratch: the FP64 accumulators, and for the
// depth-first form the y_v values of one batch after them.
size_t pairs_acc_bytes(const qts_ensemble* ens, int64_t M) {
  const int64_t F = ens->host.F;
  const int64_t MK = M * ens->host.n_groups;
  return sizeof(double) * (size_t)(MK * (F * (F - 1) / 2) + MK * F);
}
// Layout: accumulators | y values of one batch | the walk's leaf values.
size_t dfs_y_bytes(const qts_ensemble* ens, int64_t M, bool fp64) {
  return ((size_t)dfs_batch(ens, M, fp64) * (size_t)ens->dfs.n_rows * kNodes *
              (fp64 ? sizeof(double) : sizeof(float)) + 255) & ~(size_t)255;
}
size_t interactions_scratch_bytes(const qts_ensemble* ens, int64_t M, bool fp64) {
  size_t b = (pairs_acc_bytes(ens, M) + 255) & ~(size_t)255;
  if (use_dfs(ens, fp64))
    b += dfs_y_bytes(ens, M, fp64) +
         2 * (size_t)ens->dfs.n_nodes * (fp64 ? sizeof(double) : sizeof(float));
  return b;
}

void issue_interactions(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                        const double* leaf, void* phi, void* Phi, bool fp64, double* acc,
                        Lanes& ln, bool timed) {
  const HostTable& h = ens->host;
  const int64_t F = h.F;
  const int64_t ntri = F * (F - 1) / 2;
  const int64_t MK = M * h.n_groups;  // output rows: (sample, group)
  double* tri64 = acc;
  double* phi64 = tri64 + MK * ntri;
  launch_fill_zero(tri64, MK * ntri + MK * F, ln.main);
  if (use_dfs(ens, fp64)) {
    // Algorithm 1's order-2 form: per batch, the tree walk writes y_v, then
    // the pair pass adds its updates (the next walk reuses the y buffer)
    void* Y = (char*)acc + ((pairs_acc_bytes(ens, M) + 255) & ~(size_t)255);
    void* lvals = (char*)Y + dfs_y_bytes(ens, M, fp64);
    const int32_t mb = dfs_batch(ens, M, fp64);
    const int64_t tiles = (int64_t)ens->dfs.n_rows / 64;
    TimedScope ts(1, timed ? ln.main : nullptr, timed);
    for (int64_t s0 = 0; s0 < M; s0 += mb) {
      const int32_t n = (int32_t)std::min<int64_t>(mb, M - s0);
      // pair-pass chunks of 128 tiles (8192 rows): their elements, about 2 MB
      // on the interactions workload, stay in each XCD's L2 while the
      // batch's samples walk them (the next samples' workgroups follow)
      (void)tiles;
      const int32_t tpc = 128;
      launch_dfs_walk(h, ens->dfs, ens->dev, fp64, leaf, X, s0, n, ldx, Y, lvals, ln.main);
      launch_dfs_pairs(h, ens->dfs, ens->dev, fp64, X, s0, n, ldx, Y, tri64, phi64, tpc,
                       ln.main);
    }
    ts.done();
    launch_pairs_finalize(tri64, phi64, MK, (int)F, fp64, Phi, phi, ln.main);
    return;
  }
  TimedScope ts(1, timed ? ln.main : nullptr, timed);
  ln.fork((int)ens->pair_classes.size());
  for (size_t i = 0; i < ens->pair_classes.size(); ++i)
    launch_pairs(h, ens->dev, ens->pair_classes[i], fp64, X, M, ldx, leaf, tri64, phi64,
                 pair_shape(ens, fp64, i), ens->node_policy == QTS_NODES_EXACT,
                 ln.pick((int)i));
  ln.join();
  ts.done();
  launch_pairs_finalize(tri64, phi64, MK, (int)F, fp64, Phi, phi, ln.main);
}

// Scratch of a backward call: deterministic calls keep one row of leaf
// partial sums per 64-sample block.
// Layout: (wide: X feature-major | grad_phi feature-major [K][F][M]) |
// (deterministic: per-sample-block leaf partials).
size_t gt_region(const qts_ensemble* ens, int64_t M, bool fp64) {
  return ((fp64 ? sizeof(double) : sizeof(float)) * (size_t)(M * out_row(ens)) + 255) &
         ~(size_t)255;
}
size_t backward_scratch_bytes(const qts_ensemble* ens, int64_t M, bool fp64) {
  if (M == 0) return 0;
  size_t b = 0;
  if (wide_features(ens->host.F)) b += xt_region(ens, M) + gt_region(ens, M, fp64);
  if (ens->deterministic) {
    const int64_t nsb = (M + kSamplesPerBlock - 1) / kSamplesPerBlock;
    b += sizeof(double) * (size_t)(nsb * (int64_t)ens->host.leaf_value.size());
  }
  return b;
}

void issue_backward(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                    const void* grad_phi, double* grad_leaf, bool fp64, double* scratch_in,
                    Lanes& ln, bool timed) {
  const HostTable& h = ens->host;
  const int64_t L = (int64_t)h.leaf_value.size();
  char* sp = (char*)scratch_in;
  // wide feature spaces: X and grad_phi transposed into the scratch
  if (wide_features(h.F) && M > 0) {
    const int64_t F = h.F, K = h.n_groups;
    float* xt = (float*)sp;
    sp += xt_region(ens, M);
    launch_transpose(X, M, F, ldx, 0, xt, M, 0, 1, ln.main);
    if (fp64)
      launch_transpose((const double*)grad_phi, M, F, K * F, F, (double*)sp, M, F * M,
                       (int32_t)K, ln.main);
    else
      launch_transpose((const float*)grad_phi, M, F, K * F, F, (float*)sp, M, F * M,
                       (int32_t)K, ln.main);
    X = xt;
    ldx = M;
    grad_phi = sp;
    sp += gt_region(ens, M, fp64);
  }
  double* scratch = (double*)sp;
  if (ens->deterministic && M > 0) {
    const int64_t nsb = (M + kSamplesPerBlock - 1) / kSamplesPerBlock;
    launch_fill_zero(scratch, nsb * L, ln.main);
    const std::vector<Bucket>& bks = ens->merge_siblings ? h.mbuckets : h.buckets;
    const PathArrays arr = ens->merge_siblings ? merged_arrays(ens->dev, ens->host)
                                               : plain_arrays(ens->dev, ens->host);
    TimedScope ts(2, timed ? ln.main : nullptr, timed);
    for (const Bucket& bk : bks)
      launch_adjoint(h, ens->dev, arr, bk, fp64, X, grad_phi, M, ldx, scratch,
                     ens->ashape[pol_index(ens)][fp64 ? 1 : 0][cap_index(bk.dmax)],
                     nodes_of(ens), ln.main, L);
    ts.done();
    launch_sum_rows(scratch, nsb, L, grad_leaf, ln.main);
    return;
  }
  launch_fill_zero(grad_leaf, L, ln.main);
  if (M == 0) return;
  TimedScope ts(2, timed ? ln.main : nullptr, timed);
  const std::vector<Bucket>& bks = ens->merge_siblings ? h.mbuckets : h.buckets;
  const PathArrays arr = ens->merge_siblings ? merged_arrays(ens->dev, ens->host)
                                             : plain_arrays(ens->dev, ens->host);
  ln.fork((int)bks.size());
  for (size_t i = 0; i < bks.size(); ++i) {
    const Bucket& bk = bks[i];
    launch_adjoint(h, ens->dev, arr, bk, fp64, X, grad_phi, M, ldx, grad_leaf,
                   ens->ashape[pol_index(ens)][fp64 ? 1 : 0][cap_index(bk.dmax)], nodes_of(ens),
                   ln.pick((int)i));
  }
  ln.join();
  ts.done();
}

void destroy_entry(GraphEntry& e) {
  // the graph may still run: wait for its last launch (an event of the
  // library's own, so the caller's stream need not outlive the cache)
  if (e.done) {
    (void)hipEventSynchronize(e.done);
    (void)hipEventDestroy(e.done);
  }
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.scratch) (void)hipFree(e.scratch);
  e.exec = nullptr;
  e.scratch = nullptr;
  e.done = nullptr;
}

void clear_graphs(GraphCache& g) {
  for (GraphEntry& e : g.entries) destroy_entry(e);
  g.entries.clear();
}

void release_graph_cache(GraphCache& g) {
  clear_graphs(g);
  if (g.cap) (void)hipStreamDestroy(g.cap);
  for (hipStream_t& st : g.side)
    if (st) (void)hipStreamDestroy(st);
  if (g.fork) (void)hipEventDestroy(g.fork);
  for (hipEvent_t& ev : g.join)
    if (ev) (void)hipEventDestroy(ev);
  g.cap = nullptr;
  g.fork = nullptr;
  for (int k = 0; k < kSideStreams; ++k) {
    g.side[k] = nullptr;
    g.join[k] = nullptr;
  }
  g.on = false;
}

// Replay the graph of `key`, capturing it first (with `issue(lanes, scratch)`
// on the cache's capture stream) if it is not cached.  The graph is launched
// on the caller's stream, so it orders after the work already queued there.
template <class Issue>
void run_graph(qts_ensemble* ens, const GraphKey& key, size_t scratch_bytes, int kind,
               Issue&& issue) {
  GraphCache& g = ens->graphs;
  std::lock_guard<std::mutex> lock(g.mu);
  GraphEntry* hit = nullptr;
  for (GraphEntry& e : g.entries)
    if (e.key == key) hit = &e;
  if (!hit) {
    GraphEntry ne;
    ne.key = key;
    if (scratch_bytes) check_hip(device_alloc(&ne.scratch, scratch_bytes, nullptr, false), "hipMalloc");
    hipGraph_t graph = nullptr;
    try {
      check_hip(hipEventCreateWithFlags(&ne.done, hipEventDisableTiming), "hipEventCreate");
      check_hip(hipStreamBeginCapture(g.cap, hipStreamCaptureModeRelaxed),
                "hipStreamBeginCapture");
      try {
        Lanes ln{g.cap, &g};
        issue(ln, (double*)ne.scratch);
      } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(g.cap, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        throw;
      }
      check_hip(hipStreamEndCapture(g.cap, &graph), "hipStreamEndCapture");
      check_hip(hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0),
                "hipGraphInstantiate");
      (void)hipGraphDestroy(graph);
    } catch (...) {
      if (graph) (void)hipGraphDestroy(graph);
      if (ne.scratch) (void)hipFree(ne.scratch);
      if (ne.done) (void)hipEventDestroy(ne.done);
      throw;
    }
    if (g.entries.size() >= kMaxGraphs) {
      size_t victim = 0;
      for (size_t i = 1; i < g.entries.size(); ++i)
        if (g.entries[i].stamp < g.entries[victim].stamp) victim = i;
      destroy_entry(g.entries[victim]);
      g.entries.erase(g.entries.begin() + (std::ptrdiff_t)victim);
    }
    g.entries.push_back(ne);
    hit = &g.entries.back();
  }
  hit->stamp = ++g.clock;
  TimedScope ts(kind, key.stream, true);
  check_hip(hipGraphLaunch(hit->exec, key.stream), "hipGraphLaunch");
  check_hip(hipEventRecord(hit->done, key.stream), "hipEventRecord");
  ts.done();
}

}  // namespace

// Scratch of qts_shap_values_noalloc: a file-scope device array, so the call
// needs no allocation.  Every GPU the library runs on holds its own copy for
// the life of the process.  On the host the array's name is not a device
// address: the per-device address comes from hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;  // 64 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
void* noalloc_scratch() {
  int dev = -1;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) fail(QTS_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  fail(e == hipErrorOutOfMemory ? QTS_E_OOM : QTS_E_HIP,
       std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace qts

using namespace qts;

extern "C" {

int qts_build_host_grouped(const qts_tree_arrays* trees, const int32_t* tree_group,
                           int32_t n_groups, int32_t n_features, const double* base_scores,
                           qts_ensemble** out) {
  return guarded([&] {
    if (!trees || !out || !base_scores) fail(QTS_E_INVALID_ARG, "null argument");
    *out = nullptr;
    qts_ensemble* e = new qts_ensemble();
    try {
      e->host = build_host_table(*trees, n_features, n_groups, tree_group, base_scores);
    } catch (...) {
      delete e;
      throw;
    }
    *out = e;
  });
}

int qts_build_host(const qts_tree_arrays* trees, int32_t n_features, double base_score,
                   qts_ensemble** out) {
  return qts_build_host_grouped(trees, nullptr, 1, n_features, &base_score, out);
}

int qts_load_ensemble_grouped(const qts_tree_arrays* trees, const int32_t* tree_group,
                              int32_t n_groups, int32_t n_features, const double* base_scores,
                              void* stream, qts_ensemble** out) {
  return guarded([&] {
    if (!trees || !out || !base_scores) fail(QTS_E_INVALID_ARG, "null argument");
    *out = nullptr;
    qts_ensemble* e = new qts_ensemble();
    try {
      e->host = build_host_table(*trees, n_features, n_groups, tree_group, base_scores);
      keep_trees(*trees, e->trees);
      const HostTable& h = e->host;
      hipStream_t s = (hipStream_t)stream;
      DeviceTable& d = e->dev;
      check_hip(hipGetDevice(&d.device), "hipGetDevice");
      build_nodes(d);
      upload_paths(h.hdr, h.feat, h.lo, h.hi, h.b, h.cb, h.compact, s, &d.hdr, &d.feat, &d.lo,
                   &d.hi, &d.b32, &d.cb32, &d.b64, &d.cb64, &d.lfeat, &d.segs, &d.seg_feat);
      upload_paths(h.mhdr, h.mfeat, h.mlo, h.mhi, h.mb, h.mcb, h.mcompact, s, &d.mhdr, &d.mfeat,
                   &d.mlo, &d.mhi, &d.mb32, &d.mcb32, &d.mb64, &d.mcb64, &d.mlfeat, &d.msegs,
                   &d.mseg_feat);
      d.side = upload(h.side, s);
      d.share = upload(h.share, s);
      d.mshare = upload(h.mshare, s);
      {
        const auto r32 = short_rows<float>(h.hdr, h.feat, h.compact, h.lo, h.hi, h.b, h.cb,
                                           h.share, h.buckets);
        const auto r64 = short_rows<double>(h.hdr, h.feat, h.compact, h.lo, h.hi, h.b, h.cb,
                                            h.share, h.buckets);
        const auto m32 = short_rows<float>(h.mhdr, h.mfeat, h.mcompact, h.mlo, h.mhi, h.mb,
                                           h.mcb, h.mshare, h.mbuckets);
        const auto m64 = short_rows<double>(h.mhdr, h.mfeat, h.mcompact, h.mlo, h.mhi, h.mb,
                                            h.mcb, h.mshare, h.mbuckets);
        d.srow32 = upload(r32, s);
        d.srow64 = upload(r64, s);
        d.msrow32 = upload(m32, s);
        d.msrow64 = upload(m64, s);
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
      }
      d.leaf_val = upload(h.leaf_value, s);
      {
        PairTable pt = build_pair_table(h);
        e->pair_classes = pt.classes;
        e->pair_rows = (int64_t)pt.d.size();
        for (int32_t dr : pt.d) {
          e->pair_elements += dr;
          e->pair_updates += (int64_t)dr * (dr - 1) / 2;
        }
        d.pr_d = upload(pt.d, s);
        d.pr_leaf = upload(pt.leaf, s);
        d.pr_side = upload(pt.side, s);
        d.pr_feat = upload(pt.feat, s);
        d.pr_lo = upload(pt.lo, s);
        d.pr_hi = upload(pt.hi, s);
        const std::vector<float> pb32 = narrow<float>(pt.b), pcb32 = narrow<float>(pt.cb);
        d.pr_b32 = upload(pb32, s);
        d.pr_cb32 = upload(pcb32, s);
        d.pr_b64 = upload(pt.b, s);
        d.pr_cb64 = upload(pt.cb, s);
        // the uploads above are asynchronous: wait before the host vectors die
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
      }
      check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
      e->on_device = true;
    } catch (...) {
      free_device(e->dev);
      delete e;
      throw;
    }
    *out = e;
  });
}

int qts_load_ensemble(const qts_tree_arrays* trees, int32_t n_features, double base_score,
                      void* stream, qts_ensemble** out) {
  return qts_load_ensemble_grouped(trees, nullptr, 1, n_features, &base_score, stream, out);
}

int qts_free_ensemble(qts_ensemble* ens) {
  return guarded([&] {
    if (!ens) return;
    {
      std::lock_guard<std::mutex> lock(ens->graphs.mu);
      release_graph_cache(ens->graphs);
    }
    if (ens->on_device) {
      free_dfs(ens->dfs);
      free_device(ens->dev);
    }
    delete ens;
  });
}

int qts_expected_value(const qts_ensemble* ens, double* out) {
  return guarded([&] {
    if (!ens || !out) fail(QTS_E_INVALID_ARG, "null argument");
    *out = ens->host.expected;
  });
}

int qts_expected_values(const qts_ensemble* ens, double* out) {
  return guarded([&] {
    if (!ens || !out) fail(QTS_E_INVALID_ARG, "null argument");
    for (size_t g = 0; g < ens->host.expected_g.size(); ++g) out[g] = ens->host.expected_g[g];
  });
}

int qts_num_leaves(const qts_ensemble* ens, int64_t* out) {
  return guarded([&] {
    if (!ens || !out) fail(QTS_E_INVALID_ARG, "null argument");
    *out = (int64_t)ens->host.leaf_value.size();
  });
}

int qts_get_info(const qts_ensemble* ens, qts_info* out) {
  return guarded([&] {
    if (!ens || !out) fail(QTS_E_INVALID_ARG, "null argument");
    const HostTable& h = ens->host;
    out->n_features = h.F;
    out->n_trees = h.n_trees;
    out->n_leaves = (int64_t)h.leaf_value.size();
    out->n_paths = (int64_t)h.hdr.size();
    out->n_elements = (int64_t)h.feat.size();
    out->max_depth = h.max_depth;
    out->max_unique = h.max_unique;
    out->n_buckets = (int32_t)h.buckets.size();
    out->device = ens->on_device ? ens->dev.device : -1;
    out->n_pair_classes = (int32_t)ens->pair_classes.size();
    out->n_graphs = (int32_t)ens->graphs.entries.size();
    out->n_merged = (int64_t)h.side.size();
    out->n_value_paths = (int64_t)h.mhdr.size();
    out->n_value_elements = (int64_t)h.mfeat.size();
    out->n_pair_rows = ens->pair_rows;
    out->n_pair_elements = ens->pair_elements;
    out->n_pair_updates = ens->pair_updates;
    out->n_value_shared = 0;
    for (int32_t v : h.mshare) out->n_value_shared += v;
    out->n_path_shared = 0;
    for (int32_t v : h.share) out->n_path_shared += v;
    auto prefix_kept = [](const std::vector<Bucket>& bks, const std::vector<int32_t>& share) {
      int64_t n = 0;
      for (const Bucket& bk : bks)
        if (bk.dmax == 8)
          for (int32_t p = bk.path_begin; p < bk.path_end; ++p)
            n += std::min<int32_t>(share[(size_t)p], 6);
      return n;
    };
    out->n_value_prefix_kept = prefix_kept(h.mbuckets, h.mshare);
    out->n_path_prefix_kept = prefix_kept(h.buckets, h.share);
    out->n_value_segments = (int64_t)h.mcompact.segs.size();
    out->n_groups = h.n_groups;
    out->pairs_dfs = (use_dfs(ens, false) ? 1 : 0) | (use_dfs(ens, true) ? 2 : 0) |
                     (use_dfs3(ens, false) ? 4 : 0) | (use_dfs3(ens, true) ? 8 : 0);
    out->n_dfs_nodes = ens->dfs.n_nodes;
    out->n_dfs_updates = ens->dfs.n_updates;
    out->n_dfs_updates3 = ens->dfs.n_updates3;
  });
}

int qts_export_paths(const qts_ensemble* ens, int32_t* path_leaf, int32_t* path_len,
                     int32_t* path_off, int32_t* feat, float* lo, float* hi,
                     uint8_t* missing_ok, double* b, double* one_minus_b) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    const HostTable& h = ens->host;
    for (size_t i = 0; i < h.hdr.size(); ++i) {
      if (path_leaf) path_leaf[i] = h.hdr[i].leaf;
      if (path_len) path_len[i] = h.hdr[i].d;
      if (path_off) path_off[i] = h.hdr[i].off;
    }
    for (size_t i = 0; i < h.feat.size(); ++i) {
      if (feat) feat[i] = h.feat[i] & kFeatureMask;
      if (missing_ok) missing_ok[i] = (h.feat[i] & kMissingOkBit) ? 1 : 0;
      if (lo) lo[i] = h.lo[i];
      if (hi) hi[i] = h.hi[i];
      if (b) b[i] = h.b[i];
      if (one_minus_b) one_minus_b[i] = h.cb[i];
    }
  });
}

int qts_gauss_legendre(int32_t n, double* t, double* one_minus_t, double* weight) {
  return guarded([&] {
    if (!t || !one_minus_t || !weight) fail(QTS_E_INVALID_ARG, "null argument");
    gauss_legendre(n, t, one_minus_t, weight);
  });
}

int qts_shap_values(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                    const double* leaf_values, void* phi, qts_precision precision,
                    void* stream) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    check_rows(ens, X, M, ldx);
    if (M > 0 && !phi) fail(QTS_E_INVALID_ARG, "null phi");
    require_device(ens);
    if (M == 0) return;
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    const double* leaf = leaf_values ? leaf_values : ens->dev.leaf_val;
    const size_t scratch_bytes = values_scratch_bytes(ens, M, fp64);
    qts_ensemble* me = const_cast<qts_ensemble*>(ens);  // the graph cache only
    if (ens->graphs.on) {
      GraphKey key{0, fp64, X, M, ldx, leaf, phi, nullptr, s};
      run_graph(me, key, scratch_bytes, 0, [&](Lanes& ln, double* scratch) {
        issue_values(ens, X, M, ldx, leaf, phi, fp64, scratch, ln, false);
      });
      return;
    }
    Lanes ln{s, nullptr};
    Scratch scratch(scratch_bytes, s);
    issue_values(ens, X, M, ldx, leaf, phi, fp64, scratch.p, ln, true);
  });
}

int qts_shap_values_noalloc(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                            const double* leaf_values, void* phi, qts_precision precision,
                            void* stream) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    check_rows(ens, X, M, ldx);
    if (M > 0 && !phi) fail(QTS_E_INVALID_ARG, "null phi");
    require_device(ens);
    if (M == 0) return;
    const bool fp64 = precision == QTS_FP64;
    const size_t need = values_scratch_bytes(ens, M, fp64);
    if (need > kNoAllocScratchBytes)
      fail(QTS_E_UNSUPPORTED,
           "qts_shap_values_noalloc: this call needs " + std::to_string(need) +
               " bytes of scratch, more than its fixed " +
               std::to_string(kNoAllocScratchBytes) + "; use fewer samples per call");
    void* buf = noalloc_scratch();
    const double* leaf = leaf_values ? leaf_values : ens->dev.leaf_val;
    Lanes ln{(hipStream_t)stream, nullptr};
    issue_values(ens, X, M, ldx, leaf, phi, fp64, buf, ln, false);
  });
}

int qts_shap_interactions(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                          const double* leaf_values, void* phi, void* Phi,
                          qts_precision precision, void* stream) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    check_rows(ens, X, M, ldx);
    if (M > 0 && !Phi) fail(QTS_E_INVALID_ARG, "null Phi");
    require_device(ens);
    if (M == 0) return;
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    const double* leaf = leaf_values ? leaf_values : ens->dev.leaf_val;
    const size_t acc_bytes = interactions_scratch_bytes(ens, M, fp64);
    qts_ensemble* me = const_cast<qts_ensemble*>(ens);
    if (ens->graphs.on) {
      GraphKey key{1, fp64, X, M, ldx, leaf, Phi, phi, s};
      run_graph(me, key, acc_bytes, 1, [&](Lanes& ln, double* acc) {
        issue_interactions(ens, X, M, ldx, leaf, phi, Phi, fp64, acc, ln, false);
      });
      return;
    }
    Lanes ln{s, nullptr};
    Scratch acc(acc_bytes, s);
    issue_interactions(ens, X, M, ldx, leaf, phi, Phi, fp64, (double*)acc.p, ln, true);
  });
}

namespace {

// Scratch of one third-order call: the depth-first form's (FP32: the FP64
// accumulator) | y values of one sample batch | the walk's leaf values; the
// path form's FP64 accumulator (FP32 only).
size_t interactions3_scratch_bytes(const qts_ensemble* ens, int64_t M, bool fp64) {
  const int64_t F = ens->host.F;
  const int64_t T3 = F * (F - 1) * (F - 2) / 6;
  const int64_t MK = M * ens->host.n_groups;
  if (use_dfs3(ens, fp64)) {
    const size_t ab = fp64 ? 0 : ((sizeof(double) * (size_t)(MK * T3) + 255) & ~(size_t)255);
    const size_t yb = dfs_y_bytes(ens, M, fp64);
    const size_t lb = 2 * (size_t)std::max<int64_t>(1, ens->dfs.n_nodes) *
                      (fp64 ? sizeof(double) : sizeof(float));
    return ab + yb + lb;
  }
  return fp64 ? 0 : sizeof(double) * (size_t)(MK * T3);
}

// The launches of one third-order call on stream s, with `scratch` of
// interactions3_scratch_bytes (owned by the caller or by a graph).
void issue_interactions3(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                         const double* leaf, void* out, bool fp64, void* scratch,
                         hipStream_t s, bool timed) {
  const int64_t F = ens->host.F;
  const int64_t T3 = F * (F - 1) * (F - 2) / 6;
  const int64_t MK = M * ens->host.n_groups;
  TimedScope ts(3, timed ? s : nullptr, timed);
  if (use_dfs3(ens, fp64)) {
    // Algorithm 1 at order 3: per batch the tree walk writes y_v, then the
    // third-order pass adds its updates.
    const size_t ab = fp64 ? 0 : ((sizeof(double) * (size_t)(MK * T3) + 255) & ~(size_t)255);
    const size_t yb = dfs_y_bytes(ens, M, fp64);
    double* acc = fp64 ? static_cast<double*>(out) : (double*)scratch;
    void* Y = (char*)scratch + ab;
    void* lvals = (char*)Y + yb;
    launch_fill_zero(acc, MK * T3, s);
    const int32_t mb = dfs_batch(ens, M, fp64);
    for (int64_t s0 = 0; s0 < M; s0 += mb) {
      const int32_t n = (int32_t)std::min<int64_t>(mb, M - s0);
      launch_dfs_walk(ens->host, ens->dfs, ens->dev, fp64, leaf, X, s0, n, ldx, Y, lvals, s);
      launch_dfs_triples(ens->host, ens->dfs, ens->dev, fp64, X, s0, n, ldx, Y, acc, 128, s);
    }
    if (!fp64) launch_narrow_f64_f32(acc, MK * T3, static_cast<float*>(out), s);
    ts.done();
    return;
  }
  double* acc = fp64 ? static_cast<double*>(out) : (double*)scratch;
  launch_fill_zero(acc, MK * T3, s);
  for (const PairClass& pc : ens->pair_classes)
    launch_triples(ens->host, ens->dev, pc, fp64, X, M, ldx, leaf, acc, s);
  if (!fp64) launch_narrow_f64_f32(acc, MK * T3, static_cast<float*>(out), s);
  ts.done();
}

}  // namespace

int qts_shap_interactions3(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                           const double* leaf_values, void* out, qts_precision precision,
                           void* stream) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    check_rows(ens, X, M, ldx);
    const int64_t F = ens->host.F;
    const int64_t T3 = F * (F - 1) * (F - 2) / 6;
    if (M > 0 && T3 > 0 && !out) fail(QTS_E_INVALID_ARG, "null out");
    require_device(ens);
    if (M == 0 || T3 == 0) return;
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    const double* leaf = leaf_values ? leaf_values : ens->dev.leaf_val;
    const size_t scratch_bytes = interactions3_scratch_bytes(ens, M, fp64);
    if (ens->graphs.on) {
      GraphKey key{3, fp64, X, M, ldx, leaf, out, nullptr, s};
      run_graph(const_cast<qts_ensemble*>(ens), key, scratch_bytes, 3,
                [&](Lanes& ln, double* scratch) {
                  issue_interactions3(ens, X, M, ldx, leaf, out, fp64, scratch, ln.main, false);
                });
      return;
    }
    Scratch sc(scratch_bytes, s);
    issue_interactions3(ens, X, M, ldx, leaf, out, fp64, sc.p, s, true);
  });
}

int qts_shap_backward(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                      const void* grad_phi, double* grad_leaf, qts_precision precision,
                      void* stream) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    check_rows(ens, X, M, ldx);
    if (!grad_leaf) fail(QTS_E_INVALID_ARG, "null grad_leaf");
    if (M > 0 && !grad_phi) fail(QTS_E_INVALID_ARG, "null grad_phi");
    require_device(ens);
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    qts_ensemble* me = const_cast<qts_ensemble*>(ens);
    const size_t scratch_bytes = backward_scratch_bytes(ens, M, fp64);
    if (ens->graphs.on && M > 0) {
      GraphKey key{2, fp64, X, M, ldx, grad_phi, grad_leaf, nullptr, s};
      run_graph(me, key, scratch_bytes, 2, [&](Lanes& ln, double* scratch) {
        issue_backward(ens, X, M, ldx, grad_phi, grad_leaf, fp64, scratch, ln, false);
      });
      return;
    }
    Lanes ln{s, nullptr};
    if (scratch_bytes == 0) {
      issue_backward(ens, X, M, ldx, grad_phi, grad_leaf, fp64, nullptr, ln, true);
      return;
    }
    Scratch scratch(scratch_bytes, s);
    issue_backward(ens, X, M, ldx, grad_phi, grad_leaf, fp64, (double*)scratch.p, ln, true);
  });
}

int qts_set_graph_replay(qts_ensemble* ens, int32_t enable) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    require_device(ens);
    GraphCache& g = ens->graphs;
    std::lock_guard<std::mutex> lock(g.mu);
    if (!enable) {
      clear_graphs(g);
      g.on = false;
      return;
    }
    if (!g.cap) {
      try {
        check_hip(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking), "hipStreamCreate");
        for (int k = 0; k < kSideStreams; ++k)
          check_hip(hipStreamCreateWithFlags(&g.side[k], hipStreamNonBlocking),
                    "hipStreamCreate");
        check_hip(hipEventCreateWithFlags(&g.fork, hipEventDisableTiming), "hipEventCreate");
        for (int k = 0; k < kSideStreams; ++k)
          check_hip(hipEventCreateWithFlags(&g.join[k], hipEventDisableTiming),
                    "hipEventCreate");
      } catch (...) {
        release_graph_cache(g);
        throw;
      }
    }
    g.on = true;
  });
}

int qts_set_sibling_merge(qts_ensemble* ens, int32_t enable) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    std::lock_guard<std::mutex> lock(ens->graphs.mu);
    if (ens->merge_siblings != (enable != 0)) clear_graphs(ens->graphs);
    ens->merge_siblings = enable != 0;
  });
}

int qts_set_pair_traversal(qts_ensemble* ens, int32_t traversal) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (traversal != QTS_PAIRS_PATHS && traversal != QTS_PAIRS_DFS &&
        traversal != QTS_PAIRS_AUTO)
      fail(QTS_E_INVALID_ARG, "unknown pair traversal");
    std::lock_guard<std::mutex> lock(ens->graphs.mu);
    if (traversal != QTS_PAIRS_PATHS) {
      require_device(ens);
      if (dfs_walk_lds_bytes(ens->host.F, ens->host.max_depth, true) > (size_t)kMaxLdsBytes)
        fail(QTS_E_UNSUPPORTED, "the depth-first walk's stacks do not fit in LDS");
      build_dfs(ens);
    }
    if (ens->pair_traversal != traversal) clear_graphs(ens->graphs);
    ens->pair_traversal = traversal;
  });
}

int qts_debug_fail_allocations(int64_t after) {
  return guarded([&] { g_alloc_budget.store(after < 0 ? -1 : after); });
}

int qts_set_deterministic(qts_ensemble* ens, int32_t enable) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    std::lock_guard<std::mutex> lock(ens->graphs.mu);
    if (ens->deterministic != (enable != 0)) clear_graphs(ens->graphs);
    ens->deterministic = enable != 0;
  });
}

int qts_set_node_policy(qts_ensemble* ens, int32_t policy) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (policy != QTS_NODES_FIXED8 && policy != QTS_NODES_EXACT)
      fail(QTS_E_INVALID_ARG, "unknown node policy");
    std::lock_guard<std::mutex> lock(ens->graphs.mu);
    if (ens->node_policy != policy) clear_graphs(ens->graphs);
    ens->node_policy = policy;
  });
}

int qts_autotune(qts_ensemble* ens, int64_t M_hint, qts_precision precision, void* stream) {
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    require_device(ens);
    const HostTable& h = ens->host;
    const DeviceTable& d = ens->dev;
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    const int pi = fp64 ? 1 : 0;
    const int64_t F = h.F;
    // synthetic rows: uniform in [-3, 3), M_hint rows capped to [64, 262144]
    // (the chunking a shape gives depends on the row count, so tuning at the
    // real count matters)
    const int64_t Mt = std::max<int64_t>(64, std::min<int64_t>(M_hint > 0 ? M_hint : 16384,
                                                               262144));
    // tuning cache key parts: the device, and the row count's size class
    std::string device;
    {
      int dev = -1;
      check_hip(hipGetDevice(&dev), "hipGetDevice");
      hipDeviceProp_t prop;
      check_hip(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
      device = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
      for (char& ch : device)
        if (ch == ' ') ch = '_';
    }
    int64_t m_class = 0;
    while (((int64_t)1 << m_class) < Mt) ++m_class;
    const int pol = pol_index(ens);
    const int64_t K = h.n_groups;
    Scratch xs(sizeof(float) * (size_t)(Mt * F), s);
    const float* X = (const float*)xs.p;
    // the first-order kernels of wide feature spaces read it feature-major
    const int64_t ldt = wide_features((int)F) ? Mt : F;
    launch_fill_uniform((float*)xs.p, Mt * F, 0x2605u, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    struct EvGuard {
      hipEvent_t* a;
      hipEvent_t* b;
      ~EvGuard() {
        if (*a) (void)hipEventDestroy(*a);
        if (*b) (void)hipEventDestroy(*b);
      }
    } guard{&e0, &e1};
    check_hip(hipEventCreate(&e1), "hipEventCreate");
    // one untimed launch, then the mean of `reps` timed ones
    auto time_ms = [&](int reps, auto&& launch) {
      launch();
      check_hip(hipEventRecord(e0, s), "hipEventRecord");
      for (int r = 0; r < reps; ++r) launch();
      check_hip(hipEventRecord(e1, s), "hipEventRecord");
      check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      return ms / reps;
    };

    // first-order kernel (its shapes also serve the adjoint), per bucket
    {
      Scratch acc(sizeof(double) * (size_t)(Mt * K * F), s);
      launch_fill_zero((double*)acc.p, Mt * K * F, s);
      const std::vector<Bucket>& bks = ens->merge_siblings ? h.mbuckets : h.buckets;
      const PathArrays arr = ens->merge_siblings ? merged_arrays(d, h) : plain_arrays(d, h);
      Scratch slot0(slot0_bytes(value_rows(ens), fp64), s);
      launch_slot0(arr, value_rows(ens), d.leaf_val, fp64, slot0.p, s);
      for (const Bucket& bk : largest_per_capacity(bks)) {
        const std::string key = tune_key(device, "values", fp64, pol, h, bk.dmax, bk.group,
                                         bk.path_end - bk.path_begin, m_class);
        ValuesShape best;
        if (!tune_cache_get(key, &best.waves_per_block, &best.items)) {
          float best_ms = 1e30f;
          for (int waves : {4, 6, 8})
            for (int items : {4096, 8192, 16384, 32768, 65536}) {
              const ValuesShape cand{waves, items};
              const float ms = time_ms(3, [&] {
                launch_values(h, d, arr, bk, fp64, X, Mt, ldt, slot0.p, (double*)acc.p, nullptr,
                              cand, nodes_of(ens), s);
              });
              if (ms < best_ms) {
                best_ms = ms;
                best = cand;
              }
            }
          tune_cache_put(key, best.waves_per_block, best.items);
        }
        ens->vshape[pol][pi][cap_index(bk.dmax)] = best;
      }
    }
    // adjoint kernel, per bucket, with a synthetic upstream gradient
    {
      Scratch gl(sizeof(double) * (size_t)std::max<size_t>(1, h.leaf_value.size()), s);
      Scratch g32(sizeof(float) * (size_t)(Mt * K * F), s);
      launch_fill_uniform((float*)g32.p, Mt * K * F, 0x4a11u, s);
      Scratch g64(fp64 ? sizeof(double) * (size_t)(Mt * K * F) : 8, s);
      if (fp64) launch_widen_f32_f64((const float*)g32.p, (double*)g64.p, Mt * K * F, s);
      const void* G = fp64 ? g64.p : g32.p;
      launch_fill_zero((double*)gl.p, (int64_t)h.leaf_value.size(), s);
      const std::vector<Bucket>& bks = ens->merge_siblings ? h.mbuckets : h.buckets;
      const PathArrays arr = ens->merge_siblings ? merged_arrays(d, h) : plain_arrays(d, h);
      for (const Bucket& bk : largest_per_capacity(bks)) {
        const std::string key = tune_key(device, "adjoint", fp64, pol, h, bk.dmax, bk.group,
                                         bk.path_end - bk.path_begin, m_class);
        ValuesShape best;
        if (!tune_cache_get(key, &best.waves_per_block, &best.items)) {
          float best_ms = 1e30f;
          for (int waves : {4, 6, 8})
            for (int items : {4096, 8192, 16384, 32768, 65536}) {
              const ValuesShape cand{waves, items};
              const float ms = time_ms(3, [&] {
                launch_adjoint(h, d, arr, bk, fp64, X, G, Mt, ldt, (double*)gl.p, cand,
                               nodes_of(ens), s);
              });
              if (ms < best_ms) {
                best_ms = ms;
                best = cand;
              }
            }
          tune_cache_put(key, best.waves_per_block, best.items);
        }
        ens->ashape[pol][pi][cap_index(bk.dmax)] = best;
      }
    }
    // interactions, per capacity class, on at most 256 of the rows (and an
    // accumulator of at most 512 MiB)
    if (!ens->pair_classes.empty() && F >= 2) {
      const int64_t per_row = K * (F * (F - 1) / 2 + F);
      const int64_t Mp = std::max<int64_t>(
          1, std::min<int64_t>({Mt, (int64_t)256, ((int64_t)512 << 20) / (8 * per_row)}));
      Scratch acc(sizeof(double) * (size_t)(Mp * per_row), s);
      double* tri64 = (double*)acc.p;
      double* phi64 = tri64 + Mp * K * (F * (F - 1) / 2);
      launch_fill_zero(tri64, Mp * per_row, s);
      std::vector<PairShape>& out = ens->pshape[pol_index(ens)][pi];
      out.assign(ens->pair_classes.size(), PairShape{});
      for (size_t i = 0; i < ens->pair_classes.size(); ++i) {
        const PairClass& pc = ens->pair_classes[i];
        const std::string key = tune_key(device, "pairs", fp64, pol, h, pc.cap, pc.group, pc.np,
                                         m_class);
        PairShape best;
        if (!tune_cache_get(key, &best.max_chunk, &best.fill)) {
          float best_ms = 1e30f;
          for (int max_chunk : {8192, 32768, 131072})
            for (int fill : {1024, 4096}) {
              const PairShape cand{max_chunk, fill};
              const float ms = time_ms(1, [&] {
                launch_pairs(h, d, pc, fp64, X, Mp, F, d.leaf_val, tri64, phi64, cand,
                             ens->node_policy == QTS_NODES_EXACT, s);
              });
              if (ms < best_ms) {
                best_ms = ms;
                best = cand;
              }
            }
          tune_cache_put(key, best.max_chunk, best.fill);
        }
        out[i] = best;
      }
      // QTS_PAIRS_AUTO: time a whole interactions pass both ways on the same
      // rows (at most one depth-first batch) and keep the faster form
      // (the depth-first tables are built here on first use, where its walk
      // fits in LDS; otherwise the path form stays)
      if (ens->pair_traversal == QTS_PAIRS_AUTO && !ens->dfs.built &&
          dfs_walk_lds_bytes((int)F, h.max_depth, true) <= (size_t)kMaxLdsBytes)
        build_dfs(ens);
      if (ens->pair_traversal == QTS_PAIRS_AUTO && ens->dfs.built) {
        const std::string key = tune_key(device, "traversal", fp64, pol, h, 0, 0,
                                         ens->dfs.n_nodes, m_class);
        int choice = -1, unused = 0;
        if (!tune_cache_get(key, &choice, &unused)) {
          const int32_t md = (int32_t)std::min<int64_t>(Mp, dfs_batch(ens, Mp, fp64));
          Scratch y((size_t)md * (size_t)ens->dfs.n_rows * kNodes *
                        (fp64 ? sizeof(double) : sizeof(float)) + 256, s);
          Scratch lv(2 * (size_t)std::max<int64_t>(1, ens->dfs.n_nodes) *
                         (fp64 ? sizeof(double) : sizeof(float)), s);
          const float t_paths = time_ms(1, [&] {
            for (size_t i = 0; i < ens->pair_classes.size(); ++i)
              launch_pairs(h, d, ens->pair_classes[i], fp64, X, md, F, d.leaf_val, tri64, phi64,
                           out[i], ens->node_policy == QTS_NODES_EXACT, s);
          });
          const float t_dfs = time_ms(1, [&] {
            launch_dfs_walk(h, ens->dfs, d, fp64, d.leaf_val, X, 0, md, F, y.p, lv.p, s);
            launch_dfs_pairs(h, ens->dfs, d, fp64, X, 0, md, F, y.p, tri64, phi64, 128, s);
          });
          choice = t_dfs < t_paths ? 1 : 0;
          tune_cache_put(key, choice, 0);
        }
        ens->dfs_faster[pi] = choice == 1;
      }
      // the same choice for the third-order call, on fewer samples where its
      // accumulator (F(F-1)(F-2)/6 per sample) needs it
      if (ens->pair_traversal == QTS_PAIRS_AUTO && ens->dfs.built &&
          dfs_triples_supported(ens->dfs) && F >= 3) {
        const std::string key = tune_key(device, "traversal3", fp64, pol, h, 0, 0,
                                         ens->dfs.n_nodes, m_class);
        int choice = -1, unused = 0;
        if (!tune_cache_get(key, &choice, &unused)) {
          const int64_t T3 = F * (F - 1) * (F - 2) / 6;
          const int32_t m3 = (int32_t)std::max<int64_t>(
              1, std::min<int64_t>({Mp, (int64_t)dfs_batch(ens, Mp, fp64),
                                    ((int64_t)512 << 20) / (8 * K * T3)}));
          Scratch a3(sizeof(double) * (size_t)(m3 * K * T3), s);
          launch_fill_zero((double*)a3.p, m3 * K * T3, s);
          Scratch y((size_t)m3 * (size_t)ens->dfs.n_rows * kNodes *
                        (fp64 ? sizeof(double) : sizeof(float)) + 256, s);
          Scratch lv(2 * (size_t)std::max<int64_t>(1, ens->dfs.n_nodes) *
                         (fp64 ? sizeof(double) : sizeof(float)), s);
          float t_paths = 1e30f;
          try {
            t_paths = time_ms(1, [&] {
              for (const PairClass& pc : ens->pair_classes)
                launch_triples(h, d, pc, fp64, X, m3, F, d.leaf_val, (double*)a3.p, s);
            });
          } catch (const Error&) {
            // the path form's kernels do not fit this feature count
          }
          const float t_dfs = time_ms(1, [&] {
            launch_dfs_walk(h, ens->dfs, d, fp64, d.leaf_val, X, 0, m3, F, y.p, lv.p, s);
            launch_dfs_triples(h, ens->dfs, d, fp64, X, 0, m3, F, y.p, (double*)a3.p, 128, s);
          });
          choice = t_dfs < t_paths ? 1 : 0;
          tune_cache_put(key, choice, 0);
        }
        ens->dfs3_faster[pi] = choice == 1;
      }
    }
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    // cached graphs hold the old shapes
    std::lock_guard<std::mutex> lock(ens->graphs.mu);
    clear_graphs(ens->graphs);
  });
}

int qts_get_launch_shape(const qts_ensemble* ens, int32_t kind, qts_precision precision,
                         int32_t index, int32_t* a, int32_t* b) {
  return guarded([&] {
    if (!ens || !a || !b) fail(QTS_E_INVALID_ARG, "null argument");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    const bool fp64 = precision == QTS_FP64;
    if (kind == 0 || kind == 2) {
      if (index < 0 || index > 3) fail(QTS_E_INVALID_ARG, "bucket index out of range");
      const ValuesShape& v =
          (kind == 0 ? ens->vshape : ens->ashape)[pol_index(ens)][fp64 ? 1 : 0][index];
      *a = v.waves_per_block;
      *b = v.items;
    } else if (kind == 1) {
      if (index < 0 || (size_t)index >= ens->pair_classes.size())
        fail(QTS_E_INVALID_ARG, "class index out of range");
      const PairShape& v = pair_shape(ens, fp64, (size_t)index);
      *a = v.max_chunk;
      *b = v.fill;
    } else {
      fail(QTS_E_INVALID_ARG, "unknown kind");
    }
  });
}

int qts_set_tune_cache(const char* path) {
  return guarded([&] {
    TuneCache& c = tune_cache();
    std::lock_guard<std::mutex> g(c.mu);
    c.path = path ? path : "";
    c.loaded = false;
    c.entries.clear();
    c.hits = c.misses = 0;
  });
}

int qts_tune_cache_stats(int64_t* hits, int64_t* misses) {
  return guarded([&] {
    if (!hits || !misses) fail(QTS_E_INVALID_ARG, "null argument");
    TuneCache& c = tune_cache();
    std::lock_guard<std::mutex> g(c.mu);
    *hits = c.hits;
    *misses = c.misses;
  });
}

int qts_set_kernel_timing(int32_t enable) {
  return guarded([&] {
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.on = enable != 0;
  });
}

int qts_kernel_timing_read(int32_t kind, double* total_ms, int64_t* calls) {
  return guarded([&] {
    if (kind < 0 || kind > 3 || !total_ms || !calls) fail(QTS_E_INVALID_ARG, "bad argument");
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
      Timing& t = timing();
      std::lock_guard<std::mutex> g(t.mu);
      ev.swap(t.ev[kind]);
    }
    double total = 0.0;
    for (auto& pr : ev) {
      check_hip(hipEventSynchronize(pr.second), "hipEventSynchronize");
      float ms = 0.f;
      check_hip(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
      total += ms;
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    *total_ms = total;
    *calls = (int64_t)ev.size();
  });
}

const char* qts_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
