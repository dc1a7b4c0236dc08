// C-ABI entry points (declared in include/qtreeshap.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "qts_device.h"
#include "qts_internal.h"
#include "qtreeshap.h"

struct qts_ensemble {
  qts::HostTable host;
  std::vector<qts::PairClass> pair_classes;
  qts::DeviceTable dev;
  bool on_device = false;
  // launch shapes per bucket capacity index (8, 16, 32, 64) and precision
  qts::ValuesShape vshape[2][4];
};

namespace qts {

namespace {
thread_local std::string g_last_error;

int cap_index(int dmax) { return dmax <= 8 ? 0 : dmax <= 16 ? 1 : dmax <= 32 ? 2 : 3; }

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

template <class T>
T* upload(const std::vector<T>& v, hipStream_t s) {
  if (v.empty()) return nullptr;
  T* p = nullptr;
  check_hip(hipMalloc(reinterpret_cast<void**>(&p), v.size() * sizeof(T)), "hipMalloc");
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

void free_device(DeviceTable& d) {
  void* ptrs[] = {d.hdr,    d.feat,    d.lo,      d.hi,      d.b32,     d.cb32,
                  d.b64,    d.cb64,    d.leaf_val, d.pr_d,   d.pr_leaf, d.pr_feat,
                  d.pr_lo,  d.pr_hi,   d.pr_b32,  d.pr_cb32, d.pr_b64,  d.pr_cb64};
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
  }
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
    check_hip(hipMallocAsync(&p, bytes, s), "hipMallocAsync");
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
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
};
Timing& timing() {
  static Timing t;
  return t;
}

// Records an event pair around a scope when timing is enabled.
class TimedScope {
 public:
  TimedScope(int kind, hipStream_t s) : kind_(kind), s_(s) {
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

int qts_build_host(const qts_tree_arrays* trees, int32_t n_features, double base_score,
                   qts_ensemble** out) {
  return guarded([&] {
    if (!trees || !out) fail(QTS_E_INVALID_ARG, "null argument");
    *out = nullptr;
    qts_ensemble* e = new qts_ensemble();
    try {
      e->host = build_host_table(*trees, n_features, base_score);
    } catch (...) {
      delete e;
      throw;
    }
    *out = e;
  });
}

int qts_load_ensemble(const qts_tree_arrays* trees, int32_t n_features, double base_score,
                      void* stream, qts_ensemble** out) {
  return guarded([&] {
    if (!trees || !out) fail(QTS_E_INVALID_ARG, "null argument");
    *out = nullptr;
    qts_ensemble* e = new qts_ensemble();
    try {
      e->host = build_host_table(*trees, n_features, base_score);
      const HostTable& h = e->host;
      hipStream_t s = (hipStream_t)stream;
      DeviceTable& d = e->dev;
      check_hip(hipGetDevice(&d.device), "hipGetDevice");
      build_nodes(d);
      // Device layout: every path is padded to whole batches of eight
      // elements with inert slots (feature 0, no bounds, missing_ok, b = 1,
      // 1-b = 0): their factor is exactly 1 and their contribution 0, so the
      // kernels process whole batches without per-slot tests.
      std::vector<PathHdr> hdr = h.hdr;
      std::vector<int32_t> feat;
      std::vector<float> lo, hi;
      std::vector<double> b64, cb64;
      size_t n_pad = 0;
      for (const PathHdr& p : h.hdr) n_pad += (size_t)((p.d + 7) / 8) * 8;
      feat.reserve(n_pad); lo.reserve(n_pad); hi.reserve(n_pad);
      b64.reserve(n_pad); cb64.reserve(n_pad);
      for (size_t i = 0; i < h.hdr.size(); ++i) {
        const PathHdr& p = h.hdr[i];
        hdr[i].off = (int32_t)feat.size();
        const int padded_d = (p.d + 7) / 8 * 8;
        for (int k = 0; k < padded_d; ++k) {
          const bool real = k < p.d;
          const size_t e = (size_t)p.off + (size_t)k;
          feat.push_back(real ? h.feat[e] : kMissingOkBit);
          lo.push_back(real ? h.lo[e] : -INFINITY);
          hi.push_back(real ? h.hi[e] : NAN);
          b64.push_back(real ? h.b[e] : 1.0);
          cb64.push_back(real ? h.cb[e] : 0.0);
        }
      }
      if (feat.size() > (size_t)0x7fffffff) fail(QTS_E_UNSUPPORTED, "path table too large");
      feat = padded(feat, (int32_t)kMissingOkBit);
      lo = padded(lo, -INFINITY);
      hi = padded(hi, NAN);
      b64 = padded(b64, 1.0);
      cb64 = padded(cb64, 0.0);
      std::vector<float> b32 = narrow<float>(b64), cb32 = narrow<float>(cb64);
      d.hdr = upload(hdr, s);
      d.feat = upload(feat, s);
      d.lo = upload(lo, s);
      d.hi = upload(hi, s);
      d.b32 = upload(b32, s);
      d.cb32 = upload(cb32, s);
      d.b64 = upload(b64, s);
      d.cb64 = upload(cb64, s);
      d.leaf_val = upload(h.leaf_value, s);
      {
        PairTable pt = build_pair_table(h);
        e->pair_classes = pt.classes;
        d.pr_d = upload(pt.d, s);
        d.pr_leaf = upload(pt.leaf, s);
        d.pr_feat = upload(pt.feat, s);
        d.pr_lo = upload(pt.lo, s);
        d.pr_hi = upload(pt.hi, s);
        d.pr_b32 = upload(narrow<float>(pt.b), s);
        d.pr_cb32 = upload(narrow<float>(pt.cb), s);
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

int qts_free_ensemble(qts_ensemble* ens) {
  return guarded([&] {
    if (!ens) return;
    if (ens->on_device) free_device(ens->dev);
    delete ens;
  });
}

int qts_expected_value(const qts_ensemble* ens, double* out) {
  return guarded([&] {
    if (!ens || !out) fail(QTS_E_INVALID_ARG, "null argument");
    *out = ens->host.expected;
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
    const HostTable& h = ens->host;
    const DeviceTable& d = ens->dev;
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    const int64_t n = M * h.F;
    const double* leaf = leaf_values ? leaf_values : d.leaf_val;
    if (fp64) {
      double* acc = (double*)phi;
      launch_fill_zero(acc, n, s);
      TimedScope ts(0, s);
      for (const Bucket& bk : h.buckets)
        launch_values(h, d, bk, true, X, M, ldx, leaf, acc, ens->vshape[1][cap_index(bk.dmax)], s);
      ts.done();
    } else {
      Scratch acc(sizeof(double) * (size_t)n, s);
      double* a = (double*)acc.p;
      launch_fill_zero(a, n, s);
      TimedScope ts(0, s);
      for (const Bucket& bk : h.buckets)
        launch_values(h, d, bk, false, X, M, ldx, leaf, a, ens->vshape[0][cap_index(bk.dmax)], s);
      ts.done();
      launch_cast_f64_f32(a, (float*)phi, n, s);
    }
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
    const HostTable& h = ens->host;
    const DeviceTable& d = ens->dev;
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    const int64_t F = h.F;
    const int64_t ntri = F * (F - 1) / 2;
    const double* leaf = leaf_values ? leaf_values : d.leaf_val;
    Scratch acc(sizeof(double) * (size_t)(M * ntri + M * F), s);
    double* tri64 = (double*)acc.p;
    double* phi64 = tri64 + M * ntri;
    launch_fill_zero(tri64, M * ntri + M * F, s);
    TimedScope ts(1, s);
    for (const PairClass& pc : ens->pair_classes)
      launch_pairs(h, d, pc, fp64, X, M, ldx, leaf, tri64, phi64, s);
    ts.done();
    launch_pairs_finalize(tri64, phi64, M, (int)F, fp64, Phi, phi, s);
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
    const HostTable& h = ens->host;
    const DeviceTable& d = ens->dev;
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = precision == QTS_FP64;
    launch_fill_zero(grad_leaf, (int64_t)h.leaf_value.size(), s);
    if (M == 0) return;
    TimedScope ts(2, s);
    for (const Bucket& bk : h.buckets)
      launch_adjoint(h, d, bk, fp64, X, grad_phi, M, ldx, grad_leaf,
                     ens->vshape[fp64 ? 1 : 0][cap_index(bk.dmax)], s);
    ts.done();
  });
}

int qts_autotune(qts_ensemble* ens, int64_t M_hint, qts_precision precision, void* stream) {
  (void)M_hint; (void)stream;
  return guarded([&] {
    if (!ens) fail(QTS_E_INVALID_ARG, "null ensemble");
    if (precision != QTS_FP32 && precision != QTS_FP64)
      fail(QTS_E_INVALID_ARG, "unknown precision");
    require_device(ens);
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
    if (kind < 0 || kind > 2 || !total_ms || !calls) fail(QTS_E_INVALID_ARG, "bad argument");
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
