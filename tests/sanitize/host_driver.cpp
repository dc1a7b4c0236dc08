// Host-side driver for the sanitizer run: builds the path table, its pair
// table and the Gauss-Legendre rule from tree arrays read from a binary file,
// with the library's own host sources compiled under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Prints a summary line that the test compares
// with the library's host-only build of the same model.
//
// File layout (little endian): int32 n_trees, n_features, n_groups, n_nodes;
// int64 tree_offsets[n_trees + 1]; int32 left[n], right[n], feature[n];
// float threshold[n]; uint8 default_left[n]; double cover[n], value[n];
// int32 tree_group[n_trees]; double base_scores[n_groups].
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "qts_internal.h"

namespace qts {
[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }
}  // namespace qts

template <class T>
static void rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  if (n && std::fread(v.data(), sizeof(T), n, f) != n) {
    std::fprintf(stderr, "short file\n");
    std::exit(3);
  }
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[4];
  if (std::fread(hdr, sizeof(int32_t), 4, f) != 4) return 3;
  const int32_t T = hdr[0], F = hdr[1], K = hdr[2], N = hdr[3];
  std::vector<int64_t> off;
  std::vector<int32_t> left, right, feat, group;
  std::vector<float> thr;
  std::vector<uint8_t> dl;
  std::vector<double> cover, value, base;
  rd(f, off, (size_t)T + 1);
  rd(f, left, (size_t)N);
  rd(f, right, (size_t)N);
  rd(f, feat, (size_t)N);
  rd(f, thr, (size_t)N);
  rd(f, dl, (size_t)N);
  rd(f, cover, (size_t)N);
  rd(f, value, (size_t)N);
  rd(f, group, (size_t)T);
  rd(f, base, (size_t)K);
  std::fclose(f);
  qts_tree_arrays ta{T, off.data(), left.data(), right.data(), feat.data(), thr.data(),
                     dl.data(), cover.data(), value.data()};
  try {
    qts::HostTable h = qts::build_host_table(ta, F, K, group.data(), base.data());
    qts::PairTable pt = qts::build_pair_table(h);
    double t[64], s[64], w[64];
    double wsum = 0.0;
    for (int n : {1, 2, 4, 6, 8, 32, 64}) {
      qts::gauss_legendre(n, t, s, w);
      for (int m = 0; m < n; ++m) wsum += w[m];
    }
    int64_t pair_updates = 0;
    for (int32_t d : pt.d) pair_updates += (int64_t)d * (d - 1) / 2;
    const qts::DfsTable dt = qts::build_dfs_table(ta, h);
    std::printf("ok paths=%zu elements=%zu merged_rows=%zu pair_rows=%zu pair_updates=%lld "
                "segments=%zu dfs_nodes=%zu dfs_updates=%lld dfs_rows=%d expected=%.17g "
                "wsum=%.17g\n",
                h.hdr.size(), h.feat.size(), h.mhdr.size(), pt.d.size(),
                (long long)pair_updates, h.mcompact.segs.size(), dt.nodes.size(),
                (long long)dt.n_updates, dt.n_rows, h.expected, wsum);
  } catch (const qts::Error& e) {
    std::printf("error %d %s\n", e.code, e.msg.c_str());
  }
  return 0;
}
