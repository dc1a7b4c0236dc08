/* Depth-first tree grower for the synthetic "grown" ensembles.
 *
 * Part of the seeded input generator only: it builds tree structure and
 * training-row counts (covers).  It holds no Shapley/quadrature arithmetic.
 * All random draws come from the caller (numpy PCG64), consumed in order,
 * so the Python side owns the seed.
 *
 * Recipe: at each node a feature is drawn uniformly; the threshold is the
 * order statistic of the node's own training rows at rank round(u*n),
 * u ~ U(0.05, 0.95), clamped to [1, n-1] so both children start non-empty.
 * Rows go left iff x < threshold (float32 compare).  Nodes are expanded
 * depth-first, bigger child first, until the maximum depth, fewer than two
 * rows, or the leaf cap is reached.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int32_t node; int32_t depth; int64_t begin, end; } frame_t;

/* k-th smallest of v[0..n) (Hoare quickselect, deterministic middle pivot);
 * reorders v. */
static float select_kth(float* v, int64_t n, int64_t k) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    float pivot = v[lo + (hi - lo) / 2];
    int64_t i = lo, j = hi;
    while (i <= j) {
      while (v[i] < pivot) ++i;
      while (v[j] > pivot) --j;
      if (i <= j) { float t = v[i]; v[i] = v[j]; v[j] = t; ++i; --j; }
    }
    if (k <= j) hi = j;
    else if (k >= i) lo = i;
    else return v[k];
  }
  return v[k];
}

/* Returns the number of nodes written, or -1 when max_nodes is too small.
 * xt: training matrix transposed, [n_features][n_rows] float32.
 * rand_feat / rand_u: per-split random draws (feature in [0,F), u in [0.05,0.95)),
 *   at least max_nodes of each.  rand_left: bernoulli bits for default_left.
 * Outputs (length max_nodes): left, right (-1 for leaves), feature, threshold,
 *   default_left, cover. */
int64_t grow_tree(const float* xt, int64_t n_rows, int32_t n_features,
                  int32_t max_depth, int64_t leaf_cap,
                  const int32_t* rand_feat, const double* rand_u,
                  const uint8_t* rand_left, int64_t max_nodes,
                  int32_t* left, int32_t* right, int32_t* feature,
                  float* threshold, uint8_t* default_left, double* cover) {
  (void)n_features;
  int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_rows > 0 ? n_rows : 1));
  int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_rows > 0 ? n_rows : 1));
  float* vals = (float*)malloc(sizeof(float) * (size_t)(n_rows > 0 ? n_rows : 1));
  frame_t* stack = (frame_t*)malloc(sizeof(frame_t) * (size_t)(max_nodes + 1));
  if (!rows || !tmp || !vals || !stack) { free(rows); free(tmp); free(vals); free(stack); return -1; }
  for (int64_t i = 0; i < n_rows; ++i) rows[i] = i;

  int64_t n_nodes = 1, n_leaves = 1, draw = 0, sp = 0;
  left[0] = right[0] = -1; feature[0] = 0; threshold[0] = 0.f; default_left[0] = 0;
  cover[0] = (double)n_rows;
  stack[sp++] = (frame_t){0, 0, 0, n_rows};
  while (sp > 0) {
    frame_t fr = stack[--sp];
    int64_t n = fr.end - fr.begin;
    if (fr.depth >= max_depth || n < 2 || n_leaves >= leaf_cap) continue;
    if (n_nodes + 2 > max_nodes || draw >= max_nodes) { n_nodes = -1; break; }
    int32_t f = rand_feat[draw];
    double u = rand_u[draw];
    uint8_t dl = rand_left[draw];
    ++draw;
    const float* col = xt + (int64_t)f * n_rows;
    for (int64_t i = 0; i < n; ++i) vals[i] = col[rows[fr.begin + i]];
    int64_t k = (int64_t)(u * (double)n + 0.5);
    if (k < 1) k = 1;
    if (k > n - 1) k = n - 1;
    float thr = select_kth(vals, n, k);
    /* stable partition: left rows first */
    int64_t nl = 0, nr = 0;
    for (int64_t i = 0; i < n; ++i) {
      int64_t r = rows[fr.begin + i];
      if (col[r] < thr) rows[fr.begin + nl++] = r; else tmp[nr++] = r;
    }
    if (nl == 0 || nr == 0) {  /* ties: restore order-insensitive content, keep leaf */
      memcpy(rows + fr.begin + nl, tmp, sizeof(int64_t) * (size_t)nr);
      continue;
    }
    memcpy(rows + fr.begin + nl, tmp, sizeof(int64_t) * (size_t)nr);
    int32_t l = (int32_t)n_nodes, r = (int32_t)n_nodes + 1;
    n_nodes += 2;
    n_leaves += 1;
    left[fr.node] = l; right[fr.node] = r; feature[fr.node] = f;
    threshold[fr.node] = thr; default_left[fr.node] = dl;
    left[l] = right[l] = left[r] = right[r] = -1;
    feature[l] = feature[r] = 0; threshold[l] = threshold[r] = 0.f;
    default_left[l] = default_left[r] = 0;
    cover[l] = (double)nl; cover[r] = (double)nr;
    frame_t fl = {l, fr.depth + 1, fr.begin, fr.begin + nl};
    frame_t fg = {r, fr.depth + 1, fr.begin + nl, fr.end};
    /* bigger child is expanded first: push it last */
    if (nl >= nr) { stack[sp++] = fg; stack[sp++] = fl; }
    else          { stack[sp++] = fl; stack[sp++] = fg; }
  }
  free(rows); free(tmp); free(vals); free(stack);
  return n_nodes;
}

/* Breadth-first full-depth tree for the "random" recipe.
 * Candidate splits are pre-drawn by the caller: for the k-th node considered
 * for a split (breadth-first order) and try t, the feature is
 * cand_feat[k*max_tries+t] and the threshold cand_thr_int[...] on an integer
 * column (is_int[f] != 0), cand_thr_norm[...] otherwise.  The first candidate
 * that leaves both children non-empty is taken; after max_tries the node stays
 * a leaf.  Returns the node count, or -1 when max_nodes is too small. */
int64_t random_tree(const float* xt, int64_t n_rows, int32_t n_features,
                    int32_t max_depth, const uint8_t* is_int,
                    const int32_t* cand_feat, const float* cand_thr_norm,
                    const float* cand_thr_int, const uint8_t* rand_left,
                    int32_t max_tries, int64_t max_cands, int64_t max_nodes,
                    int32_t* left, int32_t* right, int32_t* feature,
                    float* threshold, uint8_t* default_left, double* cover) {
  (void)n_features;
  int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_rows > 0 ? n_rows : 1));
  int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_rows > 0 ? n_rows : 1));
  frame_t* queue = (frame_t*)malloc(sizeof(frame_t) * (size_t)(max_nodes + 1));
  if (!rows || !tmp || !queue) { free(rows); free(tmp); free(queue); return -1; }
  for (int64_t i = 0; i < n_rows; ++i) rows[i] = i;
  int64_t n_nodes = 1, head = 0, tail = 0, k = 0;
  left[0] = right[0] = -1; feature[0] = 0; threshold[0] = 0.f; default_left[0] = 0;
  cover[0] = (double)n_rows;
  queue[tail++] = (frame_t){0, 0, 0, n_rows};
  while (head < tail) {
    frame_t fr = queue[head++];
    int64_t n = fr.end - fr.begin;
    if (fr.depth >= max_depth || n < 2) continue;
    if (k >= max_cands || n_nodes + 2 > max_nodes) { n_nodes = -1; break; }
    int32_t f = 0; float thr = 0.f; int64_t nl = 0; int ok = 0;
    for (int32_t t = 0; t < max_tries && !ok; ++t) {
      int64_t c = k * max_tries + t;
      f = cand_feat[c];
      thr = is_int[f] ? cand_thr_int[c] : cand_thr_norm[c];
      const float* col = xt + (int64_t)f * n_rows;
      nl = 0;
      for (int64_t i = fr.begin; i < fr.end; ++i) nl += (col[rows[i]] < thr);
      ok = (nl > 0 && nl < n);
    }
    uint8_t dl = rand_left[k];
    ++k;
    if (!ok) continue;
    const float* col = xt + (int64_t)f * n_rows;
    int64_t a = 0, b = 0;
    for (int64_t i = fr.begin; i < fr.end; ++i) {
      int64_t r = rows[i];
      if (col[r] < thr) rows[fr.begin + a++] = r; else tmp[b++] = r;
    }
    memcpy(rows + fr.begin + a, tmp, sizeof(int64_t) * (size_t)b);
    int32_t l = (int32_t)n_nodes, r = (int32_t)n_nodes + 1;
    n_nodes += 2;
    left[fr.node] = l; right[fr.node] = r; feature[fr.node] = f;
    threshold[fr.node] = thr; default_left[fr.node] = dl;
    left[l] = right[l] = left[r] = right[r] = -1;
    feature[l] = feature[r] = 0; threshold[l] = threshold[r] = 0.f;
    default_left[l] = default_left[r] = 0;
    cover[l] = (double)a; cover[r] = (double)b;
    queue[tail++] = (frame_t){l, fr.depth + 1, fr.begin, fr.begin + a};
    queue[tail++] = (frame_t){r, fr.depth + 1, fr.begin + a, fr.end};
  }
  free(rows); free(tmp); free(queue);
  return n_nodes;
}
