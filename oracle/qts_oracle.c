/* FP64 CPU oracle for Path-Dependent TreeSHAP computed as Gauss-Legendre
 * quadrature of the weighted-Banzhaf polynomial.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * tables or constants with the GPU library: it builds its own quadrature
 * rule, walks the trees itself and evaluates every formula in the plainest
 * form, in double precision, with no blocking or reordering.
 *
 * Model semantics (the paper leaves them to the tree format; see the readings
 * listed with the tests):
 *   - a row goes left iff x < threshold, compared in float32; ties go right;
 *     a NaN feature value follows the node's default direction;
 *   - the edge weight is w_e = cover(child) / cover(parent) (section 2), taken
 *     as 0 when the parent cover is 0.
 *
 * Per root-to-leaf path P with leaf value val and unique features M(P):
 *   b_j = prod of w_e over the edges of P that split on j
 *   o_j = prod of 1[x satisfies e] over the same edges            (Eq. 2)
 * With R_empty = val * prod_j b_j (Eq. 1) and q_j = o_j / b_j (Eq. 2),
 * Theorem 1 (Eq. 7) gives the weighted-Banzhaf value of S inside M(P):
 *   B_p(S) = R_empty prod_{j in S}(q_j - 1) prod_{j notin S}((1-p) + p q_j)
 *          = val prod_{j in S}(o_j - b_j) prod_{j notin S}(b_j (1-p) + o_j p),
 * the second line multiplying every factor through by b_j, which also
 * defines the value when some b_j = 0.  Shapley values and Shapley
 * interaction indices are its integrals over p in [0,1] (Eq. 9), evaluated
 * with an n-point Gauss-Legendre rule on [0,1] (Eq. 10); the rule is exact
 * when 2n-1 >= d - |S| (Theorem 2, Eq. 12).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DEPTH 256
#define ORC_MAX_NODES 64

typedef struct {
  int32_t n_trees;
  const int64_t* tree_offsets;
  const int32_t* left;
  const int32_t* right;
  const int32_t* feature;
  const float* threshold;
  const uint8_t* default_left;
  const double* cover;
  const double* value;
  int32_t n_features;
} orc_model;

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [0,1]: Newton's method on the Legendre polynomial  */
/* P_n, evaluated by its three-term recurrence; weights 2/((1-x^2) P_n'(x)^2) */
/* on [-1,1], then t = (1-x)/2, s = 1-t = (1+x)/2, omega = W/2.               */
/* ------------------------------------------------------------------------ */
int orc_gauss_legendre(int n, double* t, double* s, double* omega) {
  if (n < 1 || n > ORC_MAX_NODES) return -1;
  const double pi = 3.14159265358979323846264338327950288;
  for (int i = 0; i < n; ++i) {
    double x = cos(pi * ((double)i + 0.75) / ((double)n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / (double)k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? x : p1, pm = (n == 1) ? 1.0 : p0;
      dp = (double)n * (x * pn - pm) / (x * x - 1.0);
      double dx = pn / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    /* final derivative at the converged root */
    {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / (double)k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? x : p1, pm = (n == 1) ? 1.0 : p0;
      dp = (double)n * (x * pn - pm) / (x * x - 1.0);
    }
    t[i] = 0.5 * (1.0 - x);
    s[i] = 0.5 * (1.0 + x);
    omega[i] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Tree walking                                                              */
/* ------------------------------------------------------------------------ */
static int goes_left(const orc_model* m, int64_t g, float xv) {
  if (isnan(xv)) return m->default_left[g] != 0;
  return xv < m->threshold[g];
}

static double edge_weight(const orc_model* m, int64_t parent, int64_t child) {
  double cp = m->cover[parent];
  if (cp == 0.0) return 0.0;
  return m->cover[child] / cp;
}

/* one edge on the current root-to-leaf path */
typedef struct { int32_t f; double w; int sat; } edge_t;

/* collapse the edges into unique features: b_j and o_j (Eq. 2) */
static int collapse(const edge_t* e, int ne, int32_t* fu, double* b, double* o) {
  int d = 0;
  for (int i = 0; i < ne; ++i) {
    int k = -1;
    for (int j = 0; j < d; ++j)
      if (fu[j] == e[i].f) { k = j; break; }
    if (k < 0) { k = d++; fu[k] = e[i].f; b[k] = 1.0; o[k] = 1.0; }
    b[k] *= e[i].w;
    o[k] *= e[i].sat ? 1.0 : 0.0;
  }
  return d;
}

/* Per-leaf callback signature: features, b, o, d, leaf value, leaf ordinal. */
typedef void (*leaf_fn)(void* ctx, const int32_t* fu, const double* b, const double* o,
                        int d, double val, int64_t leaf_ord);

/* Leaves are numbered in tree-major node-id order (the order of the model's
 * leaf values): the ordinal of a leaf is the number of leaf nodes with a
 * smaller id in its tree. */
static int64_t leaf_ordinal(const orc_model* m, int64_t base, int32_t node) {
  int64_t k = 0;
  for (int64_t g = base; g < base + node; ++g) k += (m->left[g] < 0);
  return k;
}

static void walk(const orc_model* m, int64_t base, int32_t node, const float* x,
                 edge_t* path, int depth, void* ctx, leaf_fn fn, int64_t* leaf_ord) {
  int64_t g = base + node;
  (void)leaf_ord;
  if (m->left[g] < 0) {
    int32_t fu[ORC_MAX_DEPTH];
    double b[ORC_MAX_DEPTH], o[ORC_MAX_DEPTH];
    int d = collapse(path, depth, fu, b, o);
    fn(ctx, fu, b, o, d, m->value[g], leaf_ordinal(m, base, node));
    return;
  }
  int32_t f = m->feature[g];
  int left_taken = goes_left(m, g, x[f]);
  int32_t kids[2] = {m->left[g], m->right[g]};
  for (int c = 0; c < 2; ++c) {
    path[depth].f = f;
    path[depth].w = edge_weight(m, g, base + kids[c]);
    path[depth].sat = (c == 0) ? left_taken : !left_taken;
    walk(m, base, kids[c], x, path, depth + 1, ctx, fn, leaf_ord);
  }
}

/* ------------------------------------------------------------------------ */
/* Quadrature contributions                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n;
  const double* t;
  const double* s;
  const double* omega;
  double* phi;     /* [F] for one sample, or NULL */
  double* sii;     /* [F*F] for one sample, or NULL */
  int32_t F;
  const double* gphi;  /* [F] upstream gradient for one sample (adjoint), or NULL */
  double* grad_leaf;   /* [n_leaves] (adjoint) */
  int64_t leaf_base;
} quad_ctx;

/* F_j(t) = b_j (1-t) + o_j t : the factor of feature j in Theorem 1,
 * multiplied through by b_j. */
static double factor(double b, double o, double t, double s) { return b * s + o * t; }

static void leaf_quadrature(void* vctx, const int32_t* fu, const double* b, const double* o,
                            int d, double val, int64_t leaf_ord) {
  quad_ctx* c = (quad_ctx*)vctx;
  /* first order: phi_i += val (o_i - b_i) sum_m omega_m prod_{j != i} F_j(t_m) */
  for (int i = 0; i < d; ++i) {
    double integral = 0.0;
    for (int m = 0; m < c->n; ++m) {
      double prod = 1.0;
      for (int j = 0; j < d; ++j)
        if (j != i) prod *= factor(b[j], o[j], c->t[m], c->s[m]);
      integral += c->omega[m] * prod;
    }
    double coef = (o[i] - b[i]) * integral; /* d phi_i / d val */
    if (c->phi) c->phi[fu[i]] += val * coef;
    if (c->grad_leaf) c->grad_leaf[c->leaf_base + leaf_ord] += c->gphi[fu[i]] * coef;
  }
  if (!c->sii) return;
  /* pairs: SII_ik += val (o_i-b_i)(o_k-b_k) sum_m omega_m prod_{j != i,k} F_j(t_m) */
  for (int i = 0; i < d; ++i) {
    for (int k = 0; k < d; ++k) {
      if (k == i) continue;
      double integral = 0.0;
      for (int m = 0; m < c->n; ++m) {
        double prod = 1.0;
        for (int j = 0; j < d; ++j)
          if (j != i && j != k) prod *= factor(b[j], o[j], c->t[m], c->s[m]);
        integral += c->omega[m] * prod;
      }
      c->sii[(int64_t)fu[i] * c->F + fu[k]] += val * (o[i] - b[i]) * (o[k] - b[k]) * integral;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Thread pool over work items                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t next;
  int64_t count;
  pthread_mutex_t mu;
  void (*run)(void* arg, int64_t item, int tid);
  void* arg;
} pool_t;

typedef struct { pool_t* p; int tid; } worker_arg;

static void* worker(void* va) {
  worker_arg* wa = (worker_arg*)va;
  pool_t* p = wa->p;
  for (;;) {
    pthread_mutex_lock(&p->mu);
    int64_t i = p->next++;
    pthread_mutex_unlock(&p->mu);
    if (i >= p->count) break;
    p->run(p->arg, i, wa->tid);
  }
  return NULL;
}

static void run_pool(int n_threads, int64_t count, void (*run)(void*, int64_t, int), void* arg) {
  if (n_threads < 1) n_threads = 1;
  pool_t p;
  p.next = 0;
  p.count = count;
  p.run = run;
  p.arg = arg;
  pthread_mutex_init(&p.mu, NULL);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  worker_arg* wa = (worker_arg*)malloc(sizeof(worker_arg) * (size_t)n_threads);
  for (int i = 0; i < n_threads; ++i) {
    wa[i].p = &p;
    wa[i].tid = i;
    pthread_create(&th[i], NULL, worker, &wa[i]);
  }
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  pthread_mutex_destroy(&p.mu);
  free(th);
  free(wa);
}

/* ------------------------------------------------------------------------ */
/* phi / SII by path quadrature                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_model* m;
  const float* X;
  int64_t M, ldx;
  int n;
  double t[ORC_MAX_NODES], s[ORC_MAX_NODES], omega[ORC_MAX_NODES];
  double* phi;  /* [M*F] or NULL */
  double* sii;  /* [M*F*F] or NULL */
  /* tree-parallel mode: per-thread buffers */
  int tree_parallel;
  double** tphi;
  double** tsii;
} quad_job;

static void quad_sample_tree(quad_job* j, int64_t sidx, int32_t tree, double* phi, double* sii) {
  const orc_model* m = j->m;
  quad_ctx c;
  memset(&c, 0, sizeof(c));
  c.n = j->n; c.t = j->t; c.s = j->s; c.omega = j->omega;
  c.phi = phi; c.sii = sii; c.F = m->n_features;
  edge_t path[ORC_MAX_DEPTH];
  int64_t leaf_ord = 0;
  walk(m, m->tree_offsets[tree], 0, j->X + sidx * j->ldx, path, 0, &c, leaf_quadrature,
       &leaf_ord);
}

static void quad_run(void* arg, int64_t item, int tid) {
  quad_job* j = (quad_job*)arg;
  const orc_model* m = j->m;
  int64_t F = m->n_features;
  if (!j->tree_parallel) {
    int64_t sidx = item;
    for (int32_t t = 0; t < m->n_trees; ++t)
      quad_sample_tree(j, sidx, t, j->phi ? j->phi + sidx * F : NULL,
                       j->sii ? j->sii + sidx * F * F : NULL);
  } else {
    int64_t sidx = item % j->M;
    int32_t t = (int32_t)(item / j->M);
    quad_sample_tree(j, sidx, t, j->tphi[tid] ? j->tphi[tid] + sidx * F : NULL,
                     j->tsii[tid] ? j->tsii[tid] + sidx * F * F : NULL);
  }
}

static int quad_common(const orc_model* m, const float* X, int64_t M, int64_t ldx, int n,
                       double* phi, double* sii, int n_threads) {
  if (!m || (M > 0 && !X) || n < 1 || n > ORC_MAX_NODES) return -1;
  quad_job j;
  memset(&j, 0, sizeof(j));
  j.m = m; j.X = X; j.M = M; j.ldx = ldx; j.n = n; j.phi = phi; j.sii = sii;
  if (orc_gauss_legendre(n, j.t, j.s, j.omega) != 0) return -1;
  int64_t F = m->n_features;
  if (phi) memset(phi, 0, sizeof(double) * (size_t)(M * F));
  if (sii) memset(sii, 0, sizeof(double) * (size_t)(M * F * F));
  if (n_threads < 1) n_threads = 1;
  if (M >= 2 * n_threads || m->n_trees <= 1) {
    run_pool(n_threads, M, quad_run, &j);
    return 0;
  }
  /* few samples: split trees across threads, each with private buffers */
  j.tree_parallel = 1;
  j.tphi = (double**)calloc((size_t)n_threads, sizeof(double*));
  j.tsii = (double**)calloc((size_t)n_threads, sizeof(double*));
  for (int i = 0; i < n_threads; ++i) {
    if (phi) j.tphi[i] = (double*)calloc((size_t)(M * F), sizeof(double));
    if (sii) j.tsii[i] = (double*)calloc((size_t)(M * F * F), sizeof(double));
  }
  run_pool(n_threads, M * (int64_t)m->n_trees, quad_run, &j);
  for (int i = 0; i < n_threads; ++i) {
    if (phi) for (int64_t k = 0; k < M * F; ++k) phi[k] += j.tphi[i][k];
    if (sii) for (int64_t k = 0; k < M * F * F; ++k) sii[k] += j.tsii[i][k];
    free(j.tphi[i]);
    free(j.tsii[i]);
  }
  free(j.tphi);
  free(j.tsii);
  return 0;
}

/* phi[M*F]: Shapley values by n-point path quadrature. */
int orc_shap_values(const orc_model* m, const float* X, int64_t M, int64_t ldx, int n,
                    double* phi, int n_threads) {
  if (!phi) return -1;
  return quad_common(m, X, M, ldx, n, phi, NULL, n_threads);
}

/* phi[M*F] (may be NULL) and sii[M*F*F]: Shapley interaction indices of every
 * ordered pair i != k (the diagonal is left 0). */
int orc_shap_interactions(const orc_model* m, const float* X, int64_t M, int64_t ldx, int n,
                          double* phi, double* sii, int n_threads) {
  if (!sii) return -1;
  return quad_common(m, X, M, ldx, n, phi, sii, n_threads);
}

/* ------------------------------------------------------------------------ */
/* Third-order Shapley interaction indices by path quadrature                */
/* ------------------------------------------------------------------------ */
/* Theorem 1 with |S| = 3 (Eq. 9-10): for three distinct features i, j, k of a
 * path,
 *   SII_ijk += val (o_i-b_i)(o_j-b_j)(o_k-b_k) sum_m omega_m prod_{l != i,j,k} F_l(t_m),
 * written to all six orderings of (i, j, k) of a dense [F*F*F] block. */
typedef struct {
  int n;
  const double* t;
  const double* s;
  const double* omega;
  double* sii3; /* [F*F*F] for one sample */
  int64_t F;
} tri_ctx;

static void leaf_triples(void* vctx, const int32_t* fu, const double* b, const double* o,
                         int d, double val, int64_t leaf_ord) {
  tri_ctx* c = (tri_ctx*)vctx;
  (void)leaf_ord;
  const int64_t F = c->F;
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j)
      for (int k = j + 1; k < d; ++k) {
        double integral = 0.0;
        for (int m = 0; m < c->n; ++m) {
          double prod = 1.0;
          for (int l = 0; l < d; ++l)
            if (l != i && l != j && l != k) prod *= factor(b[l], o[l], c->t[m], c->s[m]);
          integral += c->omega[m] * prod;
        }
        const double v = val * (o[i] - b[i]) * (o[j] - b[j]) * (o[k] - b[k]) * integral;
        const int64_t x = fu[i], y = fu[j], z = fu[k];
        c->sii3[(x * F + y) * F + z] += v;
        c->sii3[(x * F + z) * F + y] += v;
        c->sii3[(y * F + x) * F + z] += v;
        c->sii3[(y * F + z) * F + x] += v;
        c->sii3[(z * F + x) * F + y] += v;
        c->sii3[(z * F + y) * F + x] += v;
      }
}

typedef struct {
  const orc_model* m;
  const float* X;
  int64_t ldx;
  int n;
  double t[ORC_MAX_NODES], s[ORC_MAX_NODES], omega[ORC_MAX_NODES];
  double* sii3; /* [M*F*F*F] */
} tri_job;

static void tri_run(void* arg, int64_t sidx, int tid) {
  tri_job* j = (tri_job*)arg;
  const orc_model* m = j->m;
  const int64_t F = m->n_features;
  (void)tid;
  tri_ctx c;
  memset(&c, 0, sizeof(c));
  c.n = j->n; c.t = j->t; c.s = j->s; c.omega = j->omega;
  c.sii3 = j->sii3 + sidx * F * F * F;
  c.F = F;
  edge_t path[ORC_MAX_DEPTH];
  int64_t leaf_ord = 0;
  for (int32_t t = 0; t < m->n_trees; ++t)
    walk(m, m->tree_offsets[t], 0, j->X + sidx * j->ldx, path, 0, &c, leaf_triples, &leaf_ord);
}

/* sii3[M*F*F*F]: third-order Shapley interaction indices of every ordered
 * triple of distinct features (entries with a repeated index are 0). */
int orc_shap_sii3(const orc_model* m, const float* X, int64_t M, int64_t ldx, int n,
                  double* sii3, int n_threads) {
  if (!m || !sii3 || (M > 0 && !X) || n < 1 || n > ORC_MAX_NODES) return -1;
  tri_job j;
  memset(&j, 0, sizeof(j));
  j.m = m; j.X = X; j.ldx = ldx; j.n = n; j.sii3 = sii3;
  if (orc_gauss_legendre(n, j.t, j.s, j.omega) != 0) return -1;
  const int64_t F = m->n_features;
  memset(sii3, 0, sizeof(double) * (size_t)(M * F * F * F));
  run_pool(n_threads < 1 ? 1 : n_threads, M, tri_run, &j);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint: grad_leaf = J^T G with J[s,i,leaf] = d phi[s,i] / d val(leaf)    */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_model* m;
  const float* X;
  int64_t M, ldx;
  int n;
  double t[ORC_MAX_NODES], s[ORC_MAX_NODES], omega[ORC_MAX_NODES];
  const double* G;
  double* grad_leaf;
  int64_t* leaf_base; /* [n_trees] */
} grad_job;

static void grad_run(void* arg, int64_t tree, int tid) {
  (void)tid;
  grad_job* j = (grad_job*)arg;
  const orc_model* m = j->m;
  edge_t path[ORC_MAX_DEPTH];
  for (int64_t sidx = 0; sidx < j->M; ++sidx) {
    quad_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = j->n; c.t = j->t; c.s = j->s; c.omega = j->omega; c.F = m->n_features;
    c.gphi = j->G + sidx * m->n_features;
    c.grad_leaf = j->grad_leaf;
    c.leaf_base = j->leaf_base[tree];
    int64_t leaf_ord = 0;
    walk(m, m->tree_offsets[tree], 0, j->X + sidx * j->ldx, path, 0, &c, leaf_quadrature,
         &leaf_ord);
  }
}

int orc_leaf_grad(const orc_model* m, const float* X, int64_t M, int64_t ldx, int n,
                  const double* G, double* grad_leaf, int n_threads) {
  if (!m || !G || !grad_leaf || n < 1 || n > ORC_MAX_NODES) return -1;
  grad_job j;
  memset(&j, 0, sizeof(j));
  j.m = m; j.X = X; j.M = M; j.ldx = ldx; j.n = n; j.G = G; j.grad_leaf = grad_leaf;
  if (orc_gauss_legendre(n, j.t, j.s, j.omega) != 0) return -1;
  j.leaf_base = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m->n_trees + 1));
  int64_t nl = 0;
  for (int32_t t = 0; t < m->n_trees; ++t) {
    j.leaf_base[t] = nl;
    for (int64_t g = m->tree_offsets[t]; g < m->tree_offsets[t + 1]; ++g) nl += (m->left[g] < 0);
  }
  memset(grad_leaf, 0, sizeof(double) * (size_t)nl);
  run_pool(n_threads, m->n_trees, grad_run, &j);
  free(j.leaf_base);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* E[f] = v(empty) = sum over leaves of val * prod w_e (Eq. 1, Eq. 3), and    */
/* f(x) = v(all features) = the routed prediction.                           */
/* ------------------------------------------------------------------------ */
static double expected_rec(const orc_model* m, int64_t base, int32_t node) {
  int64_t g = base + node;
  if (m->left[g] < 0) return m->value[g];
  double acc = 0.0;
  int32_t kids[2] = {m->left[g], m->right[g]};
  for (int c = 0; c < 2; ++c)
    acc += edge_weight(m, g, base + kids[c]) * expected_rec(m, base, kids[c]);
  return acc;
}

int orc_expected_value(const orc_model* m, double* out) {
  if (!m || !out) return -1;
  double acc = 0.0;
  for (int32_t t = 0; t < m->n_trees; ++t) acc += expected_rec(m, m->tree_offsets[t], 0);
  *out = acc;
  return 0;
}

int orc_predict(const orc_model* m, const float* X, int64_t M, int64_t ldx, double* out) {
  if (!m || !out) return -1;
  for (int64_t i = 0; i < M; ++i) {
    const float* x = X + i * ldx;
    double acc = 0.0;
    for (int32_t t = 0; t < m->n_trees; ++t) {
      int64_t base = m->tree_offsets[t];
      int32_t node = 0;
      while (m->left[base + node] >= 0) {
        int64_t g = base + node;
        node = goes_left(m, g, x[m->feature[g]]) ? m->left[g] : m->right[g];
      }
      acc += m->value[base + node];
    }
    out[i] = acc;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Recursive TreeSHAP (Lundberg et al. 2020, the polynomial-time exact        */
/* algorithm the paper compares against).  Independent route to phi: it       */
/* tracks, per unique feature on the path, the fraction of zero paths (cover  */
/* ratio) and one paths (follow indicator), and the permutation weights of    */
/* each subset size, extending and unwinding them as the recursion moves.     */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t d; double z, o, w; } pe_t;

static void ts_extend(pe_t* m, int l, double pz, double po, int32_t pi) {
  /* m has l elements; append one and update the subset-size weights */
  m[l].d = pi; m[l].z = pz; m[l].o = po; m[l].w = (l == 0) ? 1.0 : 0.0;
  for (int i = l - 1; i >= 0; --i) {
    m[i + 1].w += po * m[i].w * (double)(i + 1) / (double)(l + 1);
    m[i].w = pz * m[i].w * (double)(l - i) / (double)(l + 1);
  }
}

/* remove element i from m (l elements); m ends with l-1 elements */
static void ts_unwind(pe_t* m, int l, int i) {
  double n = m[l - 1].w;
  double oi = m[i].o, zi = m[i].z;
  for (int j = l - 2; j >= 0; --j) {
    if (oi != 0.0) {
      double tmp = m[j].w;
      m[j].w = n * (double)l / ((double)(j + 1) * oi);
      n = tmp - m[j].w * zi * (double)(l - 1 - j) / (double)l;
    } else {
      m[j].w = m[j].w * (double)l / (zi * (double)(l - 1 - j));
    }
  }
  for (int j = i; j < l - 1; ++j) { m[j].d = m[j + 1].d; m[j].z = m[j + 1].z; m[j].o = m[j + 1].o; }
}

/* sum of the weights after removing element i, without modifying m */
static double ts_unwound_sum(const pe_t* m, int l, int i) {
  double oi = m[i].o, zi = m[i].z;
  double n = m[l - 1].w, total = 0.0;
  for (int j = l - 2; j >= 0; --j) {
    if (oi != 0.0) {
      double tmp = n * (double)l / ((double)(j + 1) * oi);
      total += tmp;
      n = m[j].w - tmp * zi * (double)(l - 1 - j) / (double)l;
    } else {
      total += (m[j].w / zi) / ((double)(l - 1 - j) / (double)l);
    }
  }
  return total;
}

static void ts_recurse(const orc_model* mdl, int64_t base, int32_t node, const float* x,
                       double* phi, pe_t* parent, int pl, double pz, double po, int32_t pi) {
  pe_t m[ORC_MAX_DEPTH + 2];
  memcpy(m, parent, sizeof(pe_t) * (size_t)pl);
  ts_extend(m, pl, pz, po, pi);
  int l = pl + 1;
  int64_t g = base + node;
  if (mdl->left[g] < 0) {
    for (int i = 1; i < l; ++i) {
      double w = ts_unwound_sum(m, l, i);
      phi[m[i].d] += w * (m[i].o - m[i].z) * mdl->value[g];
    }
    return;
  }
  int32_t f = mdl->feature[g];
  int32_t hot = goes_left(mdl, g, x[f]) ? mdl->left[g] : mdl->right[g];
  int32_t cold = (hot == mdl->left[g]) ? mdl->right[g] : mdl->left[g];
  double iz = 1.0, io = 1.0;
  int k = -1;
  for (int i = 1; i < l; ++i)
    if (m[i].d == f) { k = i; break; }
  if (k >= 0) {
    iz = m[k].z;
    io = m[k].o;
    ts_unwind(m, l, k);
    --l;
  }
  double cg = mdl->cover[g];
  double rh = cg == 0.0 ? 0.0 : mdl->cover[base + hot] / cg;
  double rc = cg == 0.0 ? 0.0 : mdl->cover[base + cold] / cg;
  ts_recurse(mdl, base, hot, x, phi, m, l, iz * rh, io, f);
  ts_recurse(mdl, base, cold, x, phi, m, l, iz * rc, 0.0, f);
}

typedef struct {
  const orc_model* m;
  const float* X;
  int64_t ldx;
  double* phi;
} ts_job;

static void ts_run(void* arg, int64_t sidx, int tid) {
  (void)tid;
  ts_job* j = (ts_job*)arg;
  const orc_model* m = j->m;
  double* phi = j->phi + sidx * m->n_features;
  pe_t root[1];
  for (int32_t t = 0; t < m->n_trees; ++t)
    ts_recurse(m, m->tree_offsets[t], 0, j->X + sidx * j->ldx, phi, root, 0, 1.0, 1.0, -1);
}

int orc_treeshap(const orc_model* m, const float* X, int64_t M, int64_t ldx, double* phi,
                 int n_threads) {
  if (!m || !phi) return -1;
  memset(phi, 0, sizeof(double) * (size_t)(M * m->n_features));
  ts_job j = {m, X, ldx, phi};
  run_pool(n_threads, M, ts_run, &j);
  return 0;
}
