/* qtreeshap: Path-Dependent TreeSHAP as Gauss-Legendre quadrature of the
 * weighted-Banzhaf polynomial, on AMD Instinct MI355X (gfx950).
 *
 * Method (Wettenstein, Mitchell, Yu, "Quadrature-TreeSHAP"):
 *   For a leaf v reached by a root-to-leaf path, each unique feature j on the
 *   path has a cover ratio b_j (the product of the path's edge weights
 *   w_e = cover(child)/cover(parent) on splits of j, section 2) and a follow
 *   indicator o_j (1 iff the sample satisfies every split on j, Eq. 2).
 *   Theorem 1 gives the weighted-Banzhaf interaction of a set S at inclusion
 *   probability p; multiplied through by prod_j b_j it reads
 *     B_p(S) = val(v) prod_{j in S}(o_j - b_j) prod_{j notin S}(b_j (1-p) + o_j p).
 *   Shapley values (|S|=1) and pairwise Shapley interaction indices (|S|=2)
 *   are its integrals over p in [0,1] (Eq. 9), computed with the fixed
 *   8-node Gauss-Legendre rule on [0,1] (Eq. 10, section 5).  The rule is
 *   exact whenever the path has at most 16 unique features for values and 17
 *   for pairs (Theorem 2, Eq. 12); beyond that it is the paper's quadrature
 *   approximation.
 *
 * Conventions used by this library (the paper leaves them to the tree format):
 *   - a sample goes to the left child iff x[feature] < threshold (float32
 *     compare; ties go right); NaN means "missing" and follows default_left;
 *   - w_e = 0 when the parent cover is 0;
 *   - interaction matrix Phi[i][k] = SII_ik / 2 for i != k and
 *     Phi[i][i] = phi_i - sum_{k != i} Phi[i][k], so rows sum to phi and Phi is
 *     symmetric (the layout of XGBoost's pred_interactions, which the paper's
 *     implementation keeps, section 1);
 *   - outputs exclude the bias: expected_value() returns sum_T E_T[f] + base_score,
 *     so phi.sum(-1) + expected_value = prediction.
 *
 * Memory: every X, output and gradient pointer is DEVICE memory owned by the
 * caller; host arrays passed to qts_load_ensemble are copied and may be freed
 * after it returns.  Outputs are overwritten, never accumulated into.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Compute
 * calls are asynchronous on that stream; the caller synchronises before
 * reading outputs.  Compute calls on one ensemble may run from several
 * streams concurrently; the settings calls (qts_autotune,
 * qts_set_graph_replay, qts_set_sibling_merge, qts_set_node_policy) must not
 * overlap compute calls on the same ensemble.  qts_free_ensemble requires that
 * no work on the ensemble is still in flight.
 *
 * Errors: every call returns QTS_OK (0) or a negative code below; the text of
 * the last error on the calling thread is available from qts_last_error().
 * No C++ exception crosses this interface.
 */
#ifndef QTREESHAP_H
#define QTREESHAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QTS_OK = 0,
  QTS_E_INVALID_ARG = -1,   /* null pointer, negative size, ldx < n_features, ... */
  QTS_E_INVALID_MODEL = -2, /* child out of range, cycle, one-child node, feature >= F,
                               negative or NaN cover, NaN threshold */
  QTS_E_UNSUPPORTED = -3,   /* tree deeper than 128, path with > 64 unique features;
                               qts_shap_interactions3 in the path form also
                               when one feature's triples do not fit in LDS
                               (F above about 180 to 203) */
  QTS_E_HIP = -4,           /* a HIP runtime error; its text is in qts_last_error() */
  QTS_E_OOM = -5            /* host or device allocation failed */
};

typedef enum { QTS_FP32 = 0, QTS_FP64 = 1 } qts_precision;

typedef struct qts_ensemble qts_ensemble; /* opaque, owned by the library */

/* A tree ensemble as structure-of-arrays host memory (node ids local to each
 * tree, root = node 0 of each tree). */
typedef struct {
  int32_t n_trees;
  const int64_t* tree_offsets; /* [n_trees+1]: tree t owns nodes [off[t], off[t+1]) */
  const int32_t* left;         /* [N] local child id, -1 for a leaf */
  const int32_t* right;        /* [N] local child id, -1 for a leaf */
  const int32_t* feature;      /* [N] split feature in [0, n_features) (internal nodes) */
  const float* threshold;      /* [N] left iff x < threshold (internal nodes) */
  const uint8_t* default_left; /* [N] missing-value direction; NULL = all go right */
  const double* cover;         /* [N] training rows (or weight) reaching the node, >= 0 */
  const double* value;         /* [N] leaf value (leaves only) */
} qts_tree_arrays;

/* Validate the model, build its path table and copy it to the current HIP
 * device (the device current on the calling thread).  Per leaf, the path is
 * collapsed to its unique features (Eq. 2) with b_j in FP64, 1-b_j computed in
 * FP64, and the interval of x values that follows every split on j.  Paths
 * are grouped by unique-feature count.  Synchronous with respect to host
 * memory.  `stream` orders the uploads. */
int qts_load_ensemble(const qts_tree_arrays* trees, int32_t n_features, double base_score,
                      void* stream, qts_ensemble** out);

/* Same validation and path table, host memory only (no device is touched).
 * Usable with the query calls and qts_export_paths; compute calls reject it. */
int qts_build_host(const qts_tree_arrays* trees, int32_t n_features, double base_score,
                   qts_ensemble** out);

/* Multi-output ensembles: each tree adds to the output of one group (for
 * example one group per class of a multiclass model; the XGBoost entry points
 * the paper's implementation serves, section 1, return attributions per
 * output).  The game of group g is the sum over its own trees of the
 * path-dependent games of Eq. 3, so each group's Shapley values and
 * interaction indices are those of its sub-ensemble.
 *   tree_group   [n_trees] group of each tree in [0, n_groups) (NULL: all in
 *                group 0); a group outside that range is QTS_E_INVALID_MODEL
 *   base_scores  [n_groups] bias of each group (host memory)
 * The compute calls then return one block per group inside each sample row:
 * phi [M, n_groups, F], Phi [M, n_groups, F, F], third-order
 * [M, n_groups, F(F-1)(F-2)/6], and take grad_phi as [M, n_groups, F];
 * grad_leaf keeps its length and order.  qts_load_ensemble and qts_build_host
 * are these calls with one group (n_groups = 1: the shapes below). */
int qts_load_ensemble_grouped(const qts_tree_arrays* trees, const int32_t* tree_group,
                              int32_t n_groups, int32_t n_features, const double* base_scores,
                              void* stream, qts_ensemble** out);
int qts_build_host_grouped(const qts_tree_arrays* trees, const int32_t* tree_group,
                           int32_t n_groups, int32_t n_features, const double* base_scores,
                           qts_ensemble** out);

int qts_free_ensemble(qts_ensemble* ens);

/* sum over trees of E_T[f] = v(empty set) (Eq. 1, Eq. 3) plus base_score, FP64
 * (with output groups: group 0's). */
int qts_expected_value(const qts_ensemble* ens, double* out);

/* The same per output group: out[n_groups]. */
int qts_expected_values(const qts_ensemble* ens, double* out);

/* Number of leaves = length of grad_leaf and of a leaf_values override, in
 * tree-major, node-id order. */
int qts_num_leaves(const qts_ensemble* ens, int64_t* out);

typedef struct {
  int32_t n_features;
  int32_t n_trees;
  int64_t n_leaves;    /* leaves in tree-major node-id order (incl. unreachable slots) */
  int64_t n_paths;     /* root-to-leaf paths with at least one split (table rows) */
  int64_t n_elements;  /* sum over paths of unique features */
  int32_t max_depth;   /* D */
  int32_t max_unique;  /* d */
  int32_t n_buckets;
  int32_t device;      /* -1 for a host-only ensemble */
  int32_t n_pair_classes;  /* capacity classes of the interactions table */
  int32_t n_graphs;        /* graphs held by the replay cache */
  int64_t n_merged;        /* sibling-leaf pairs merged in the first-order table */
  int64_t n_value_paths;   /* rows of the first-order table (n_paths - n_merged) */
  int64_t n_value_elements;  /* sum of d over those rows */
  int64_t n_pair_rows;       /* rows of the interactions table (0: host-only ensemble) */
  int64_t n_pair_elements;   /* sum of d over them */
  int64_t n_pair_updates;    /* sum of d(d-1)/2 over them: pair updates per sample */
  int64_t n_value_shared;    /* first-order rows: leading slots after slot 0 equal
                                to the previous row's, summed (the kernels reuse
                                their work instead of evaluating it again) */
  int64_t n_path_shared;     /* the same for the unmerged table */
  int64_t n_value_segments;  /* work segments of the merged first-order table when
                                the sample tile of all features does not fit in
                                LDS (more than 210 features): consecutive rows
                                using at most 96 distinct features; 0 otherwise */
  int32_t n_groups;          /* output groups (1 unless loaded grouped) */
  int32_t pairs_dfs;         /* bit 0 (FP32), bit 1 (FP64): qts_shap_interactions takes
                                the depth-first form; bit 2 (FP32), bit 3 (FP64):
                                qts_shap_interactions3 does */
  int64_t n_dfs_nodes;       /* internal nodes of the depth-first interactions form
                                (0 until its tables are built) */
  int64_t n_dfs_updates;     /* its pair updates per sample: the features split above
                                each internal node, summed */
  int64_t n_dfs_updates3;    /* its third-order updates per sample: pairs of those
                                features, summed over the internal nodes */
  int64_t n_value_prefix_kept;  /* first-order rows of at most 8 features: min(shared
                                   slots, 6) summed, the prefix products the walk over
                                   them keeps from the previous row */
  int64_t n_path_prefix_kept;   /* the same for the unmerged table */
} qts_info;

int qts_get_info(const qts_ensemble* ens, qts_info* out);

/* Copy the collapsed path table to caller host arrays, in path order:
 *   path_leaf[n_paths], path_len[n_paths], path_off[n_paths]   (int32)
 *   feat[n_elements] (int32), lo[n_elements], hi[n_elements] (float32),
 *   missing_ok[n_elements] (uint8), b[n_elements], one_minus_b[n_elements] (FP64).
 * Element e of a path follows iff lo <= x < hi (hi = NaN means no upper
 * bound), or x is NaN and missing_ok.  Any pointer may be NULL. */
int qts_export_paths(const qts_ensemble* ens, int32_t* path_leaf, int32_t* path_len,
                     int32_t* path_off, int32_t* feat, float* lo, float* hi,
                     uint8_t* missing_ok, double* b, double* one_minus_b);

/* The n-node Gauss-Legendre rule on [0,1] used by the kernels (Eq. 10), built
 * on the host in FP64 by the Golub-Welsch eigenvalue method: nodes t, 1-t
 * (computed separately, not by subtraction) and weights.  n in [1, 64]. */
int qts_gauss_legendre(int32_t n, double* t, double* one_minus_t, double* weight);

/* Shapley values phi[M, F] (row-major, F = n_features) of every sample.
 *   X            [M, ldx] float32 device rows (ldx >= F); NaN = missing.
 *   leaf_values  NULL, or [n_leaves] FP64 device array replacing the model's leaf
 *                values (phi is linear in them; used by the autograd wrapper).
 *   phi          [M, F] device output: float32 for QTS_FP32, double for QTS_FP64
 *                ([M, n_groups, F] for a grouped ensemble).
 * QTS_FP32 evaluates the quadrature in FP32 and accumulates across paths and
 * trees in FP64; QTS_FP64 does everything in FP64.  M = 0 is a no-op. */
int qts_shap_values(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                    const double* leaf_values, void* phi, qts_precision precision,
                    void* stream);

/* qts_shap_values for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, kernels and results, but the call's scratch (the
 * per-row slot-0 records and, for QTS_FP32 calls that need it, the FP64
 * accumulator of M * n_groups * F doubles) lives in a fixed 64 MiB device
 * array of the library instead of a per-call allocation.  Each GPU holds its
 * own copy of that array until the process ends.  A call whose scratch would
 * exceed it returns QTS_E_UNSUPPORTED without launching anything: split the
 * samples (the FP32 form of a 100-feature model takes up to about 80k samples
 * per call).  The call runs eagerly on `stream` (graph replay does not apply)
 * and allocates nothing.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (different streams or threads) race
 * and must be serialised by the caller. */
int qts_shap_values_noalloc(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                            const double* leaf_values, void* phi, qts_precision precision,
                            void* stream);

/* Pairwise interaction matrices Phi[M, F, F] (and optionally phi[M, F]; with
 * output groups [M, n_groups, F, F] and [M, n_groups, F]) with the
 * convention above.  Pair indices are the |S|=2 case of Theorem 1 and Eq. 9.
 * Output types follow `precision` as for qts_shap_values; phi may be NULL. */
int qts_shap_interactions(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                          const double* leaf_values, void* phi, void* Phi,
                          qts_precision precision, void* stream);

/* Third-order Shapley interaction indices: Theorem 1 with |S| = 3 and Eq. 9,
 * integrated with the 8-node rule of Eq. 10,
 *   SII_ijk = sum over paths with i, j, k among their unique features of
 *             val (o_i - b_i)(o_j - b_j)(o_k - b_k)
 *             * sum_m w_m prod_{l != i,j,k} (b_l (1 - t_m) + o_l t_m).
 *   out  [M, F(F-1)(F-2)/6] device array, float32 for QTS_FP32, double for
 *        QTS_FP64, packed: the triple of features i < j < k at
 *        k(k-1)(k-2)/6 + j(j-1)/2 + i (the index is symmetric in its three
 *        features; triples with a repeated feature are not stored).
 *        Overwritten.  With F < 3 there is nothing to write (out may be NULL).
 *   leaf_values, X, M, ldx, precision, stream as for qts_shap_values.
 * Accumulation is in FP64 throughout; the FP32 form allocates an FP64
 * accumulator of M * F(F-1)(F-2)/6 doubles on `stream` for the call (and the
 * depth-first form the y values of one sample batch), or, under graph
 * replay (qts_set_graph_replay), the call's graph owns them.
 * The traversal follows qts_set_pair_traversal: the path form, or Algorithm 1
 * taken to order 3 (section 5): along a path the product of three features'
 * ratios r = (o - b) / F changes only where one of them is split, by that
 * feature's change times the other two ratios, so with the walk's y_v of
 * qts_shap_interactions
 *   SII_{f j k} += sum_m y_v(t_m) r_j^v(t_m) r_k^v(t_m)
 * at each internal node v on feature f, for every pair {j, k} of the other
 * features split above v.  That form holds rows of at most 32 such features
 * (trees of depth up to 33); deeper ensembles keep the path form.  It adds
 * into the sample's tensor in LDS, in ranges of the largest feature, or,
 * where that takes more than four ranges (F above about 80), straight into
 * the output with FP64 atomics.
 * Errors: QTS_E_UNSUPPORTED in the path form when one feature's triples
 * (k(k-1)/2 of them) do not fit in LDS: F above 203 for rows of at most 8
 * features, above about 180 to 200 for longer rows (by row length and
 * precision).  The depth-first
 * form has no such limit: select it with QTS_PAIRS_DFS, or call qts_autotune
 * under QTS_PAIRS_AUTO, which takes it where the path form does not fit. */
int qts_shap_interactions3(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                           const double* leaf_values, void* out, qts_precision precision,
                           void* stream);

/* Adjoint of qts_shap_values with respect to the leaf values: phi is linear
 * in val(v) (Eq. 1, Eq. 10), so
 *   grad_leaf[v] = sum_s sum_{j on path(v)} grad_phi[s, f_j] (o_j - b_j)
 *                  * sum_m w_m prod_{k != j} (b_k (1 - t_m) + o_k t_m).
 *   grad_phi   [M, F] device array, float32 for QTS_FP32, double for QTS_FP64
 *              ([M, n_groups, F] for a grouped ensemble).
 *   grad_leaf  [n_leaves] FP64 device output (overwritten). */
int qts_shap_backward(const qts_ensemble* ens, const float* X, int64_t M, int64_t ldx,
                      const void* grad_phi, double* grad_leaf, qts_precision precision,
                      void* stream);

/* Launch-shape autotuner.  Times, with HIP events on `stream`, candidate
 * launch shapes on M_hint synthetic rows (uniform in [-3, 3), M_hint capped to
 * [64, 262144]; interactions on at most 256 of them) and keeps the fastest for
 * this ensemble and precision:
 *   first-order kernel, and separately the adjoint kernel (upstream
 *     gradient uniform in [-3, 3)), per length bucket: wavefronts per
 *     workgroup {4, 6, 8} x target work items {4096 .. 65536};
 *   interactions, per capacity class: largest path chunk {8192, 32768,
 *     131072} x least work items {1024, 4096}.
 * First-order and adjoint shapes are kept per node policy and tuned for the
 * policy in effect (qts_set_node_policy).
 * Synchronises `stream`; drops the ensemble's cached graphs.  Optional:
 * untuned ensembles use fixed defaults.  Not thread-safe against concurrent
 * compute calls on the same ensemble. */
int qts_autotune(qts_ensemble* ens, int64_t M_hint, qts_precision precision, void* stream);

/* Persistent autotune cache (process-wide; NULL or "" turns it off, the
 * default).  While set, qts_autotune looks up each bucket's and class's launch
 * shape in the text file at `path` before timing candidates, and appends the
 * shapes it times.  A key names everything the timing depends on: the
 * library's kernel sources, the device (architecture and compute units), the
 * kernel kind, precision and node policy, the feature and output counts, the
 * bucket or class (capacity, output group, rows) and the size class of
 * M_hint; a file that cannot be written still serves hits.  Lines are
 * "<key> -> a b"; later lines win. */
int qts_set_tune_cache(const char* path);
/* Cache lookups since the last qts_set_tune_cache: hits and misses. */
int qts_tune_cache_stats(int64_t* hits, int64_t* misses);

/* The launch shape in use (first order and adjoint: for the node policy in
 * effect): kind 0 = first-order bucket `index`, kind 2 =
 * adjoint bucket `index` (0..3 for lengths <= 8, 16, 32, 64) -> (*a, *b) =
 * (wavefronts per workgroup, target work items); kind 1 = interactions
 * capacity class `index` (0 .. n_pair_classes-1) -> (largest path chunk,
 * least work items). */
int qts_get_launch_shape(const qts_ensemble* ens, int32_t kind, qts_precision precision,
                         int32_t index, int32_t* a, int32_t* b);

/* Sibling merging for qts_shap_values (on by default).  Two leaves A, B that
 * are the two children of one node have the same collapsed feature set and
 * differ only in the element of the node's split feature L.  Their
 * polynomials of Eq. 7 (multiplied through by b) therefore share every factor
 * but L's, and since phi is linear in each path's polynomial,
 *   vA prod_j F^A_j(p) + vB prod_j F^B_j(p)
 *     = (vA F^A_L(p) + vB F^B_L(p)) prod_{j != L} F_j(p),
 * which is again linear in p in the L factor.  With merging on, the first-order
 * kernel walks one path per such pair, carrying that combined factor (built
 * in FP64 from the current leaf values) and a leaf value of 1: the same
 * result up to rounding, with about half the work on full trees.  The
 * interactions and adjoint calls always walk every path.  Changing the
 * setting drops the ensemble's cached graphs. */
int qts_set_sibling_merge(qts_ensemble* ens, int32_t enable);

/* Deterministic first-order and adjoint results (off by default).  phi and
 * grad_leaf are sums over paths and trees in FP64; with atomics their order,
 * and so their last bits, depend on scheduling.  While enabled:
 *   qts_shap_values (and qts_shap_values_noalloc) run one wavefront per
 *     workgroup and one launch per row chunk, in order, on the call's stream,
 *     each adding its tiles without atomics: every (sample, feature) has one
 *     writer per launch;
 *   qts_shap_backward stores each 64-sample block's leaf sums in a row of its
 *     own (every leaf belongs to one row of the table) and adds the rows in
 *     order (scratch of ceil(M / 64) * n_leaves doubles).
 * Results are then identical bit for bit from run to run on one device and
 * build, and equal the default mode's up to rounding.  The first-order call
 * runs several times slower (one wavefront per workgroup).  Interactions and
 * third-order calls are not affected.  Changing it drops the cached graphs. */
int qts_set_deterministic(qts_ensemble* ens, int32_t enable);

/* Allocation-failure injection, for testing the error paths of callers and of
 * the library.  after >= 0: the next `after` device allocations the library
 * makes (on any ensemble and thread: table uploads, call scratch, graph
 * scratch) succeed and every later one fails as if the device were out of
 * memory, so the call that needed it returns QTS_E_OOM; after < 0: off (the
 * default).  A failed call releases what it allocated, and the ensemble stays
 * usable; a failed qts_load_ensemble returns no ensemble. */
int qts_debug_fail_allocations(int64_t after);

/* Node count of every call.
 *   QTS_NODES_FIXED8 (default): the 8-node Gauss-Legendre rule for every path
 *     (section 5).
 *   QTS_NODES_EXACT: the fewest nodes that are exact where that is fewer than
 *     8.  An n-node rule integrates degree 2n - 1 exactly (Theorem 2); the
 *     order-s integrand of a path of d unique features has degree d - s.
 *     First order and adjoint: paths of at most 8 features use 4 nodes.
 *     Interactions: capacity classes 4, 8 and 12 use 2, 4 and 6 nodes (their
 *     first-order sums too).  Longer paths keep 8 nodes.  Results equal the
 *     8-node ones up to rounding.
 * Launch shapes are kept per policy.  Changing the policy drops the
 * ensemble's cached graphs. */
enum { QTS_NODES_FIXED8 = 0, QTS_NODES_EXACT = 1 };
int qts_set_node_policy(qts_ensemble* ens, int32_t policy);

/* Traversal of qts_shap_interactions.
 *   QTS_PAIRS_PATHS: every root-to-leaf path (or merged pair of
 *     sibling leaves) collapsed to its unique features; each adds its
 *     d(d-1)/2 pair terms (Theorem 1 with |S| = 2).
 *   QTS_PAIRS_DFS: Algorithm 1 at order 2 (section 5).  A depth-first walk of
 *     each tree carries, per sample and node t_m, the product of the factors
 *     of the features split above the current node and returns each
 *     subtree's summed polynomial H_u; at each internal node v on feature f
 *     the change of f's ratio r_f = (o_f - b_f) / F_f across each child edge
 *     (the telescoping update of Eq. 11) gives
 *       y_v(t_m) = w_m sum_u H_u(t_m) (r_f^u - r_f^v)(t_m),
 *     and the pair pass adds phi_f += sum_m y_v and, for every feature j
 *     split above v, SII_fj += sum_m y_v r_j^v: one update per (internal
 *     node, feature above it) instead of per pair of a path's features.  The
 *     samples go in batches whose y_v values fit 4 GiB of scratch.  Same
 *     results up to rounding, always with the 8-node rule.
 * Selecting QTS_PAIRS_DFS builds its tables on the current device (from the
 * tree arrays kept at load) the first time; QTS_E_UNSUPPORTED if its walk's
 * per-level stacks do not fit in LDS.  Changing it drops the cached graphs. */
/*   QTS_PAIRS_AUTO (default): the form qts_autotune finds faster on the
 *     ensemble, per precision (timed on one batch of its synthetic rows; kept
 *     in the autotune cache); the path form until the ensemble is tuned, and
 *     where the walk's stacks do not fit in LDS.  qts_autotune builds the
 *     depth-first tables on first use.
 * The setting also selects the form of qts_shap_interactions3 (chosen
 * separately by qts_autotune under QTS_PAIRS_AUTO). */
enum { QTS_PAIRS_PATHS = 0, QTS_PAIRS_DFS = 1, QTS_PAIRS_AUTO = 2 };
int qts_set_pair_traversal(qts_ensemble* ens, int32_t traversal);

/* HIP graph replay.  While enabled, each compute call on this ensemble
 * (qts_shap_values, qts_shap_interactions, qts_shap_interactions3,
 * qts_shap_backward) is captured once (on an internal stream, with its
 * per-bucket or per-class launches as parallel branches where the call has
 * them) into a graph keyed by (call kind, precision,
 * X, M, ldx, leaf values or grad_phi, output pointers, stream), and replayed
 * with hipGraphLaunch on the caller's stream on every later call with the same
 * key.  A graph owns its FP64 accumulators, so a replay allocates nothing.
 * The graphs contain kernel nodes only (zeroing is a kernel, not a memset).
 * At most 16 graphs are kept (least recently used evicted, after waiting for
 * its last launch on an event of the library's own, so the caller's stream
 * may be destroyed while its graphs stay cached).  The caller keeps the keyed buffers alive and at the same size
 * while their graph may replay; disabling drops every graph.  Calls of one
 * ensemble are serialised by the cache. */
int qts_set_graph_replay(qts_ensemble* ens, int32_t enable);

/* Measurement aid.  While enabled, each compute call records a HIP event pair
 * on its stream around the launches of its main kernel (kind 0: the values
 * kernel, 1: the interactions kernel, 2: the adjoint kernel, 3: the
 * third-order kernels of qts_shap_interactions3, zero-fill and narrowing
 * included), excluding the zero-fill and cast kernels around the others.  qts_kernel_timing_read waits for
 * the recorded events of one kind, returns their summed duration in
 * milliseconds and the number of calls since the last read, and clears them.
 * With graph replay on, the pair spans the whole replay (zero-fill and cast
 * included).  Not meant to be enabled while a HIP graph is being captured. */
int qts_set_kernel_timing(int32_t enable);
int qts_kernel_timing_read(int32_t kind, double* total_ms, int64_t* calls);

/* Text of the last error raised on the calling thread ("" if none). */
const char* qts_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QTREESHAP_H */
