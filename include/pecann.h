/*
 * pecann.h -- C ABI of libpecann.so, the MI355X (gfx950) hot path of PECANN's
 * density peaks clustering (Yu, Engels, Huang, Shun, arXiv 2312.03940).
 *
 * The calls follow the paper's statement of the problem (Alg. 2): build a graph
 * index over the point set (BuildIndex), find every point's k nearest neighbours
 * and its density (the Find-Knn and F_density loops), compute every point's
 * dependent point (ComputeDepPts, Alg. 3), then noise, centers and cluster labels
 * (the F_noise / F_center / union-find steps).  The dependent forest (dep, delta)
 * is returned so that a caller can re-cut the dendrogram (Sec. 1) by calling
 * pecann_cluster again.
 *
 * Conventions shared by every call
 *   - Device pointers: every array argument documented "device" is GPU memory
 *     owned by the caller (for example a torch tensor); the library allocates
 *     nothing and keeps no state between calls.
 *   - Streams: every call is asynchronous on `stream` (a hipStream_t; NULL is
 *     the null stream).  Outputs are valid once the stream has synchronised.
 *     Argument errors are returned synchronously before anything is launched;
 *     a launch failure returns PECANN_EHIP; a fault inside a kernel surfaces at
 *     the caller's next synchronisation.
 *   - Errors: no exception crosses the ABI.  On error the outputs are
 *     unspecified.  pecann_last_error() gives a thread-local description.
 *   - Workspace: calls that need scratch memory take (ws, ws_bytes); the
 *     matching *_workspace_size() gives the minimum.  ws must be 256-byte
 *     aligned.  A workspace may be reused across calls on the same stream.
 *   - Orders: every "closest"/"smallest" order is (distance, index) ascending.
 *     The density rank is the total order of (D_k, index) ascending, i.e. rho
 *     descending with ties to the lower index (Sec. 3, step 3).  A rank key is
 *     the 64-bit value (float bits of the squared L2 distance -- or of the
 *     cosine distance -- to the k-th neighbour) << 32 | index, so that a
 *     smaller key means a strictly higher density.
 *   - Determinism: identical inputs on the same device give identical outputs.
 */
#ifndef PECANN_H
#define PECANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PECANN_OK = 0,
  PECANN_EINVAL = 1,       /* an argument is out of range or misaligned */
  PECANN_EWORKSPACE = 2,   /* ws is NULL or smaller than *_workspace_size() */
  PECANN_EHIP = 3,         /* a HIP runtime call or launch failed */
  PECANN_EUNSUPPORTED = 4, /* valid but not supported combination */
  PECANN_ECHECK = 5        /* checked builds only (PECANN_CHECKED): a kernel found
                              a broken invariant; pecann_last_error() names it */
} pecann_status;

/* Element type of a row store. */
typedef enum {
  PECANN_F32 = 0,     /* IEEE float32 */
  PECANN_U8 = 1,      /* unsigned 8-bit integer */
  PECANN_BF16 = 2,    /* bfloat16, round-to-nearest-even from float32 */
  PECANN_FP8E4M3 = 3, /* OCP float8 e4m3 with a float32 scale per row */
  PECANN_MXFP6 = 4    /* search rows only: OCP MX FP6 e2m3 (blocks of 32 values
                         sharing a power-of-two scale) for the beam searches,
                         with an FP8E4M3 copy for the distance tiles */
} pecann_dtype;

/* Distance D(x, y) (Sec. 2.1; the paper's experiments use Euclidean). */
typedef enum {
  PECANN_L2 = 0,     /* sqrt(sum (x_t - y_t)^2) */
  PECANN_COSINE = 1  /* 1 - x.y / (|x| |y|) */
} pecann_metric;

typedef enum {
  PECANN_CENTER_PRODUCT = 0,    /* the n_c largest rho * delta (Sec. 4.2) */
  PECANN_CENTER_THRESHOLD = 1,  /* delta >= delta_min (Sec. 4.2) */
  PECANN_CENTER_GIVEN = 2       /* is_center is an input, e.g. from pecann_local_centers */
} pecann_center_mode;

/* Density functions (Sec. 4.2; appendix A). */
typedef enum {
  PECANN_DENSITY_KTH = 0,         /* 1 / D(x_i, k-th neighbour) */
  PECANN_DENSITY_NORMALIZED = 1,  /* rho_i k / sum_{j in N_i} rho_j, kth densities */
  PECANN_DENSITY_EXP_SUM = 2,     /* exp(-sum_{j in N_i} D(x_i, x_j)^2 / k) */
  PECANN_DENSITY_SUM_EXP = 3,     /* sum_{j in N_i} exp(-D(x_i, x_j)^2) / k */
  PECANN_DENSITY_SUM = 4          /* -sum_{j in N_i} D(x_i, x_j) */
} pecann_density_fn;

/* ---------------------------------------------------------------------------
 * Prepared point set.
 *
 * pecann_prepare_vectors converts the caller's rows once into a "prepared"
 * buffer, owned by the caller, that every later call reads:
 *   search rows  n rows of the search element type (F32, U8, BF16 or FP8E4M3),
 *                each padded with zeros to a multiple of 16 bytes (BF16: 64,
 *                FP8E4M3: 128 -- one matrix-core step of the search's scoring);
 *   rerank rows  n float32 rows padded to 16 bytes, present when the search
 *                type is BF16 or FP8E4M3 (used to re-score candidates so that
 *                every reported distance and every ordering is float32);
 *   row scale    n floats (FP8E4M3 only): row t of the search copy holds
 *                x_t / scale_t with scale_t = max_j |x_tj| / 448 for L2, and
 *                scale_t = 1 / 448 for every row under PECANN_COSINE (unit
 *                rows: one scale keeps e4m3's relative precision, and the
 *                searches need not gather a scale per candidate);
 *   row norms    n 32-bit squared norms of the search rows, and for BF16/FP8
 *                also of the float32 rerank rows (used when distances are
 *                formed from matrix-core dot products);
 *   for PECANN_COSINE every row is divided by its norm first, so that
 *   D = 1 - x.y on the prepared rows (a zero row stays zero: D = 1).
 * Only the sizes matter to the caller: pecann_prepared_bytes() gives the
 * buffer size for (n, d, metric, search type).
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t n;             /* number of points, 2 <= n < 2^31 */
  int32_t d;             /* dimensions, 1 <= d <= 4096 */
  int32_t metric;        /* pecann_metric */
  int32_t search_dtype;  /* pecann_dtype of the search rows */
  int32_t reserved;      /* must be 0 */
  const void *prep;      /* device: buffer written by pecann_prepare_vectors */
} pecann_dataset;

/* Bytes of the prepared buffer; 0 if the combination is invalid. */
size_t pecann_prepared_bytes(int64_t n, int32_t d, int32_t metric, int32_t search_dtype);

/* Convert the caller's rows x (device; n rows of d elements of x_dtype, F32 or
 * U8, consecutive rows x_row_stride elements apart) into the prepared buffer
 * `prep` (device, prep_bytes >= pecann_prepared_bytes()).  U8 search rows
 * require U8 input and the L2 metric (they are then an exact copy).
 * No distance computation happens here: this is the step that makes the
 * reduced-precision copies of the point set P (Sec. 2.1). */
pecann_status pecann_prepare_vectors(const void *x, int32_t x_dtype, int64_t x_row_stride,
                                     int64_t n, int32_t d, int32_t metric,
                                     int32_t search_dtype, void *prep, size_t prep_bytes,
                                     void *stream);

/* ---------------------------------------------------------------------------
 * Graph index: BuildIndex of Alg. 2 with the batched Vamana construction of
 * Sec. 3.2 / Sec. 4.1, in the two-pass schedule of DiskANN's Vamana (the
 * paper defers the construction details to it): pass 1 prunes with alpha = 1,
 * pass 2 with the given alpha (passes = 1: a single pass with the given alpha).
 *
 * Points are inserted in the order perm (device, n distinct int32 indices; NULL
 * means a permutation drawn from `seed` with SplitMix64-driven Fisher-Yates).
 * The first pass starts the graph with perm[0] alone, then inserts batches of
 * 1, 2, 4, ... points capped at max_batch; the second pass, with every point
 * already in the graph, re-inserts perm in batches of max_batch from the start.
 * max_batch = 0 selects max(floor(n / 50), 8192): the paper's 0.02 n, raised to
 * the number of concurrent searches that keeps all 256 CUs busy (the cap
 * leaves the construction's bounds unchanged, Sec. 4.1).  Every search of a
 * batch sees the graph as it was when the batch began.  The start set S of a batch is the first
 * min(num_starts, points in the graph) points of perm (the random multi-start
 * of Sec. 3.2).  For each point p of the batch: V_p = the points expanded by a
 * greedy beam search (Alg. 1, beam width L) for p from S, p excluded; when a
 * search expands more than visited_cap points, the visited_cap closest by
 * (D, index) are kept (the final beam and the closest of the rest);
 * Nout(p) = RobustPrune(p, V_p u Nout(p), alpha, R).  Then each target q
 * receives the batch's new in-edges not already present, in ascending source
 * index: appended if they fit in R, otherwise
 * Nout(q) = RobustPrune(q, Nout(q) u new, alpha, R).  RobustPrune is DiskANN's:
 * repeatedly keep the closest surviving candidate c* and drop every candidate
 * c with alpha * D(c*, c) <= D(p, c) (compared as alpha^2 * D^2 <= D^2 for L2).
 * Distances use the search rows.  Each D(p, v) to a pruned point is formed once
 * and reused: the search's value for the visited set, and for an adjacency
 * entry the value it was selected or appended with (a reverse edge p -> q
 * carries D(p, q) as D(q, p)); distances between candidates come from
 * matrix-core tiles.  On float rows the search's and the tiles' roundings of
 * one pair may differ in the last bits; on integer-valued rows both are exact.
 * The workspace holds, besides the round's batch state, one 8-byte key per
 * adjacency entry (n * R * 8 bytes) and one int32 per point.
 *
 * Output adj (device, n*R int32): row v holds Nout(v) in adj[v*R .. v*R+deg[v]),
 * the rest -1; deg (device, n int32).
 * Limits: 1 <= R <= 128, 1 <= L <= 1024, alpha >= 1, 1 <= num_starts <= 64,
 * max_batch >= 0, L <= visited_cap <= 2048, passes in {0 (= 2), 1, 2}.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t R;            /* degree bound */
  int32_t L;            /* build beam width */
  float alpha;          /* prune slack, >= 1 */
  int32_t num_starts;   /* random start points */
  int32_t max_batch;    /* batch size cap in points (0: max(n / 50, 8192)) */
  int32_t visited_cap;  /* candidates kept per insertion (0 = 2L) */
  int32_t passes;       /* 2 (default, 0 means 2): alpha = 1 then alpha; 1: alpha only */
  int32_t reserved;     /* must be 0 */
} pecann_build_params;

/* counters (device, may be NULL): 8 uint64 work tallies accumulated over the
 * call -- [0] search expansions, [1] neighbour ids read, [2] rows gathered by
 * the searches, [3] searches that expanded more than visited_cap points, [4] row reads of the forward prunes' 16 x 16 distance
 * tiles (32 per tile), [5] the same for the reverse prunes, [6] targets pruned,
 * [7] targets appended.  The caller zeroes
 * them; they measure the work that algorithmic-traffic figures are built on. */
size_t pecann_build_graph_workspace_size(const pecann_dataset *ds, const pecann_build_params *bp);
pecann_status pecann_build_graph(const pecann_dataset *ds, const pecann_build_params *bp,
                                 const int32_t *perm, uint64_t seed, int32_t *adj,
                                 int32_t *deg, uint64_t *counters, void *ws, size_t ws_bytes,
                                 void *stream);

/* ---------------------------------------------------------------------------
 * Second graph index: NN-descent (the PyNNDescent index that the paper's
 * framework offers beside Vamana, Sec. 4.1; the graph comparison of Sec. 6
 * prunes both with alpha).  The paper does not print the construction; this
 * is Dong, Charikar and Li's NN-descent in synchronous rounds:
 *   every point keeps K neighbours in (distance, index) order, each flagged
 *   new or old; point i's first list holds init[i][0..K), all new.
 *   A round: U_i = i's new entries and the K closest points whose list holds
 *   i as new; W_i = i's old entries and the K closest points holding i as
 *   old, minus U_i.  Every pair of U_i x U_i and U_i x W_i is proposed both
 *   ways; a point's next list is the K smallest of its list and its proposals
 *   (distinct ids) and an entry that was not in its list is new.  Rounds end
 *   after max_iters, or after the first round that leaves at most
 *   floor(delta * n * K) new entries.
 *   num_repeats runs (run r from init + r*n*K) are merged: the K smallest of
 *   the union of their final lists.
 *   Graph: Nout(i) = RobustPrune(i, list_i u rev_i, alpha, R) (the rule of
 *   pecann_build_graph) with rev_i the K closest points whose list holds i.
 * Distances come from matrix-core dot-product tiles of the search rows and
 * the stored norms; a pair gets the same measure bit for bit wherever it is
 * formed, so a point's list never holds an id twice.
 *
 *   init      device, num_repeats * n * K int32: K distinct ids other than the
 *             point, per repeat and point.  An id outside [0, n) or equal to
 *             the point is an empty entry; repeated ids give unspecified
 *             (memory-safe) results.
 *   adj, deg  device outputs laid out as for pecann_build_graph
 *   knn_idx   device n*K int32 or NULL: the final lists (-1 = empty entry)
 *   knn_dist  device n*K float or NULL: their distances (+inf = empty)
 *   rounds    device num_repeats int32 or NULL: rounds run by each repeat
 *   counters  device 4 uint64 or NULL (caller zeroes): [0] proposals written,
 *             [1] 16 x 16 join tiles, [2] proposal merges (targets), [3] row
 *             reads of the final prune's tiles (32 per tile)
 * The proposal buffer holds `chunk` worst-case joins (12 K^2 - 2 K proposals
 * each; 0: as many as fit 4 GiB); a round's joins run in passes that fill it
 * at the actual counts.  The result does not depend on the chunking; the
 * workspace grows with it.
 * Limits: 1 <= K <= 64, K <= n - 1, 1 <= R <= 128, alpha >= 1,
 * 0 <= max_iters <= 1000, delta >= 0, 1 <= num_repeats <= 16, chunk >= 0.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t K;            /* list length */
  int32_t R;            /* degree bound of the graph */
  float alpha;          /* prune slack, >= 1 */
  int32_t max_iters;    /* rounds per repeat */
  float delta;          /* stop level as a fraction of n * K */
  int32_t num_repeats;  /* independent runs merged */
  int32_t chunk;        /* local joins per proposal batch (0: automatic) */
  int32_t reserved;     /* must be 0 */
} pecann_nnd_params;

size_t pecann_build_graph_nndescent_workspace_size(const pecann_dataset *ds,
                                                   const pecann_nnd_params *np);
pecann_status pecann_build_graph_nndescent(const pecann_dataset *ds, const pecann_nnd_params *np,
                                           const int32_t *init, int32_t *adj, int32_t *deg,
                                           int32_t *knn_idx, float *knn_dist, int32_t *rounds,
                                           uint64_t *counters, void *ws, size_t ws_bytes,
                                           void *stream);

/* ---------------------------------------------------------------------------
 * k nearest neighbours and kth density (Alg. 2, Find-Knn and F_density loops;
 * Sec. 4.2 "kth density": rho_i = 1 / D(x_i, k-th neighbour)).
 *
 * With a graph (adj != NULL): for every point i a greedy beam search (Alg. 1)
 * with beam width L_search from S = {i}, i itself expanded first but never
 * occupying a beam slot nor returned (Sec. 3, step 2 starts the search at the
 * query point; its nearest neighbour is another point).  With BF16/FP8 search
 * rows the `rerank` closest beam entries are re-scored from float32 rows and
 * the k closest of them reported.  A search that returns fewer than k points
 * falls back to an exact search for that point (Sec. 4.1).
 * Without a graph (adj == NULL): exact brute force over all other points (the
 * paper's BruteForce index); distances always from float32 (or exact U8) rows.
 * From n >= 4096 on, the exact search runs as a matrix-core scan (float32 dot
 * products, or exact int8 ones on U8 rows) that keeps 128 candidates per
 * point, followed by a direct-difference re-score; a point whose k-th distance
 * is not separated from the dropped candidates by the scan's rounding bound is
 * searched again by the direct-difference kernel, so the result is the same.
 *
 * Outputs (device): knn_idx[n*k] int32 and knn_dist[n*k] float (distances D,
 * not squared), ascending; rho[n] float (+inf when D_k = 0); rank_key[n]
 * uint64 (see conventions).  counters (device, may be NULL, zeroed by the
 * caller): 4 uint64 tallies of the graph search -- [0] expansions, [1]
 * neighbour ids read, [2] rows gathered, [3] float32 rows re-scored.
 * Limits: 1 <= k <= min(n-1, 64); k <= L_search <= 1024; k <= rerank <= L_search.
 * ------------------------------------------------------------------------- */
/* exact != 0 sizes the workspace of the no-graph (exact) mode. */
size_t pecann_knn_density_workspace_size(const pecann_dataset *ds, int32_t k, int32_t L_search,
                                         int32_t exact);
pecann_status pecann_knn_density(const pecann_dataset *ds, const int32_t *adj,
                                 const int32_t *deg, int32_t R, int32_t k, int32_t L_search,
                                 int32_t rerank, int32_t *knn_idx, float *knn_dist,
                                 float *rho, uint64_t *rank_key, uint64_t *counters, void *ws,
                                 size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Dependent points: ComputeDepPts of Alg. 3 (Def. 1: the closest point of
 * strictly higher density, here strictly smaller rank key).
 *   1. DPBruteForce over each point's own kNN list (its distances are reused);
 *      the densest point gets dep = -1, delta = +inf and is skipped (Sec. 3.1);
 *   2. with a graph: rounds with k_dep = L_d, 2 L_d, 4 L_d, ... while more than
 *      `threshold` points are unfinished and k_dep <= min(kdep_cap, n-1):
 *      for each unfinished i, greedy beam search from S = {i} with beam
 *      max(k_dep, L_search), then DPBruteForce over the k_dep closest found;
 *   3. DPBruteForce over all of P for every point still unfinished (exact).
 * Without a graph (adj == NULL) step 2 is skipped: the exact instantiation.
 * Outputs (device): dep[n] int32 (-1 = none) and delta[n] float (D to dep,
 * +inf for none).  stats (device, may be NULL) receives int32 counts: [0] the
 * unfinished points after step 1, [1 + r] those after round r for r < 30,
 * [31] the points handled by step 3.
 * Limits: L_d > k, threshold >= 0, L_d <= kdep_cap <= 1024.
 * ------------------------------------------------------------------------- */
size_t pecann_dependent_search_workspace_size(const pecann_dataset *ds, int32_t kdep_cap,
                                              int32_t L_search);
pecann_status pecann_dependent_search(const pecann_dataset *ds, const int32_t *adj,
                                      const int32_t *deg, int32_t R, const uint64_t *rank_key,
                                      const int32_t *knn_idx, const float *knn_dist,
                                      int32_t k, int32_t L_d, int32_t L_search,
                                      int32_t threshold, int32_t kdep_cap, int32_t *dep,
                                      float *delta, int32_t *stats, void *ws,
                                      size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Noise, centers and labels (Alg. 2 after ComputeDepPts; Sec. 4.2).
 *   noise:   rho_i < rho_min (strict);
 *   centers: PECANN_CENTER_PRODUCT -- the n_c non-noise points with the
 *            largest gamma_i = rho_i * delta_i (float32 product; inf*0 counts
 *            as 0), ties to the lower index; PECANN_CENTER_THRESHOLD -- the
 *            non-noise points with delta_i >= delta_min; PECANN_CENTER_GIVEN --
 *            is_center is an input (e.g. pecann_local_centers), noise points
 *            are never centers;
 *   labels:  every non-noise, non-center point joins its dependent's cluster;
 *            labels[i] = index of the root reached along dep (a center, a
 *            noise point, or the point with dep = -1).
 * Inputs rho, dep, delta (device, n).  Outputs labels[n] int32, is_center[n]
 * uint8 (device; an input as well with PECANN_CENTER_GIVEN).  Limits:
 * 1 <= n_c <= n in product mode.
 * ------------------------------------------------------------------------- */
size_t pecann_cluster_workspace_size(int64_t n);
pecann_status pecann_cluster(int64_t n, const float *rho, const int32_t *dep,
                             const float *delta, int32_t center_mode, int32_t n_c,
                             float delta_min, float rho_min, int32_t *labels,
                             uint8_t *is_center, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Batches of independent instances (many clustering problems per call).
 *
 * A prepared point set may hold several independent instances: instance t
 * owns the points [offsets[t], offsets[t+1]).  The *_batched calls run each
 * step on every instance at once (one launch per step covers all of them)
 * and nothing crosses instances: graph edges, neighbours, dependent points,
 * centers and labels stay inside each instance, with global indices.  Each
 * instance's results equal those of the single-instance call applied to that
 * instance alone (its rows, its insertion order, its k and n_c).
 *   num_instances  1 <= num_instances <= 4096
 *   offsets        host, num_instances + 1 values: offsets[0] = 0, ascending,
 *                  offsets[num_instances] = n, every instance >= 2 points
 *   k              host, k of each instance (NULL: the call's k for all);
 *                  1 <= k[t] <= min(n_t - 1, k_max)
 *   n_c            host, center count of each instance in product mode (NULL:
 *                  the call's n_c for all); 1 <= n_c[t] <= n_t
 * The host arrays are read during the call only.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t num_instances;
  int32_t reserved;        /* must be 0 */
  const int64_t *offsets;
  const int32_t *k;
  const int32_t *n_c;
} pecann_instances;

/* pecann_build_graph for every instance.  perm (device, n int32, may be NULL):
 * perm[offsets[t] .. offsets[t+1]) is instance t's insertion order (global
 * indices of its own points); NULL: a seeded shuffle of each instance (seed
 * + t for instance t).  Each instance keeps its own batch schedule and cap
 * (max_batch, or max(n_t / 50, 8192)); a launch covers the next batch of every
 * instance, so the workspace grows with the sum of the caps. */
size_t pecann_build_graph_batched_workspace_size(const pecann_dataset *ds,
                                                 const pecann_build_params *bp,
                                                 const pecann_instances *inst);
pecann_status pecann_build_graph_batched(const pecann_dataset *ds, const pecann_build_params *bp,
                                         const pecann_instances *inst, const int32_t *perm,
                                         uint64_t seed, int32_t *adj, int32_t *deg,
                                         uint64_t *counters, void *ws, size_t ws_bytes,
                                         void *stream);

/* pecann_knn_density for every instance.  Rows of knn_idx / knn_dist have
 * stride k_max: row i holds point i's k[t] neighbours, then -1 / +inf.
 * L_search >= k_max, rerank in [k_max, L_search].  Without a graph each
 * instance is searched exactly (the matrix-core scan for instances of 4096
 * points or more). */
size_t pecann_knn_density_batched_workspace_size(const pecann_dataset *ds,
                                                 const pecann_instances *inst, int32_t k_max,
                                                 int32_t L_search, int32_t exact);
pecann_status pecann_knn_density_batched(const pecann_dataset *ds, const pecann_instances *inst,
                                         const int32_t *adj, const int32_t *deg, int32_t R,
                                         int32_t k_max, int32_t L_search, int32_t rerank,
                                         int32_t *knn_idx, float *knn_dist, float *rho,
                                         uint64_t *rank_key, uint64_t *counters, void *ws,
                                         size_t ws_bytes, void *stream);

/* pecann_dependent_search for every instance (kNN rows of stride k_max as
 * written by pecann_knn_density_batched).  The densest point of each instance
 * has dep = -1; an instance stops doubling on its own once at most
 * `threshold` of its points are unfinished or k_dep exceeds
 * min(kdep_cap, n_t - 1); the final brute force scans the point's instance.
 * stats counts points over all instances. */
size_t pecann_dependent_search_batched_workspace_size(const pecann_dataset *ds,
                                                      const pecann_instances *inst,
                                                      int32_t kdep_cap, int32_t L_search);
pecann_status pecann_dependent_search_batched(const pecann_dataset *ds,
                                              const pecann_instances *inst, const int32_t *adj,
                                              const int32_t *deg, int32_t R,
                                              const uint64_t *rank_key, const int32_t *knn_idx,
                                              const float *knn_dist, int32_t k_max, int32_t L_d,
                                              int32_t L_search, int32_t threshold,
                                              int32_t kdep_cap, int32_t *dep, float *delta,
                                              int32_t *stats, void *ws, size_t ws_bytes,
                                              void *stream);

/* pecann_cluster for every instance: the n_c[t] largest gamma of instance t
 * become its centers. */
size_t pecann_cluster_batched_workspace_size(int64_t n, const pecann_instances *inst);
pecann_status pecann_cluster_batched(int64_t n, const pecann_instances *inst, const float *rho,
                                     const int32_t *dep, const float *delta,
                                     int32_t center_mode, int32_t n_c, float delta_min,
                                     float rho_min, int32_t *labels, uint8_t *is_center,
                                     void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * pecann_cluster for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation and outputs as pecann_cluster, with no workspace
 * argument.  Its scratch (8 bytes per point and a few hundred bytes more) is a
 * fixed device array inside the library, one copy per GPU, held until the
 * process ends; the call itself allocates nothing.
 *   n        1 <= n <= 2,097,152 (2^21, the array's capacity); larger n
 *            returns PECANN_EINVAL
 *   others   as pecann_cluster (device pointers, asynchronous on stream)
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other host threads) race and give undefined outputs; calls
 * ordered on one stream are safe.  What must start at zero is cleared by each
 * call with a kernel (no memset node under capture).
 * ------------------------------------------------------------------------- */
pecann_status pecann_cluster_noalloc(int64_t n, const float *rho, const int32_t *dep,
                                     const float *delta, int32_t center_mode, int32_t n_c,
                                     float delta_min, float rho_min, int32_t *labels,
                                     uint8_t *is_center, void *stream);

/* ---------------------------------------------------------------------------
 * Other density functions (Sec. 4.2: normalized; appendix A: exp-sum, sum-exp,
 * sum; see pecann_density_fn) and the local center function (appendix A).
 *
 * pecann_density replaces rho and rank_key with those of another density
 * function, computed in float32 from the kNN lists that pecann_knn_density(_batched)
 * wrote (row stride k; rows of instance t hold k[t] neighbours when inst is
 * given, inst NULL: one instance with this k).  Rank key: (~ordered(rho) << 32)
 * | index, where ordered() maps a float to an unsigned integer of the same
 * order, so a smaller key is a strictly higher density with ties to the lower
 * index.  rho and rank_key may be the arrays written by pecann_knn_density (no
 * element is read after it is written).  PECANN_DENSITY_KTH writes rho =
 * 1 / D_k and leaves rank_key untouched: the kth keys are the ones
 * pecann_knn_density wrote, which order by the k-th neighbour's measure itself
 * (its reciprocal square root can round distinct measures to one value).  Densities of
 * duplicate points (D = 0) are +inf (kth, normalized numerators) and the
 * normalized density is then undefined.
 *
 * pecann_local_centers marks is_center[i] = 1 for the non-noise points
 * (rho_i >= rho_min) whose rank key is smaller than that of each of their k
 * nearest neighbours; pecann_cluster(_batched) with PECANN_CENTER_GIVEN then
 * labels the dependent forest from those centers.
 * ------------------------------------------------------------------------- */
size_t pecann_density_workspace_size(int64_t n, const pecann_instances *inst);
pecann_status pecann_density(int64_t n, const pecann_instances *inst, int32_t k,
                             int32_t density_fn, const int32_t *knn_idx, const float *knn_dist,
                             float *rho, uint64_t *rank_key, void *ws, size_t ws_bytes,
                             void *stream);
size_t pecann_local_centers_workspace_size(int64_t n, const pecann_instances *inst);
pecann_status pecann_local_centers(int64_t n, const pecann_instances *inst, int32_t k,
                                   const int32_t *knn_idx, const uint64_t *rank_key,
                                   const float *rho, float rho_min, uint8_t *is_center, void *ws,
                                   size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (host-side instrumentation, off by default).  While enabled,
 * every kernel the library launches from this thread is bracketed by a pair of
 * HIP events recorded on the launch stream, filed under its kernel family
 * ("search_build", "search_knn", "search_dep", "prune_forward",
 * "prune_reverse", "reverse_edges", "bf_knn", "bf_dep", "exact_mfma", "prepare",
 * "cluster", "nnd_join", "nnd_update", "nnd_lists", "nnd_prune", "other").
 * pecann_profile_enable(1) clears earlier records; enable(0) stops
 * recording.  pecann_profile_report synchronises the recorded events and
 * writes up to max_entries family totals into out; it returns the number
 * written, or -1 on a HIP error.  Events come from a pool the library keeps
 * for the life of the process.
 * ------------------------------------------------------------------------- */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} pecann_profile_entry;

pecann_status pecann_profile_enable(int32_t on);
int32_t pecann_profile_report(pecann_profile_entry *out, int32_t max_entries);

/* ---------------------------------------------------------------------------
 * Launch tuning.  Chosen by the package's autotuner, which times candidates
 * through these calls and keeps the winners in a JSON cache keyed by the
 * workload's shape.
 *   hash_bits_build   log2 visited-hash slots of build searches (0: the rule
 *                     of about 10 L or 20 L slots; else 10..13)
 *   hash_bits_search  the same for kNN and doubling-round searches (0: about
 *                     20 L slots; else 10..13)
 *   grid_per_cu       one-wave blocks per compute unit of the persistent
 *                     search, prune and join launches (0: 32; else 4..64)
 *   scorer            where the searches score BF16 / FP8 candidate rows:
 *                     0 the rule (matrix cores for FP8 rows of 512 bytes or
 *                     more, else vector units), 1 vector units, 2 matrix cores
 *   prune_steps       the RobustPrune distance tiles' row steps per memory
 *                     round trip (0: the rule, 4 for float32 rows, 2 for the
 *                     narrower ones; else 2 or 4): more loads in flight
 *                     against fewer waves per SIMD
 * Hash sizes, grid and prune_steps change speed only: every output of every call is the same,
 * byte for byte, under any valid setting (the visited hash may forget ids,
 * which costs repeated distance evaluations and nothing else, and every work
 * item's result is independent of which wave takes it).  The scorer changes
 * the rounding of the reduced-precision search measures (an FMA chain on the
 * vector units, the matrix cores' sums of a two-part query), so approximate
 * graphs and lists over BF16 / FP8 rows may differ between its values;
 * float32 and uint8 rows and the exact mode are not affected.
 * The setting belongs to the calling host thread (each thread starts with the
 * rules); it governs that thread's later calls.  NULL restores the rules.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t hash_bits_build;
  int32_t hash_bits_search;
  int32_t grid_per_cu;
  int32_t scorer;    /* 0 rule, 1 vector units, 2 matrix cores */
  int32_t prune_steps; /* 0 rule, 2 or 4 */
} pecann_tuning;

pecann_status pecann_set_tuning(const pecann_tuning *t);
pecann_status pecann_get_tuning(pecann_tuning *t);

/* ---------------------------------------------------------------------------
 * Measurement aid, not a step of the method: reads `bytes` of device memory at
 * `buf` `passes` times with 16-byte vector loads spread over every compute
 * unit (eight in flight per thread; non-temporal loads when passes = 1; pass
 * r gives each block the slice of block + r, so that repeated passes are not
 * served by the L2 that read the data last), asynchronously on `stream`, so
 * that a caller timing the call gets the
 * achievable read bandwidth -- of HBM for a buffer much larger than the 256 MB
 * Infinity Cache read once, of the cache for a smaller one read many times.
 * Roofline figures put the search kernels' algorithmic bandwidth beside it.
 *   buf     device, 16-byte aligned; bytes a positive multiple of 16
 *   passes  >= 1 full reads of the buffer
 *   key     any value; sink (device uint32) is or-ed with 1 only if the XOR
 *           fold of the data equals key, so nothing else is written
 * ------------------------------------------------------------------------- */
pecann_status pecann_read_probe(const void *buf, size_t bytes, int32_t passes, uint32_t key,
                                uint32_t *sink, void *stream);

const char *pecann_status_string(pecann_status s);
/* Thread-local description of the last error returned on this thread. */
const char *pecann_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PECANN_H */
