/*
 * dpc_oracle.c -- plain FP64 CPU oracle for the PECANN density-peaks hot path
 * (Yu, Engels, Huang, Shun, "PECANN: Parallel Efficient Clustering with
 * Graph-Based Approximate Nearest Neighbor Search", arXiv 2312.03940).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The GPU library never
 * includes, links or calls it; the two share no source, header or table.
 *
 * Every routine is either the plain definition written out (brute force, FP64,
 * distances by direct differences -- never the |x|^2+|y|^2-2x.y expansion) or,
 * where the method is itself a heuristic (greedy beam search, robust prune,
 * batched Vamana insertion, the doubling rounds), the algorithm's steps in the
 * paper's order.  Nothing is blocked, fused or reordered beyond that.
 * OpenMP is used only to run independent queries side by side; each query's
 * arithmetic is sequential and deterministic.
 *
 * Conventions (readings of the paper that it leaves open; each is listed with
 * its justification in the design notes):
 *   - a point's k nearest neighbours exclude the point itself (the worked
 *     example of Sec. 3, step 2, names c as the nearest neighbour of a);
 *   - every "closest"/"smallest" order is (distance, index) ascending, so
 *     distance ties go to the lower index;
 *   - the density rank is a total order: i ranks above j iff D_k(i) < D_k(j),
 *     or they are equal and i < j (Sec. 3, step 3, ranks b, c, a, d, f, e);
 *   - "higher density" in Def. 1 and Alg. 3 means "strictly higher in that
 *     rank" (the worked example's dependents c->b and f->d need this);
 *   - noise is rho < rho_min, strictly (Sec. 2.1 and Sec. 4.2);
 *   - labels are the index of the root reached along dependent pointers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { ODT_F32 = 0, ODT_U8 = 1 };
enum { OM_L2 = 0, OM_COSINE = 1 };

typedef struct {
  const void *x;   /* n rows, row i starts at element i*stride */
  int64_t n;
  int32_t d;
  int32_t dtype;   /* ODT_F32 or ODT_U8 */
  int32_t metric;  /* OM_L2 or OM_COSINE */
  int64_t stride;  /* elements between consecutive rows */
} opoints;

/* ------------------------------------------------------------------------ */
/* Distance D(x_i, x_j) (Sec. 2.1; Euclidean in the paper's experiments).    */
/* L2:     sqrt(sum_t (x_it - x_jt)^2), by direct differences.               */
/* cosine: 1 - x_i.x_j / (|x_i| |x_j|); a zero vector is at distance 1.      */
/* u8 rows are integers, so their squared L2 distance is summed exactly in   */
/* int64 before the single FP64 square root.                                 */
/* ------------------------------------------------------------------------ */
static double dist_l2_f32(const float *a, const float *b, int32_t d) {
  /* eight interleaved partial sums: a fixed, deterministic summation order */
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int32_t t = 0;
  for (; t + 8 <= d; t += 8)
    for (int u = 0; u < 8; ++u) {
      double e = (double)a[t + u] - (double)b[t + u];
      s[u] += e * e;
    }
  for (; t < d; ++t) {
    double e = (double)a[t] - (double)b[t];
    s[0] += e * e;
  }
  double tot = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  return sqrt(tot);
}

static double dist_l2_u8(const uint8_t *a, const uint8_t *b, int32_t d) {
  int64_t s = 0;
  for (int32_t t = 0; t < d; ++t) {
    int32_t e = (int32_t)a[t] - (int32_t)b[t];
    s += (int64_t)(e * e);
  }
  return sqrt((double)s);
}

static double dist_cos_f32(const float *a, const float *b, int32_t d) {
  double dot = 0, na = 0, nb = 0;
  for (int32_t t = 0; t < d; ++t) {
    double u = a[t], v = b[t];
    dot += u * v;
    na += u * u;
    nb += v * v;
  }
  if (na == 0.0 || nb == 0.0) return 1.0;
  return 1.0 - dot / (sqrt(na) * sqrt(nb));
}

static double dist_cos_u8(const uint8_t *a, const uint8_t *b, int32_t d) {
  int64_t dot = 0, na = 0, nb = 0;
  for (int32_t t = 0; t < d; ++t) {
    int64_t u = a[t], v = b[t];
    dot += u * v;
    na += u * u;
    nb += v * v;
  }
  if (na == 0 || nb == 0) return 1.0;
  return 1.0 - (double)dot / (sqrt((double)na) * sqrt((double)nb));
}

static double D(const opoints *P, int64_t i, int64_t j) {
  if (P->dtype == ODT_U8) {
    const uint8_t *x = (const uint8_t *)P->x;
    const uint8_t *a = x + i * P->stride, *b = x + j * P->stride;
    return P->metric == OM_L2 ? dist_l2_u8(a, b, P->d) : dist_cos_u8(a, b, P->d);
  } else {
    const float *x = (const float *)P->x;
    const float *a = x + i * P->stride, *b = x + j * P->stride;
    return P->metric == OM_L2 ? dist_l2_f32(a, b, P->d) : dist_cos_f32(a, b, P->d);
  }
}

double oracle_distance(const opoints *P, int64_t i, int64_t j) { return D(P, i, j); }

/* (distance, index) order */
static int before(double da, int64_t ia, double db, int64_t ib) {
  return da < db || (da == db && ia < ib);
}

/* ------------------------------------------------------------------------ */
/* Exact k nearest neighbours (Sec. 4.1 "Brute Force"): the k smallest       */
/* (D(i,j), j) over j != i, ascending.  Fills idx/dist rows of length k for  */
/* each query (queries==NULL means all points).  Returns 0, or -1 if k is    */
/* out of range.                                                             */
/* ------------------------------------------------------------------------ */
int oracle_knn(const opoints *P, const int64_t *queries, int64_t nq, int32_t k,
               int64_t *idx, double *dist) {
  if (k < 1 || k > P->n - 1) return -1;
  if (!queries) nq = P->n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t qq = 0; qq < nq; ++qq) {
    int64_t i = queries ? queries[qq] : qq;
    int64_t *bi = idx + qq * k;
    double *bd = dist + qq * k;
    int32_t m = 0; /* entries held, kept sorted ascending */
    for (int64_t j = 0; j < P->n; ++j) {
      if (j == i) continue;
      double dj = D(P, i, j);
      if (m == k && !before(dj, j, bd[k - 1], bi[k - 1])) continue;
      int32_t pos = (m < k) ? m++ : k - 1;
      while (pos > 0 && before(dj, j, bd[pos - 1], bi[pos - 1])) {
        bd[pos] = bd[pos - 1];
        bi[pos] = bi[pos - 1];
        --pos;
      }
      bd[pos] = dj;
      bi[pos] = j;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Density rank (Sec. 3 step 3): order points by (D_k, index) ascending,     */
/* i.e. by kth density rho = 1/D_k descending with ties to the lower index.  */
/* rank[i] = position of i in that order (0 = densest).                      */
/* ------------------------------------------------------------------------ */
static const double *g_sort_key; /* qsort has no context argument */
static int cmp_by_key_then_id(const void *a, const void *b) {
  int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
  double ki = g_sort_key[i], kj = g_sort_key[j];
  if (ki < kj) return -1;
  if (ki > kj) return 1;
  return (i > j) - (i < j);
}

void oracle_rank(int64_t n, const double *dk, int64_t *order, int64_t *rank) {
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  g_sort_key = dk;
  qsort(order, (size_t)n, sizeof(int64_t), cmp_by_key_then_id);
  g_sort_key = NULL;
  for (int64_t r = 0; r < n; ++r) rank[order[r]] = r;
}

/* ------------------------------------------------------------------------ */
/* Density functions from each point's k nearest neighbours N_i (ids and     */
/* distances D, row i of knn_idx / knn_dist):                                 */
/*   fn 0 kth (Sec. 4.2):        rho_i = 1 / D(x_i, k-th neighbour)          */
/*   fn 1 normalized (Sec. 4.2): rho_i * k / sum_{j in N_i} rho_j, with the  */
/*                               kth densities                               */
/*   fn 2 exp-sum (App. A):      exp(-sum_{j in N_i} D(x_i, x_j)^2 / k)      */
/*   fn 3 sum-exp (App. A):      sum_{j in N_i} exp(-D(x_i, x_j)^2) / k      */
/*   fn 4 sum (App. A):          -sum_{j in N_i} D(x_i, x_j)                 */
/* Returns 0, or -1 for an unknown function.                                 */
/* ------------------------------------------------------------------------ */
int oracle_density(int64_t n, int32_t k, int32_t fn, const int64_t *knn_idx,
                   const double *knn_dist, double *rho) {
  if (fn < 0 || fn > 4) return -1;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t *ids = knn_idx + i * k;
    const double *ds = knn_dist + i * k;
    double v = 0.0;
    if (fn == 0) {
      v = 1.0 / ds[k - 1];
    } else if (fn == 1) {
      double s = 0.0;
      for (int32_t t = 0; t < k; ++t) s += 1.0 / knn_dist[ids[t] * k + (k - 1)];
      v = (1.0 / ds[k - 1]) * k / s;
    } else if (fn == 2) {
      double s = 0.0;
      for (int32_t t = 0; t < k; ++t) s += ds[t] * ds[t];
      v = exp(-s / k);
    } else if (fn == 3) {
      double s = 0.0;
      for (int32_t t = 0; t < k; ++t) s += exp(-ds[t] * ds[t]);
      v = s / k;
    } else {
      double s = 0.0;
      for (int32_t t = 0; t < k; ++t) s += ds[t];
      v = -s;
    }
    rho[i] = v;
  }
  return 0;
}

/* Density order of any density function: rho descending, ties to the lower */
/* index (the kth density gives the same order as oracle_rank on D_k).       */
static int cmp_rho_desc_then_id(const void *a, const void *b) {
  int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
  double ri = g_sort_key[i], rj = g_sort_key[j];
  if (ri > rj) return -1;
  if (ri < rj) return 1;
  return (i > j) - (i < j);
}
void oracle_rank_density(int64_t n, const double *rho, int64_t *order, int64_t *rank) {
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  g_sort_key = rho;
  qsort(order, (size_t)n, sizeof(int64_t), cmp_rho_desc_then_id);
  g_sort_key = NULL;
  for (int64_t r = 0; r < n; ++r) rank[order[r]] = r;
}

/* Local centers (App. A, Local Center): the non-noise points ranked above  */
/* every one of their k nearest neighbours.                                  */
void oracle_local_centers(int64_t n, int32_t k, const int64_t *knn_idx, const int64_t *rank,
                          const double *rho, double rho_min, uint8_t *is_center) {
  for (int64_t i = 0; i < n; ++i) {
    int c = !(rho[i] < rho_min);
    for (int32_t t = 0; t < k && c; ++t) c = rank[i] < rank[knn_idx[i * k + t]];
    is_center[i] = (uint8_t)c;
  }
}

/* ------------------------------------------------------------------------ */
/* Exact dependent point (Def. 1): lambda_i = argmin over points ranked      */
/* strictly above i of (D(i,j), j); delta_i = D(i, lambda_i).  The top-ranked */
/* point has lambda = -1 and delta = +inf.                                   */
/* ------------------------------------------------------------------------ */
void oracle_dependent_exact(const opoints *P, const int64_t *rank,
                            const int64_t *queries, int64_t nq, int64_t *dep,
                            double *delta) {
  if (!queries) nq = P->n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t qq = 0; qq < nq; ++qq) {
    int64_t i = queries ? queries[qq] : qq;
    int64_t best = -1;
    double bd = INFINITY;
    for (int64_t j = 0; j < P->n; ++j) {
      if (rank[j] >= rank[i]) continue;
      double dj = D(P, i, j);
      if (best < 0 || before(dj, j, bd, best)) {
        best = j;
        bd = dj;
      }
    }
    dep[qq] = best;
    delta[qq] = best < 0 ? INFINITY : bd;
  }
}

/* ------------------------------------------------------------------------ */
/* Noise, centers and labels (Alg. 2, lines after ComputeDepPts; Sec. 4.2).  */
/*   noise:   rho_i < rho_min (strict);                                      */
/*   center_mode 0 (product): the n_c non-noise points with the largest      */
/*            gamma_i = rho_i * delta_i, ties to the lower index; a product   */
/*            that is not a number (inf * 0) counts as 0;                    */
/*   center_mode 1 (threshold): non-noise points with delta_i >= delta_min;  */
/*   center_mode 2 (given): is_center is an input (e.g. local centers);      */
/*            noise points are never centers;                                */
/*   labels:  non-noise, non-center points are joined with their dependent;  */
/*            every point is labelled with the index of the root it reaches  */
/*            (a center, a noise point, or the point with no dependent).     */
/* Returns 0, or -1 on bad arguments.                                        */
/* ------------------------------------------------------------------------ */
static const double *g_gamma;
static int cmp_gamma_desc(const void *a, const void *b) {
  int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
  double gi = g_gamma[i], gj = g_gamma[j];
  if (gi > gj) return -1;
  if (gi < gj) return 1;
  return (i > j) - (i < j);
}

int oracle_cluster(int64_t n, const double *rho, const int64_t *dep,
                   const double *delta, int32_t center_mode, int64_t n_c,
                   double delta_min, double rho_min, int64_t *labels,
                   uint8_t *is_center) {
  uint8_t *noise = (uint8_t *)calloc((size_t)n, 1);
  if (!noise) return -1;
  for (int64_t i = 0; i < n; ++i) {
    noise[i] = rho[i] < rho_min;
    if (center_mode == 2) is_center[i] = is_center[i] && !noise[i];
    else is_center[i] = 0;
  }
  if (center_mode == 2) {
    /* the caller's centers */
  } else if (center_mode == 0) {
    double *gamma = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!gamma || !cand) { free(noise); free(gamma); free(cand); return -1; }
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
      double g = rho[i] * delta[i];
      gamma[i] = isnan(g) ? 0.0 : g;
      if (!noise[i]) cand[m++] = i;
    }
    g_gamma = gamma;
    qsort(cand, (size_t)m, sizeof(int64_t), cmp_gamma_desc);
    g_gamma = NULL;
    for (int64_t r = 0; r < m && r < n_c; ++r) is_center[cand[r]] = 1;
    free(gamma);
    free(cand);
  } else {
    for (int64_t i = 0; i < n; ++i)
      if (!noise[i] && delta[i] >= delta_min) is_center[i] = 1;
  }
  /* union step: parent = dependent for joined points, self for roots */
  int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!parent) { free(noise); return -1; }
  for (int64_t i = 0; i < n; ++i)
    parent[i] = (noise[i] || is_center[i] || dep[i] < 0) ? i : dep[i];
  /* find step: walk to the root */
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = i, steps = 0;
    while (parent[r] != r) {
      r = parent[r];
      if (++steps > n) { free(parent); free(noise); return -1; } /* cycle */
    }
    labels[i] = r;
  }
  free(parent);
  free(noise);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Greedy beam search (Alg. 1) for query point q over a graph given as       */
/* adj[v*R + t] (t < deg[v]).  The beam keeps the L closest (D, index)        */
/* entries; each step expands the closest unexpanded beam entry, adds its     */
/* out-neighbours to the beam and truncates.  Returns the k closest of beam  */
/* and visited set.  Point `excl` (normally q itself, or -1) may serve as a  */
/* start and is expanded, but never takes a beam slot and is never returned: */
/* the worked example of Sec. 3.1 (round 1 of d finds {e, f} with k_dep = 2) */
/* holds only with the query excluded from its own beam.                     */
/* Optionally records the visited set (expanded points) in expansion order.  */
/* Returns the number of results written (<= k), or -1 on allocation error.  */
/* ------------------------------------------------------------------------ */
typedef struct { double d; int64_t id; } cand_t;

static int64_t add_to_beam(cand_t *beam, int64_t m, double d, int64_t id) {
  /* sorted insert; caller guarantees capacity and non-membership */
  int64_t pos = m;
  while (pos > 0 && before(d, id, beam[pos - 1].d, beam[pos - 1].id)) {
    beam[pos] = beam[pos - 1];
    --pos;
  }
  beam[pos].d = d;
  beam[pos].id = id;
  return m + 1;
}

int32_t oracle_greedy_search(const opoints *P, const int32_t *adj,
                             const int32_t *deg, int32_t R, int64_t q,
                             int64_t excl, const int64_t *starts, int32_t ns,
                             int32_t L, int32_t k, int64_t *out_ids,
                             double *out_d, int64_t *vis_ids, double *vis_d,
                             int32_t max_vis, int32_t *n_vis) {
  int64_t n = P->n;
  uint8_t *in_beam = (uint8_t *)calloc((size_t)n, 1);
  uint8_t *visited = (uint8_t *)calloc((size_t)n, 1);
  cand_t *beam = (cand_t *)malloc(sizeof(cand_t) * (size_t)(L + R + ns + 1));
  /* visited list: expanded points with their distances, expansion order */
  cand_t *vlist = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n + 1));
  if (!in_beam || !visited || !beam || !vlist) {
    free(in_beam); free(visited); free(beam); free(vlist);
    return -1;
  }
  int64_t m = 0, nv = 0;

  /* L <- S.  The excluded point, if a start, is expanded at once. */
  int64_t pending_excl = -1;
  for (int32_t s = 0; s < ns; ++s) {
    int64_t v = starts[s];
    if (v == excl) { pending_excl = v; continue; }
    if (in_beam[v]) continue;
    in_beam[v] = 1;
    m = add_to_beam(beam, m, D(P, q, v), v);
  }
  if (m > L) { for (int64_t t = L; t < m; ++t) in_beam[beam[t].id] = 0; m = L; }

  for (;;) {
    int64_t pstar;
    double pd;
    if (pending_excl >= 0) {
      pstar = pending_excl;
      pd = 0.0;
      pending_excl = -1;
    } else {
      /* p* <- closest beam entry not yet visited */
      int64_t t = 0;
      while (t < m && visited[beam[t].id]) ++t;
      if (t == m) break;
      pstar = beam[t].id;
      pd = beam[t].d;
    }
    /* L <- L u Nout(p*) */
    for (int32_t e = 0; e < deg[pstar]; ++e) {
      int64_t v = adj[pstar * (int64_t)R + e];
      if (v < 0 || v == excl || in_beam[v]) continue;
      in_beam[v] = 1;
      m = add_to_beam(beam, m, D(P, q, v), v);
    }
    /* V <- V u {p*} */
    visited[pstar] = 1;
    if (pstar != excl) { vlist[nv].d = pd; vlist[nv].id = pstar; ++nv; }
    /* keep the L closest */
    if (m > L) {
      for (int64_t t = L; t < m; ++t) in_beam[beam[t].id] = 0;
      m = L;
    }
  }

  /* k closest of L u V (V entries not in L lie beyond every beam entry) */
  int32_t cnt = 0;
  {
    cand_t *all = (cand_t *)malloc(sizeof(cand_t) * (size_t)(m + nv + 1));
    int64_t na = 0;
    for (int64_t t = 0; t < m; ++t) na = add_to_beam(all, na, beam[t].d, beam[t].id);
    for (int64_t t = 0; t < nv; ++t)
      if (!in_beam[vlist[t].id]) na = add_to_beam(all, na, vlist[t].d, vlist[t].id);
    for (int64_t t = 0; t < na && cnt < k; ++t) {
      out_ids[cnt] = all[t].id;
      out_d[cnt] = all[t].d;
      ++cnt;
    }
    free(all);
  }
  if (n_vis) {
    int32_t w = 0;
    for (int64_t t = 0; t < nv && w < max_vis; ++t, ++w) {
      if (vis_ids) vis_ids[w] = vlist[t].id;
      if (vis_d) vis_d[w] = vlist[t].d;
    }
    *n_vis = (int32_t)nv;
  }
  free(in_beam); free(visited); free(beam); free(vlist);
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* RobustPrune(p, V, alpha, R) of DiskANN (Sec. 3.2 defers to it):           */
/*   V <- V \ {p}, sorted by (D(p,v), v);                                    */
/*   repeatedly move the closest surviving v* to the output (stop at R) and  */
/*   drop every surviving v' with alpha * D(v*, v') <= D(p, v').             */
/* Duplicates in the candidate list are ignored.  Returns the out-degree.    */
/* ------------------------------------------------------------------------ */
int32_t oracle_robust_prune(const opoints *P, int64_t p, const int64_t *cand,
                            int32_t nc, double alpha, int32_t R,
                            int64_t *out) {
  cand_t *v = (cand_t *)malloc(sizeof(cand_t) * (size_t)(nc + 1));
  uint8_t *alive = (uint8_t *)malloc((size_t)nc + 1);
  if (!v || !alive) { free(v); free(alive); return -1; }
  int64_t m = 0;
  for (int32_t t = 0; t < nc; ++t) {
    int64_t c = cand[t];
    if (c == p || c < 0) continue;
    int dup = 0;
    for (int64_t u = 0; u < m; ++u) if (v[u].id == c) { dup = 1; break; }
    if (dup) continue;
    m = add_to_beam(v, m, D(P, p, c), c);
  }
  for (int64_t t = 0; t < m; ++t) alive[t] = 1;
  int32_t nout = 0;
  for (int64_t t = 0; t < m && nout < R; ++t) {
    if (!alive[t]) continue;
    int64_t vs = v[t].id;
    out[nout++] = vs;
    alive[t] = 0;
    if (nout == R) break;
    for (int64_t u = t + 1; u < m; ++u) {
      if (!alive[u]) continue;
      if (alpha * D(P, vs, v[u].id) <= v[u].d) alive[u] = 0;
    }
  }
  free(v);
  free(alive);
  return nout;
}

/* ------------------------------------------------------------------------ */
/* Batched Vamana construction (Sec. 3.2 and Sec. 4.1, after ParlayANN), with  */
/* the two-pass schedule of DiskANN's Vamana (first pass alpha = 1, then the    */
/* given alpha) when passes == 2:                                            */
/*   points are inserted in the order perm[]; in the first pass perm[0] alone  */
/*   starts the graph, then batches of size 1, 2, 4, ... capped at max_batch   */
/*   (0: floor(n / 50), the paper's 0.02 n); a later pass, every point now in  */
/*   the graph, re-inserts perm in batches of max_batch from perm[0] on.       */
/*   Every search of a batch sees the graph as  */
/*   it was when the batch began; the start set S is the first                */
/*   min(num_starts, inserted) points of perm;                                */
/*   for each point p of the batch: V_p = visited set of the greedy search for */
/*   p (beam L, p excluded), Nout(p) = RobustPrune(p, V_p u Nout(p), alpha, R); */
/*   then for each target q, the batch's new in-edges (sources in ascending     */
/*   index, those already present skipped) are appended to Nout(q) if they fit */
/*   in R, otherwise Nout(q) = RobustPrune(q, Nout(q) u new, alpha, R).        */
/* max_vis > 0 bounds V_p (the paper keeps all of it): when a search expands    */
/* more points, the max_vis closest by (D, index) are kept.                   */
/* batch_log (may be NULL) receives up to log_cap triples (pass, index in perm */
/* of the batch's first point, batch size), one per batch in the order run;    */
/* *n_log (may be NULL) the number of batches run.                            */
/* adj must hold n*R entries; unused slots are set to -1.  Returns 0 or -1.   */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t tgt, src; } edge_t;
static int cmp_edge(const void *a, const void *b) {
  const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
  if (x->tgt != y->tgt) return (x->tgt > y->tgt) - (x->tgt < y->tgt);
  return (x->src > y->src) - (x->src < y->src);
}

static int cmp_cand(const void *a, const void *b) {
  const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
  return before(x->d, x->id, y->d, y->id) ? -1 : (before(y->d, y->id, x->d, x->id) ? 1 : 0);
}

int oracle_vamana_build(const opoints *P, int32_t R, int32_t L, double alpha,
                        const int64_t *perm, int32_t num_starts, int64_t max_batch,
                        int32_t passes, int32_t max_vis, int64_t *batch_log,
                        int64_t log_cap, int64_t *n_log, int32_t *adj, int32_t *deg) {
  int64_t n = P->n;
  for (int64_t i = 0; i < n * (int64_t)R; ++i) adj[i] = -1;
  for (int64_t i = 0; i < n; ++i) deg[i] = 0;
  int64_t cap = max_batch > 0 ? max_batch : n / 50;
  if (cap < 1) cap = 1;
  int64_t *new_out = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap * R + 1));
  int32_t *new_deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
  edge_t *edges = (edge_t *)malloc(sizeof(edge_t) * (size_t)(cap * R + 1));
  int64_t *vis = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R + cap * R + 1));
  if (!new_out || !new_deg || !edges || !vis || !tmp) {
    free(new_out); free(new_deg); free(edges); free(vis); free(tmp);
    return -1;
  }
  int rc = 0;
  int64_t nlog = 0;
  for (int32_t pass = 0; pass < passes && rc == 0; ++pass) {
    const double a = (passes > 1 && pass == 0) ? 1.0 : alpha;
    /* first pass: perm[0] starts the graph unsearched, batches ramp up from 1;  */
    /* later passes re-insert every point in full batches                       */
    int64_t inserted = pass == 0 ? 1 : 0;
    int64_t bsize = pass == 0 ? 1 : cap;
    while (inserted < n) {
      int64_t b0 = inserted;
      int64_t nb = bsize < cap ? bsize : cap;
      if (nb > n - b0) nb = n - b0;
      int64_t in_graph = pass == 0 ? inserted : n;
      int32_t ns = (int32_t)(in_graph < num_starts ? in_graph : num_starts);
      int err = 0;
      if (batch_log && nlog < log_cap) {
        batch_log[3 * nlog + 0] = pass;
        batch_log[3 * nlog + 1] = b0;
        batch_log[3 * nlog + 2] = nb;
      }
      ++nlog;
      /* searches and forward prunes, all against the batch-start graph */
#pragma omp parallel for schedule(dynamic, 1)
      for (int64_t t = 0; t < nb; ++t) {
        int64_t p = perm[b0 + t];
        int64_t *myvis = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + R));
        double *myvd = (double *)malloc(sizeof(double) * (size_t)(n + 1));
        int64_t dummy_id;
        double dummy_d;
        int32_t nvis = 0;
        if (!myvis || !myvd) { free(myvis); free(myvd); err = 1; continue; }
        if (oracle_greedy_search(P, adj, deg, R, p, p, perm, ns, L, 0, &dummy_id,
                                 &dummy_d, myvis, myvd, (int32_t)n, &nvis) < 0) {
          err = 1;
        } else {
          if (max_vis > 0 && nvis > max_vis) {
            /* keep the max_vis closest expanded points */
            cand_t *cv = (cand_t *)malloc(sizeof(cand_t) * (size_t)nvis);
            if (!cv) { free(myvis); free(myvd); err = 1; continue; }
            for (int32_t t = 0; t < nvis; ++t) { cv[t].d = myvd[t]; cv[t].id = myvis[t]; }
            qsort(cv, (size_t)nvis, sizeof(cand_t), cmp_cand);
            for (int32_t t = 0; t < max_vis; ++t) myvis[t] = cv[t].id;
            nvis = max_vis;
            free(cv);
          }
          for (int32_t e = 0; e < deg[p]; ++e) myvis[nvis++] = adj[p * R + e];
          int32_t no = oracle_robust_prune(P, p, myvis, nvis, a, R, new_out + t * R);
          new_deg[t] = no < 0 ? 0 : no;
          if (no < 0) err = 1;
        }
        free(myvis);
        free(myvd);
      }
      if (err) { rc = -1; break; }
      /* write the batch's out-edges; gather reverse edges */
      int64_t ne = 0;
      for (int64_t t = 0; t < nb; ++t) {
        int64_t p = perm[b0 + t];
        for (int32_t e = 0; e < R; ++e)
          adj[p * R + e] = e < new_deg[t] ? (int32_t)new_out[t * R + e] : -1;
        deg[p] = new_deg[t];
        for (int32_t e = 0; e < new_deg[t]; ++e) {
          edges[ne].tgt = new_out[t * R + e];
          edges[ne].src = p;
          ++ne;
        }
      }
      qsort(edges, (size_t)ne, sizeof(edge_t), cmp_edge);
      /* per target: append the sources not yet present, or prune */
      int64_t e0 = 0;
      while (e0 < ne && rc == 0) {
        int64_t e1 = e0;
        int64_t q = edges[e0].tgt;
        while (e1 < ne && edges[e1].tgt == q) ++e1;
        int32_t nc = 0;
        for (int32_t e = 0; e < deg[q]; ++e) tmp[nc++] = adj[q * R + e];
        int32_t nold = nc;
        for (int64_t e = e0; e < e1; ++e) {
          int present = 0;
          for (int32_t u = 0; u < nold; ++u) if (tmp[u] == edges[e].src) { present = 1; break; }
          if (!present) tmp[nc++] = edges[e].src;
        }
        if (nc <= R) {
          for (int32_t e = nold; e < nc; ++e) adj[q * R + e] = (int32_t)tmp[e];
          deg[q] = nc;
        } else {
          int32_t no = oracle_robust_prune(P, q, tmp, nc, a, R, vis);
          if (no < 0) { rc = -1; break; }
          for (int32_t e = 0; e < R; ++e) adj[q * R + e] = e < no ? (int32_t)vis[e] : -1;
          deg[q] = no;
        }
        e0 = e1;
      }
      inserted += nb;
      if (bsize < cap) bsize *= 2; /* stop doubling at the cap */
    }
  }
  free(new_out); free(new_deg); free(edges); free(vis); free(tmp);
  if (n_log) *n_log = nlog;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* NN-descent graph: the PyNNDescent index the framework offers beside        */
/* Vamana (Sec. 4.1; the graph comparison of Sec. 6 prunes both with alpha). */
/* The paper does not print the construction; this is Dong, Charikar and     */
/* Li's NN-descent in synchronous rounds:                                    */
/*   every point i keeps a list of K neighbours ordered by (D, index), each  */
/*   flagged new or old; the first list holds init[i][0..K) (K distinct ids  */
/*   other than i, drawn by the caller), all new.                            */
/*   A round: new_i / old_i are the new / old entries of list i (all count   */
/*   as old afterwards); rnew_i is the K smallest (D(i,j), j) over the j     */
/*   whose list holds i flagged new, rold_i the same over old entries;       */
/*   U_i = new_i u rnew_i, W_i = (old_i u rold_i) minus U_i.  The local join */
/*   of i proposes v to u and u to v for every pair of distinct u, v in U_i  */
/*   and for every u in U_i with v in W_i.  The next list of u is the K      */
/*   smallest (D, index) of its list and its proposals, ids distinct; an     */
/*   entry whose id was not in the list before the round is flagged new.     */
/*   Rounds stop after max_iters, or after the first round whose lists end   */
/*   with at most floor(delta * n * K) new entries.                          */
/* num_repeats runs start from init[r]; their final lists are merged (the K  */
/* smallest of the union).  Graph: Nout(i) = RobustPrune(i, list_i u rev_i,  */
/* alpha, R) with rev_i the K smallest (D(i,j), j) over j whose list holds i. */
/* Outputs adj/deg, the final lists (ids, distances) and the rounds run by   */
/* each repeat.  Returns 0, or -1 (bad init or allocation failure).          */
/* ------------------------------------------------------------------------ */

/* Offer (d, id) to the sorted list l[0..*m) of capacity K: ignored if the id */
/* is present or the list is full of smaller entries; else inserted in order  */
/* (the largest entry of a full list leaves).  Returns 1 if inserted.         */
static int nnd_offer(cand_t *l, uint8_t *fl, int32_t *m, int32_t K, double d, int64_t id,
                     uint8_t flag) {
  for (int32_t t = 0; t < *m; ++t)
    if (l[t].id == id) return 0;
  if (*m == K && !before(d, id, l[K - 1].d, l[K - 1].id)) return 0;
  int32_t pos = *m < K ? *m : K - 1;
  while (pos > 0 && before(d, id, l[pos - 1].d, l[pos - 1].id)) {
    l[pos] = l[pos - 1];
    if (fl) fl[pos] = fl[pos - 1];
    --pos;
  }
  l[pos].d = d;
  l[pos].id = id;
  if (fl) fl[pos] = flag;
  if (*m < K) ++*m;
  return 1;
}

static int nnd_contains(const int64_t *a, int32_t m, int64_t id) {
  for (int32_t t = 0; t < m; ++t)
    if (a[t] == id) return 1;
  return 0;
}

/* One repeat: lists (n*K entries, counts cnt) from init; returns rounds run. */
static int32_t nnd_descend(const opoints *P, int32_t K, int32_t max_iters, double delta,
                           const int64_t *init, cand_t *list, uint8_t *flag, int32_t *cnt,
                           cand_t *nxt, uint8_t *nflag, int32_t *ncnt, cand_t *rnew,
                           int32_t *rnew_m, cand_t *rold, int32_t *rold_m, int64_t *U,
                           int64_t *W) {
  const int64_t n = P->n;
  for (int64_t i = 0; i < n; ++i) {
    cnt[i] = 0;
    for (int32_t t = 0; t < K; ++t) {
      int64_t j = init[i * K + t];
      nnd_offer(list + i * K, flag + i * K, cnt + i, K, D(P, i, j), j, 1);
    }
  }
  const double thr = floor(delta * (double)n * (double)K);
  int32_t rounds = 0;
  for (int32_t it = 0; it < max_iters; ++it) {
    /* reverse lists of the new and of the old entries */
    for (int64_t i = 0; i < n; ++i) rnew_m[i] = rold_m[i] = 0;
    for (int64_t j = 0; j < n; ++j)
      for (int32_t t = 0; t < cnt[j]; ++t) {
        const int64_t i = list[j * K + t].id;
        if (flag[j * K + t])
          nnd_offer(rnew + i * K, NULL, rnew_m + i, K, list[j * K + t].d, j, 0);
        else
          nnd_offer(rold + i * K, NULL, rold_m + i, K, list[j * K + t].d, j, 0);
      }
    /* next lists start as the current ones, every entry old */
    for (int64_t i = 0; i < n; ++i) {
      ncnt[i] = cnt[i];
      for (int32_t t = 0; t < cnt[i]; ++t) {
        nxt[i * K + t] = list[i * K + t];
        nflag[i * K + t] = 0;
      }
    }
    /* local joins */
    for (int64_t i = 0; i < n; ++i) {
      int32_t nu = 0, nw = 0;
      for (int32_t t = 0; t < cnt[i]; ++t)
        if (flag[i * K + t] && !nnd_contains(U, nu, list[i * K + t].id)) U[nu++] = list[i * K + t].id;
      for (int32_t t = 0; t < rnew_m[i]; ++t)
        if (!nnd_contains(U, nu, rnew[i * K + t].id)) U[nu++] = rnew[i * K + t].id;
      for (int32_t t = 0; t < cnt[i]; ++t) {
        const int64_t v = list[i * K + t].id;
        if (!flag[i * K + t] && !nnd_contains(U, nu, v) && !nnd_contains(W, nw, v)) W[nw++] = v;
      }
      for (int32_t t = 0; t < rold_m[i]; ++t) {
        const int64_t v = rold[i * K + t].id;
        if (!nnd_contains(U, nu, v) && !nnd_contains(W, nw, v)) W[nw++] = v;
      }
      for (int32_t a = 0; a < nu; ++a) {
        const int64_t u = U[a];
        for (int32_t b = a + 1; b < nu + nw; ++b) {
          const int64_t v = b < nu ? U[b] : W[b - nu];
          const double d = D(P, u, v);
          /* an id already in the list is present in the next list (or was */
          /* pushed out of it by closer ones), so whatever enters is new    */
          nnd_offer(nxt + u * K, nflag + u * K, ncnt + u, K, d, v, 1);
          nnd_offer(nxt + v * K, nflag + v * K, ncnt + v, K, d, u, 1);
        }
      }
    }
    int64_t updates = 0;
    for (int64_t i = 0; i < n; ++i) {
      cnt[i] = ncnt[i];
      for (int32_t t = 0; t < ncnt[i]; ++t) {
        list[i * K + t] = nxt[i * K + t];
        flag[i * K + t] = nflag[i * K + t];
        updates += nflag[i * K + t];
      }
    }
    ++rounds;
    if ((double)updates <= thr) break;
  }
  return rounds;
}

int oracle_nndescent(const opoints *P, int32_t K, int32_t R, double alpha, int32_t max_iters,
                     double delta, int32_t num_repeats, const int64_t *init, int32_t *adj,
                     int32_t *deg, int64_t *list_idx, double *list_dist, int32_t *rounds) {
  const int64_t n = P->n;
  if (K < 1 || K > n - 1 || R < 1 || num_repeats < 1) return -1;
  for (int32_t r = 0; r < num_repeats; ++r)
    for (int64_t i = 0; i < n; ++i)
      for (int32_t t = 0; t < K; ++t) {
        const int64_t j = init[((int64_t)r * n + i) * K + t];
        if (j < 0 || j >= n || j == i) return -1;
        for (int32_t u = 0; u < t; ++u)
          if (init[((int64_t)r * n + i) * K + u] == j) return -1;
      }
  const size_t nk = (size_t)(n * K);
  cand_t *list = malloc(sizeof(cand_t) * nk), *nxt = malloc(sizeof(cand_t) * nk);
  cand_t *rnew = malloc(sizeof(cand_t) * nk), *rold = malloc(sizeof(cand_t) * nk);
  cand_t *acc = malloc(sizeof(cand_t) * nk);
  uint8_t *flag = malloc(nk), *nflag = malloc(nk);
  int32_t *cnt = malloc(sizeof(int32_t) * (size_t)n), *ncnt = malloc(sizeof(int32_t) * (size_t)n);
  int32_t *rnew_m = malloc(sizeof(int32_t) * (size_t)n), *rold_m = malloc(sizeof(int32_t) * (size_t)n);
  int32_t *acc_m = malloc(sizeof(int32_t) * (size_t)n);
  int64_t *U = malloc(sizeof(int64_t) * (size_t)(4 * K + 2)), *W = malloc(sizeof(int64_t) * (size_t)(4 * K + 2));
  int64_t *cand = malloc(sizeof(int64_t) * (size_t)(2 * K + 1)), *out = malloc(sizeof(int64_t) * (size_t)(R + 1));
  int rc = 0;
  if (!list || !nxt || !rnew || !rold || !acc || !flag || !nflag || !cnt || !ncnt || !rnew_m ||
      !rold_m || !acc_m || !U || !W || !cand || !out) {
    rc = -1;
  } else {
    for (int64_t i = 0; i < n; ++i) acc_m[i] = 0;
    for (int32_t r = 0; r < num_repeats; ++r) {
      rounds[r] = nnd_descend(P, K, max_iters, delta, init + (int64_t)r * n * K, list, flag, cnt,
                              nxt, nflag, ncnt, rnew, rnew_m, rold, rold_m, U, W);
      for (int64_t i = 0; i < n; ++i)
        for (int32_t t = 0; t < cnt[i]; ++t)
          nnd_offer(acc + i * K, NULL, acc_m + i, K, list[i * K + t].d, list[i * K + t].id, 0);
    }
    /* reverse lists of the final lists, then the pruned graph */
    for (int64_t i = 0; i < n; ++i) rnew_m[i] = 0;
    for (int64_t j = 0; j < n; ++j)
      for (int32_t t = 0; t < acc_m[j]; ++t) {
        const int64_t i = acc[j * K + t].id;
        nnd_offer(rnew + i * K, NULL, rnew_m + i, K, acc[j * K + t].d, j, 0);
      }
    for (int64_t i = 0; i < n && rc == 0; ++i) {
      int32_t nc = 0;
      for (int32_t t = 0; t < acc_m[i]; ++t) cand[nc++] = acc[i * K + t].id;
      for (int32_t t = 0; t < rnew_m[i]; ++t) cand[nc++] = rnew[i * K + t].id;
      const int32_t no = oracle_robust_prune(P, i, cand, nc, alpha, R, out);
      if (no < 0) { rc = -1; break; }
      for (int32_t e = 0; e < R; ++e) adj[i * R + e] = e < no ? (int32_t)out[e] : -1;
      deg[i] = no;
      for (int32_t t = 0; t < K; ++t) {
        list_idx[i * K + t] = t < acc_m[i] ? acc[i * K + t].id : -1;
        list_dist[i * K + t] = t < acc_m[i] ? acc[i * K + t].d : INFINITY;
      }
    }
  }
  free(list); free(nxt); free(rnew); free(rold); free(acc); free(flag); free(nflag);
  free(cnt); free(ncnt); free(rnew_m); free(rold_m); free(acc_m); free(U); free(W);
  free(cand); free(out);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* ComputeDepPts (Alg. 3) over a graph index.                                */
/*   1. DPBruteForce over each point's kNN list N_i (the list's distances    */
/*      are recomputed here);                                               */
/*   2. U <- unfinished points, excluding the top-ranked point (Sec. 3.1:   */
/*      it has no dependent and is skipped);                                 */
/*   3. k_dep <- L_d; while |U| > threshold and k_dep <= kdep_cap:          */
/*        for i in U: C = FindKnn(i, k_dep) (Alg. 1 with S = {i}, beam width */
/*        max(k_dep, L_min), i excluded); lambda_i = DPBruteForce(i, C);     */
/*        k_dep <- 2 k_dep; U <- still unfinished;                           */
/*   4. DPBruteForce(i, P) for every i still in U.                           */
/* kdep_cap bounds the doubling (the loop of Alg. 3 is unbounded); points   */
/* left when it is reached go to step 4, which is exact.  With adj == NULL   */
/* step 3 is skipped (the paper's brute-force instantiation).               */
/* rounds_out (optional) receives |U| before each round and after the last. */
/* Returns the number of doubling rounds run, or -1.                         */
/* ------------------------------------------------------------------------ */
static int64_t dp_bruteforce_list(const opoints *P, int64_t i, const int64_t *rank,
                                  const int64_t *cand, int64_t nc, double *dout) {
  int64_t best = -1;
  double bd = INFINITY;
  for (int64_t t = 0; t < nc; ++t) {
    int64_t j = cand[t];
    if (j < 0 || rank[j] >= rank[i]) continue;
    double dj = D(P, i, j);
    if (best < 0 || before(dj, j, bd, best)) { best = j; bd = dj; }
  }
  *dout = bd;
  return best;
}

int32_t oracle_dependent_alg3(const opoints *P, const int32_t *adj,
                              const int32_t *deg, int32_t R,
                              const int64_t *rank, const int64_t *knn, int32_t k,
                              int32_t L_d, int64_t threshold, int32_t L_min,
                              int32_t kdep_cap, int64_t *dep, double *delta,
                              int64_t *rounds_out, int32_t max_rounds_out) {
  int64_t n = P->n;
  int64_t top = 0;
  for (int64_t i = 1; i < n; ++i) if (rank[i] < rank[top]) top = i;
  int64_t *U = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!U) return -1;
  int64_t nu = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (i == top) { dep[i] = -1; delta[i] = INFINITY; continue; }
    double d;
    int64_t l = dp_bruteforce_list(P, i, rank, knn + i * (int64_t)k, k, &d);
    dep[i] = l;
    delta[i] = l < 0 ? INFINITY : d;
    if (l < 0) U[nu++] = i;
  }
  int32_t rounds = 0;
  int64_t kdep = L_d;
  if (adj) {
    while (nu > threshold && kdep <= kdep_cap && kdep <= n - 1) {
      if (rounds_out && rounds < max_rounds_out) rounds_out[rounds] = nu;
      int err = 0;
      int32_t beam = (int32_t)(kdep > L_min ? kdep : L_min);
#pragma omp parallel for schedule(dynamic, 1)
      for (int64_t t = 0; t < nu; ++t) {
        int64_t i = U[t];
        int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)kdep);
        double *ds = (double *)malloc(sizeof(double) * (size_t)kdep);
        if (!ids || !ds) { err = 1; free(ids); free(ds); continue; }
        int64_t s = i;
        int32_t c = oracle_greedy_search(P, adj, deg, R, i, i, &s, 1, beam,
                                         (int32_t)kdep, ids, ds, NULL, NULL, 0, NULL);
        if (c < 0) err = 1;
        else {
          double d;
          int64_t l = dp_bruteforce_list(P, i, rank, ids, c, &d);
          if (l >= 0) { dep[i] = l; delta[i] = d; }
        }
        free(ids);
        free(ds);
      }
      if (err) { free(U); return -1; }
      int64_t w = 0;
      for (int64_t t = 0; t < nu; ++t) if (dep[U[t]] < 0) U[w++] = U[t];
      nu = w;
      kdep *= 2;
      ++rounds;
    }
  }
  if (rounds_out && rounds < max_rounds_out) rounds_out[rounds] = nu;
  /* final brute force over all of P */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nu; ++t) {
    int64_t i = U[t];
    /* DPBruteForce(x_i, P): every point is a candidate */
    int64_t best = -1;
    double bd = INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (rank[j] >= rank[i]) continue;
      double dj = D(P, i, j);
      if (best < 0 || before(dj, j, bd, best)) { best = j; bd = dj; }
    }
    dep[i] = best;
    delta[i] = best < 0 ? INFINITY : bd;
  }
  free(U);
  return rounds;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
