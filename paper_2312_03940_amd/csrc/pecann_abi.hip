// C ABI of libpecann.so: argument validation, prepared-buffer layout, workspace
// carving and the launch sequences of each call (host side only).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "kernels.hpp"
#include "pecann.h"

using namespace pecann;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

static pecann_status fail(pecann_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(PECANN_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Same, naming the build pass and batch.
#define HIP_TRY_BATCH(expr)                                                                     \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(PECANN_EHIP, "%s: %s (pass %d, batch [%lld, +%lld))", #expr,                 \
                  hipGetErrorString(e_), pass, (long long)inserted, (long long)nb);             \
  } while (0)

// A HIP error left pending by earlier, unrelated runtime calls of the process
// is cleared on entry, so that it is not reported as this call's failure.
static void clear_stale_error() { (void)hipGetLastError(); }

extern "C" const char *pecann_status_string(pecann_status s) {
  switch (s) {
    case PECANN_OK: return "ok";
    case PECANN_EINVAL: return "invalid argument";
    case PECANN_EWORKSPACE: return "workspace too small";
    case PECANN_EHIP: return "HIP error";
    case PECANN_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}
extern "C" const char *pecann_last_error(void) { return g_err; }

// ---------------------------------------------------------------------------
// Kernel timing: optional HIP-event brackets around every launch
// ---------------------------------------------------------------------------
namespace {
const char *const kFamilies[] = {"search_build", "search_knn", "search_dep", "prune_forward",
                                 "prune_reverse", "reverse_edges", "bf_knn", "bf_dep",
                                 "exact_mfma", "prepare", "cluster", "other"};
enum Family { F_SEARCH_BUILD, F_SEARCH_KNN, F_SEARCH_DEP, F_PRUNE_FWD, F_PRUNE_REV, F_REV,
              F_BF_KNN, F_BF_DEP, F_EXACT_MFMA, F_PREPARE, F_CLUSTER, F_OTHER, F_COUNT };
struct ProfRec { int fam; hipEvent_t a, b; };
struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void recycle() {
    for (auto &r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
    recs.clear();
  }
};
thread_local Profiler g_prof;

// Brackets one launch; a no-op unless timing is enabled.
struct ProfScope {
  hipStream_t s;
  int fam;
  hipEvent_t a = nullptr;
  ProfScope(int f, hipStream_t st) : s(st), fam(f) {
    if (!g_prof.on) return;
    a = g_prof.get();
    if (a) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = g_prof.get();
    if (!b) { g_prof.pool.push_back(a); return; }
    (void)hipEventRecord(b, s);
    g_prof.recs.push_back({fam, a, b});
  }
};
}  // namespace

#define PROF_CAT2(a, b) a##b
#define PROF_CAT(a, b) PROF_CAT2(a, b)
#define PROF(fam, s) ProfScope PROF_CAT(prof_scope_, __LINE__)(fam, s)

extern "C" pecann_status pecann_profile_enable(int32_t on) {
  if (on) g_prof.recycle();
  g_prof.on = on != 0;
  return PECANN_OK;
}

extern "C" int32_t pecann_profile_report(pecann_profile_entry *out, int32_t max_entries) {
  double tot[F_COUNT] = {0};
  int64_t cnt[F_COUNT] = {0};
  for (auto &r : g_prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return -1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -1;
    tot[r.fam] += ms;
    cnt[r.fam] += 1;
  }
  int32_t w = 0;
  for (int f = 0; f < F_COUNT && w < max_entries; ++f) {
    if (!cnt[f]) continue;
    memset(out[w].name, 0, sizeof out[w].name);
    strncpy(out[w].name, kFamilies[f], sizeof out[w].name - 1);
    out[w].launches = cnt[f];
    out[w].total_ms = tot[f];
    ++w;
  }
  return w;
}

// ---------------------------------------------------------------------------
// Device facts
// ---------------------------------------------------------------------------
static int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    cached[dev] = c;
  }
  return cached[dev];
}

// Persistent grids: enough one-wavefront blocks to fill every CU; surplus
// blocks find the work queue empty and leave.
static int persistent_grid(int64_t items) {
  int64_t g = (int64_t)cu_count() * 32;
  if (items < g) g = items;
  if (g < 1) g = 1;
  return (int)g;
}

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

namespace pecann {
int engine_shape(int32_t sdt, int32_t d) {
  const int bytes = sdt == PECANN_F32 ? 4 : sdt == PECANN_BF16 ? 2 : 1;
  const int nch = (d * bytes + 15) / 16;
  int S = 4;
  while (S < nch) S *= 2;
  return S;
}
}  // namespace pecann

// ---------------------------------------------------------------------------
// Prepared-buffer layout
// ---------------------------------------------------------------------------
struct Layout {
  size_t off_xs, xs_stride;  // bytes
  size_t off_xr, xr_stride;  // bytes offset, floats per row
  size_t off_scale;
  size_t off_sqn;
  size_t off_sqn_r;
  size_t total;
  bool has_xr, has_scale;
};

static size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static bool valid_dtype(int32_t t) { return t >= PECANN_F32 && t <= PECANN_FP8E4M3; }

static bool make_layout(int64_t n, int32_t d, int32_t metric, int32_t sdt, Layout *L) {
  if (n < 2 || n >= (int64_t)1 << 31 || d < 1 || d > 4096) return false;
  if (metric != PECANN_L2 && metric != PECANN_COSINE) return false;
  if (!valid_dtype(sdt)) return false;
  if (sdt == PECANN_U8 && metric != PECANN_L2) return false;
  const size_t bytes = sdt == PECANN_F32 ? 4 : sdt == PECANN_BF16 ? 2 : 1;
  L->off_xs = 0;
  L->xs_stride = up((size_t)d * bytes, 16);
  size_t off = up(L->xs_stride * (size_t)n, 256);
  L->has_xr = (sdt == PECANN_BF16 || sdt == PECANN_FP8E4M3);
  L->xr_stride = up((size_t)d, 4);
  L->off_xr = off;
  if (L->has_xr) off = up(off + L->xr_stride * 4 * (size_t)n, 256);
  L->has_scale = (sdt == PECANN_FP8E4M3);
  L->off_scale = off;
  if (L->has_scale) off = up(off + 4 * (size_t)n, 256);
  L->off_sqn = off;
  off = up(off + 4 * (size_t)n, 256);
  L->off_sqn_r = off;
  if (L->has_xr) off = up(off + 4 * (size_t)n, 256);
  L->total = off;
  return true;
}

static RowsDesc rows_of(const pecann_dataset *ds, const Layout &L) {
  RowsDesc r;
  const uint8_t *base = (const uint8_t *)ds->prep;
  r.xs = base + L.off_xs;
  r.xs_stride = (int64_t)L.xs_stride;
  r.scale = L.has_scale ? (const float *)(base + L.off_scale) : nullptr;
  r.xr = L.has_xr ? (const float *)(base + L.off_xr) : nullptr;
  r.xr_stride = (int64_t)L.xr_stride;
  r.sqn = (const uint32_t *)(base + L.off_sqn);
  r.sqn_r = L.has_xr ? (const float *)(base + L.off_sqn_r) : nullptr;
  r.nch = (int32_t)(L.xs_stride / 16);
  r.nch_r = (int32_t)(L.xr_stride / 4);
  r.d = ds->d;
  r.metric = ds->metric;
  return r;
}

static pecann_status check_dataset(const pecann_dataset *ds, Layout *L) {
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  if (ds->reserved != 0) return fail(PECANN_EINVAL, "dataset.reserved must be 0");
  if (!make_layout(ds->n, ds->d, ds->metric, ds->search_dtype, L))
    return fail(PECANN_EINVAL, "invalid dataset (n=%lld d=%d metric=%d search_dtype=%d)",
                (long long)ds->n, ds->d, ds->metric, ds->search_dtype);
  if (!ds->prep || !aligned(ds->prep, 256)) return fail(PECANN_EINVAL, "dataset.prep must be a 256-byte aligned device pointer");
  return PECANN_OK;
}

extern "C" size_t pecann_prepared_bytes(int64_t n, int32_t d, int32_t metric, int32_t sdt) {
  Layout L;
  return make_layout(n, d, metric, sdt, &L) ? L.total : 0;
}

extern "C" pecann_status pecann_prepare_vectors(const void *x, int32_t x_dtype, int64_t x_stride,
                                                int64_t n, int32_t d, int32_t metric, int32_t sdt,
                                                void *prep, size_t prep_bytes, void *stream) {
  clear_stale_error();
  Layout L;
  if (!make_layout(n, d, metric, sdt, &L))
    return fail(PECANN_EINVAL, "invalid (n=%lld, d=%d, metric=%d, search_dtype=%d)", (long long)n, d,
                metric, sdt);
  if (x_dtype != PECANN_F32 && x_dtype != PECANN_U8)
    return fail(PECANN_EINVAL, "x_dtype must be PECANN_F32 or PECANN_U8");
  if (sdt == PECANN_U8 && x_dtype != PECANN_U8)
    return fail(PECANN_EINVAL, "U8 search rows need U8 input");
  if (!x || x_stride < d) return fail(PECANN_EINVAL, "x is NULL or x_row_stride < d");
  if (!prep || !aligned(prep, 256)) return fail(PECANN_EINVAL, "prep must be 256-byte aligned");
  if (prep_bytes < L.total)
    return fail(PECANN_EWORKSPACE, "prep_bytes %zu < %zu", prep_bytes, L.total);
  pecann_dataset ds = {n, d, metric, sdt, 0, prep};
  RowsDesc r = rows_of(&ds, L);
  uint8_t *base = (uint8_t *)prep;
  PROF(F_PREPARE, (hipStream_t)stream);
  HIP_TRY(launch_prepare(x, x_dtype, x_stride, n, d, metric, sdt, r, base + L.off_xs,
                         L.has_xr ? (float *)(base + L.off_xr) : nullptr,
                         L.has_scale ? (float *)(base + L.off_scale) : nullptr,
                         (uint32_t *)(base + L.off_sqn),
                         L.has_xr ? (float *)(base + L.off_sqn_r) : nullptr, (hipStream_t)stream));
  return PECANN_OK;
}

// ---------------------------------------------------------------------------
// Workspace carving: the same code computes sizes (base == nullptr) and pointers.
// ---------------------------------------------------------------------------
struct Carver {
  uint8_t *base;
  size_t off = 0;
  explicit Carver(void *b) : base((uint8_t *)b) {}
  template <class T>
  T *take(size_t count) {
    size_t o = up(off, 256);
    off = o + sizeof(T) * count;
    return base ? (T *)(base + o) : nullptr;
  }
  size_t size() const { return up(off, 256); }
};

// Visited-hash size of a search with beam L: about 20 L slots (a search
// visits some 15 L distinct points), between 2^10 and 2^13.  The hash may
// forget (results do not change, only repeated distance evaluations), and a
// larger table costs occupancy: 4096 slots measured best at L = 128 and 200.
static int hash_bits_for(int L) {
  int b = 10;
  while (b < 13 && (1 << b) < 20 * L) ++b;
  return b;
}

// ---------------------------------------------------------------------------
// Graph build
// ---------------------------------------------------------------------------
static constexpr int kCapIn = 1024;  // new in-edges merged per target per batch

struct BuildWs {
  int32_t *perm, *ctr, *vis_count, *rcnt, *tidx, *tlist, *tord, *toff, *tcnt, *ticket, *seg;
  uint64_t *vis;
};

// Batch cap: the paper's 0.02 n, but never below 8192 concurrent searches (a
// wavefront each), which is what it takes to occupy 256 CUs.
static constexpr int64_t kMinGpuBatch = 8192;
// Reverse-edge targets with at most this many new sources in a batch (nearly
// all of them) are pruned by a launch whose LDS fits R + kLightIn candidates;
// the rest by a second launch sized for R + kCapIn.
static constexpr int32_t kLightIn = 64;
static constexpr int kHeavyGridPerCu = 4;
static int64_t batch_cap(int64_t n, int32_t max_batch) {
  int64_t c = max_batch > 0 ? (int64_t)max_batch : std::max<int64_t>(n / 50, kMinGpuBatch);
  if (c > n) c = n;
  return c < 1 ? 1 : c;
}

static void carve_build(Carver &c, int64_t n, int R, int64_t cap, int vcap, BuildWs *w) {
  w->perm = c.take<int32_t>((size_t)n);
  w->ctr = c.take<int32_t>(64);
  w->vis = c.take<uint64_t>((size_t)cap * vcap);
  w->vis_count = c.take<int32_t>((size_t)cap);
  w->rcnt = c.take<int32_t>((size_t)n);
  w->tidx = c.take<int32_t>((size_t)n);
  const size_t ce = (size_t)cap * R;
  w->tlist = c.take<int32_t>(ce);
  w->tord = c.take<int32_t>(ce);
  w->toff = c.take<int32_t>(ce);
  w->tcnt = c.take<int32_t>(ce);
  w->ticket = c.take<int32_t>(ce);
  w->seg = c.take<int32_t>(ce);
}

static int effective_vcap(const pecann_build_params *bp) {
  return bp->visited_cap > 0 ? bp->visited_cap : 2 * bp->L;
}

static pecann_status check_build(const pecann_dataset *ds, const pecann_build_params *bp) {
  if (!bp) return fail(PECANN_EINVAL, "build params are NULL");
  if (bp->R < 1 || bp->R > 128) return fail(PECANN_EINVAL, "R must be in [1, 128]");
  if (bp->L < 1 || bp->L > 1024) return fail(PECANN_EINVAL, "L must be in [1, 1024]");
  if (!(bp->alpha >= 1.0f)) return fail(PECANN_EINVAL, "alpha must be >= 1");
  if (bp->num_starts < 1 || bp->num_starts > 64) return fail(PECANN_EINVAL, "num_starts must be in [1, 64]");
  if (bp->max_batch < 0) return fail(PECANN_EINVAL, "max_batch must be >= 0");
  const int vcap = effective_vcap(bp);
  if (vcap < bp->L || vcap > 2048) return fail(PECANN_EINVAL, "visited_cap must be in [L, 2048]");
  if (bp->passes < 0 || bp->passes > 2) return fail(PECANN_EINVAL, "passes must be 0, 1 or 2");
  if (bp->reserved != 0) return fail(PECANN_EINVAL, "build params reserved field must be 0");
  (void)ds;
  return PECANN_OK;
}

extern "C" size_t pecann_build_graph_workspace_size(const pecann_dataset *ds, const pecann_build_params *bp) {
  Layout L;
  if (check_dataset(ds, &L) != PECANN_OK || check_build(ds, bp) != PECANN_OK) return 0;
  Carver c(nullptr);
  BuildWs w;
  carve_build(c, ds->n, bp->R, batch_cap(ds->n, bp->max_batch), effective_vcap(bp), &w);
  return c.size();
}

// SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) driving a Fisher-Yates shuffle.
static uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

extern "C" pecann_status pecann_build_graph(const pecann_dataset *ds, const pecann_build_params *bp,
                                            const int32_t *perm, uint64_t seed, int32_t *adj,
                                            int32_t *deg, uint64_t *counters, void *ws,
                                            size_t ws_bytes, void *stream) {
  clear_stale_error();
  Layout L;
  pecann_status st = check_dataset(ds, &L);
  if (st != PECANN_OK) return st;
  if ((st = check_build(ds, bp)) != PECANN_OK) return st;
  if (!adj || !deg) return fail(PECANN_EINVAL, "adj/deg are NULL");
  const int64_t n = ds->n;
  const int R = bp->R;
  const int vcap = effective_vcap(bp);
  const int64_t cap = batch_cap(n, bp->max_batch);
  Carver c0(nullptr);
  BuildWs w;
  carve_build(c0, n, R, cap, vcap, &w);
  if (!ws || ws_bytes < c0.size() || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", c0.size(), ws_bytes);
  Carver c(ws);
  carve_build(c, n, R, cap, vcap, &w);
  hipStream_t s = (hipStream_t)stream;
  const RowsDesc rows = rows_of(ds, L);
  const int dt = ds->search_dtype;
  const int S = engine_shape(dt, ds->d);

  const int32_t *order = perm;
  if (!order) {
    std::vector<int32_t> h((size_t)n);
    for (int64_t i = 0; i < n; ++i) h[i] = (int32_t)i;
    uint64_t sm = seed;
    for (int64_t i = n - 1; i > 0; --i) {
      const int64_t j = (int64_t)(splitmix64(sm) % (uint64_t)(i + 1));
      std::swap(h[i], h[j]);
    }
    HIP_TRY(hipMemcpyAsync(w.perm, h.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // h is pageable and about to go away
    order = w.perm;
  }

  HIP_TRY(launch_fill_i32(adj, -1, n * R, s));
  HIP_TRY(launch_fill_i32(deg, 0, n, s));
  HIP_TRY(launch_fill_i32(w.rcnt, 0, n, s));

  int32_t *head_search = w.ctr + 0, *head_pf = w.ctr + 1, *head_pr = w.ctr + 2;
  int32_t *ntargets = w.ctr + 3, *cursor = w.ctr + 4;
  int32_t *nlight = w.ctr + 5, *nheavy = w.ctr + 6, *head_ph = w.ctr + 7;
  int32_t *overflow = w.ctr + 8;
  HIP_TRY(launch_fill_i32(overflow, 0, 1, s));

  SearchParams sp = {};
  sp.rows = rows;
  sp.adj = adj;
  sp.deg = deg;
  sp.R = R;
  sp.n = (int32_t)n;
  sp.item_count = nullptr;
  sp.head = head_search;
  sp.starts = order;
  sp.L = bp->L;
  sp.hbits = hash_bits_for(bp->L);
  sp.mode = MODE_BUILD;
  sp.vis = w.vis;
  sp.vis_count = w.vis_count;
  sp.vcap = vcap;
  sp.counters = (unsigned long long *)counters;

  PruneParams pp = {};
  pp.rows = rows;
  pp.n = (int32_t)n;
  pp.R = R;
  pp.alpha = bp->alpha;
  pp.adj = adj;
  pp.deg = deg;
  pp.perm = order;
  pp.vis = w.vis;
  pp.vis_count = w.vis_count;
  pp.vcap = vcap;
  pp.tlist = w.tlist;
  pp.tord = w.tord;
  pp.nlight = nlight;
  pp.nheavy = nheavy;
  pp.ntargets = ntargets;
  pp.toff = w.toff;
  pp.tcnt = w.tcnt;
  pp.seg = w.seg;
  pp.rcnt = w.rcnt;
  pp.capin = kCapIn;
  pp.overflow = overflow;
  pp.counters = counters ? (unsigned long long *)counters + 4 : nullptr;

  const int passes = bp->passes == 0 ? 2 : bp->passes;
  for (int pass = 0; pass < passes; ++pass) {
    // DiskANN's schedule: alpha = 1 first, the given alpha last
    pp.alpha = (passes == 2 && pass == 0) ? 1.0f : bp->alpha;
    // the first pass starts the graph with perm[0] and ramps batches up from 1;
    // later passes re-insert every point in full batches
    int64_t inserted = pass == 0 ? 1 : 0, bsize = pass == 0 ? 1 : cap;
    while (inserted < n) {
      int64_t nb = std::min(bsize, cap);
      nb = std::min(nb, n - inserted);
      const int b0 = (int)inserted;
      const int64_t in_graph = pass == 0 ? inserted : n;
      HIP_TRY_BATCH(launch_fill_i32(w.ctr, 0, 8, s));
      sp.items = order + b0;
      sp.nitems = (int32_t)nb;
      sp.nstarts = (int32_t)std::min<int64_t>(bp->num_starts, in_graph);
      {
        PROF(F_SEARCH_BUILD, s);
        HIP_TRY_BATCH(launch_search(dt, S, sp, persistent_grid(nb), s));
      }
      pp.b0 = b0;
      pp.nb = (int32_t)nb;
      pp.head = head_pf;
      {
        PROF(F_PRUNE_FWD, s);
        HIP_TRY_BATCH(launch_prune_forward(dt, pp, persistent_grid(nb), s));
      }
      {
        PROF(F_REV, s);
        HIP_TRY_BATCH(launch_rev_count(adj, deg, order, b0, (int32_t)nb, R, w.rcnt, ntargets, w.tlist,
                                 w.tidx, w.ticket, s));
        HIP_TRY_BATCH(launch_rev_alloc(w.tlist, ntargets, w.rcnt, w.toff, w.tcnt, cursor, w.tord,
                                       nlight, nheavy, kLightIn, (int32_t)(nb * R), s));
        HIP_TRY_BATCH(launch_rev_scatter(adj, deg, order, b0, (int32_t)nb, R, w.tidx, w.toff, w.ticket,
                                   w.seg, s));
      }
      {
        PROF(F_PRUNE_REV, s);
        pp.heavy = 0;
        pp.head = head_pr;
        pp.capin = kLightIn;
        HIP_TRY_BATCH(launch_prune_reverse(dt, pp, persistent_grid(nb * R), s));
        pp.heavy = 1;
        pp.head = head_ph;
        pp.capin = kCapIn;
        const int heavy_grid = (int)std::min<int64_t>(nb * R, (int64_t)cu_count() * kHeavyGridPerCu);
        HIP_TRY_BATCH(launch_prune_reverse(dt, pp, heavy_grid, s));
      }
      inserted += nb;
      if (bsize < cap) bsize *= 2;  // stop doubling at the cap (no overflow)
    }
  }
  return PECANN_OK;
}

// ---------------------------------------------------------------------------
// kNN + density
// ---------------------------------------------------------------------------
// Exact kNN switches to the matrix-core scan from this many points on.
static constexpr int64_t kExactMfmaMin = 4096;

struct KnnWs {
  int32_t *ctr, *fb, *cand;
  float *thr, *nmax;
};
static void carve_knn(Carver &c, int64_t n, bool exact_mfma, KnnWs *w) {
  w->ctr = c.take<int32_t>(64);
  w->fb = c.take<int32_t>((size_t)n);
  w->nmax = c.take<float>(64);
  w->cand = exact_mfma ? c.take<int32_t>((size_t)n * 256) : nullptr;
  w->thr = exact_mfma ? c.take<float>((size_t)n) : nullptr;
}

extern "C" size_t pecann_knn_density_workspace_size(const pecann_dataset *ds, int32_t k,
                                                    int32_t L_search, int32_t exact) {
  Layout L;
  if (check_dataset(ds, &L) != PECANN_OK) return 0;
  (void)k; (void)L_search;
  Carver c(nullptr);
  KnnWs w;
  carve_knn(c, ds->n, exact != 0 && ds->n >= kExactMfmaMin, &w);
  return c.size();
}

extern "C" pecann_status pecann_knn_density(const pecann_dataset *ds, const int32_t *adj,
                                            const int32_t *deg, int32_t R, int32_t k,
                                            int32_t L_search, int32_t rerank, int32_t *knn_idx,
                                            float *knn_dist, float *rho, uint64_t *rank_key,
                                            uint64_t *counters, void *ws, size_t ws_bytes,
                                            void *stream) {
  clear_stale_error();
  Layout L;
  pecann_status st = check_dataset(ds, &L);
  if (st != PECANN_OK) return st;
  const int64_t n = ds->n;
  if (k < 1 || k > 64 || k > n - 1) return fail(PECANN_EINVAL, "k must be in [1, min(n-1, 64)]");
  if (!knn_idx || !knn_dist || !rho || !rank_key) return fail(PECANN_EINVAL, "output pointer is NULL");
  if (adj) {
    if (!deg) return fail(PECANN_EINVAL, "deg is NULL");
    if (R < 1 || R > 128) return fail(PECANN_EINVAL, "R must be in [1, 128]");
    if (L_search < k || L_search > 1024) return fail(PECANN_EINVAL, "L_search must be in [k, 1024]");
    const bool lp = ds->search_dtype == PECANN_BF16 || ds->search_dtype == PECANN_FP8E4M3;
    if (lp && (rerank < k || rerank > L_search))
      return fail(PECANN_EINVAL, "rerank must be in [k, L_search]");
  }
  const bool exact_mfma = !adj && n >= kExactMfmaMin;
  Carver c0(nullptr);
  KnnWs w;
  carve_knn(c0, n, exact_mfma, &w);
  if (!ws || ws_bytes < c0.size() || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", c0.size(), ws_bytes);
  Carver c(ws);
  carve_knn(c, n, exact_mfma, &w);
  int32_t *ctr = w.ctr, *fb = w.fb;
  hipStream_t s = (hipStream_t)stream;
  const RowsDesc rows = rows_of(ds, L);
  const int dt = ds->search_dtype;
  const int S = engine_shape(dt, ds->d);
  HIP_TRY(launch_fill_i32(ctr, 0, 4, s));

  BfKnnParams bp = {};
  bp.rows = rows;
  bp.n = (int32_t)n;
  bp.k = k;
  bp.knn_idx = knn_idx;
  bp.knn_dist = knn_dist;
  bp.rho = rho;
  bp.rank_key = rank_key;
  if (!adj && !exact_mfma) {
    bp.items = nullptr;
    bp.item_count = nullptr;
    bp.nitems = (int32_t)n;
    bp.head = ctr + 0;
    PROF(F_BF_KNN, s);
    HIP_TRY(launch_bf_knn(dt, S, bp, persistent_grid(n), s));
    return PECANN_OK;
  }
  if (exact_mfma) {
    ExactMfmaParams ep = {};
    ep.rows = rows;
    ep.n = (int32_t)n;
    ep.k = k;
    ep.cand = w.cand;
    ep.thr = w.thr;
    ep.nmax = w.nmax;
    ep.head = ctr + 0;
    ep.knn_idx = knn_idx;
    ep.knn_dist = knn_dist;
    ep.rho = rho;
    ep.rank_key = rank_key;
    ep.fb_list = fb;
    ep.fb_count = ctr + 1;
    {
      PROF(F_EXACT_MFMA, s);
      HIP_TRY(launch_exact_mfma(dt, S, ep, s));
    }
    bp.items = fb;
    bp.item_count = ctr + 1;
    bp.nitems = 0;
    bp.head = ctr + 2;
    PROF(F_BF_KNN, s);
    HIP_TRY(launch_bf_knn(dt, S, bp, cu_count() * 4, s));
    return PECANN_OK;
  }
  SearchParams sp = {};
  sp.rows = rows;
  sp.adj = adj;
  sp.deg = deg;
  sp.R = R;
  sp.n = (int32_t)n;
  sp.items = nullptr;
  sp.item_count = nullptr;
  sp.nitems = (int32_t)n;
  sp.head = ctr + 0;
  sp.starts = nullptr;
  sp.nstarts = 0;
  sp.L = L_search;
  sp.hbits = hash_bits_for(L_search);
  sp.mode = MODE_KNN;
  sp.rerank = rerank;
  sp.k = k;
  sp.knn_idx = knn_idx;
  sp.knn_dist = knn_dist;
  sp.rho = rho;
  sp.rank_key = rank_key;
  sp.fb_list = fb;
  sp.fb_count = ctr + 1;
  sp.counters = (unsigned long long *)counters;
  {
    PROF(F_SEARCH_KNN, s);
    HIP_TRY(launch_search(dt, S, sp, persistent_grid(n), s));
  }
  // too-few-results fallback: exact search for those queries
  bp.items = fb;
  bp.item_count = ctr + 1;
  bp.nitems = 0;
  bp.head = ctr + 2;
  PROF(F_BF_KNN, s);
  HIP_TRY(launch_bf_knn(dt, S, bp, cu_count() * 4, s));
  return PECANN_OK;
}

// ---------------------------------------------------------------------------
// Dependent points
// ---------------------------------------------------------------------------
struct DepWs {
  int32_t *ctr, *ucnt, *ua, *ub, *stats_tmp;
  uint64_t *minkey;
  unsigned long long *best;
};
static void carve_dep(Carver &c, int64_t n, DepWs *w) {
  w->ctr = c.take<int32_t>(64);
  w->ucnt = c.take<int32_t>(64);
  w->minkey = c.take<uint64_t>(1);
  w->ua = c.take<int32_t>((size_t)n);
  w->ub = c.take<int32_t>((size_t)n);
  w->best = c.take<unsigned long long>((size_t)n);
  w->stats_tmp = nullptr;
}

extern "C" size_t pecann_dependent_search_workspace_size(const pecann_dataset *ds, int32_t kdep_cap,
                                                         int32_t L_search) {
  Layout L;
  if (check_dataset(ds, &L) != PECANN_OK) return 0;
  (void)kdep_cap; (void)L_search;
  Carver c(nullptr);
  DepWs w;
  carve_dep(c, ds->n, &w);
  return c.size();
}

__global__ void dep_stats_kernel(const int32_t *ucnt, int nr, int32_t *stats) {
  const int t = threadIdx.x;
  if (t < 32) {
    int32_t v = 0;
    if (t == 0) v = ucnt[0];
    else if (t == 31) v = ucnt[nr];
    else if (t - 1 < nr) v = ucnt[t];
    stats[t] = v;
  }
}

extern "C" pecann_status pecann_dependent_search(const pecann_dataset *ds, const int32_t *adj,
                                                 const int32_t *deg, int32_t R,
                                                 const uint64_t *rank_key, const int32_t *knn_idx,
                                                 const float *knn_dist, int32_t k, int32_t L_d,
                                                 int32_t L_search, int32_t threshold,
                                                 int32_t kdep_cap, int32_t *dep, float *delta,
                                                 int32_t *stats, void *ws, size_t ws_bytes,
                                                 void *stream) {
  clear_stale_error();
  Layout L;
  pecann_status st = check_dataset(ds, &L);
  if (st != PECANN_OK) return st;
  const int64_t n = ds->n;
  if (k < 1 || k > 64 || k > n - 1) return fail(PECANN_EINVAL, "k must be in [1, min(n-1, 64)]");
  if (!rank_key || !knn_idx || !knn_dist || !dep || !delta) return fail(PECANN_EINVAL, "pointer is NULL");
  if (threshold < 0) return fail(PECANN_EINVAL, "threshold must be >= 0");
  if (adj) {
    if (!deg) return fail(PECANN_EINVAL, "deg is NULL");
    if (R < 1 || R > 128) return fail(PECANN_EINVAL, "R must be in [1, 128]");
    if (L_d <= k) return fail(PECANN_EINVAL, "L_d must be > k");
    if (kdep_cap < L_d || kdep_cap > 1024) return fail(PECANN_EINVAL, "kdep_cap must be in [L_d, 1024]");
    if (L_search < 1 || L_search > 1024) return fail(PECANN_EINVAL, "L_search must be in [1, 1024]");
  }
  Carver c0(nullptr);
  DepWs w;
  carve_dep(c0, n, &w);
  if (!ws || ws_bytes < c0.size() || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", c0.size(), ws_bytes);
  Carver c(ws);
  carve_dep(c, n, &w);
  hipStream_t s = (hipStream_t)stream;
  const RowsDesc rows = rows_of(ds, L);
  const int dt = ds->search_dtype;
  const int S = engine_shape(dt, ds->d);

  HIP_TRY(launch_fill_i32(w.ctr, 0, 64, s));
  HIP_TRY(launch_fill_i32(w.ucnt, 0, 64, s));
  HIP_TRY(launch_min_key(rank_key, n, w.minkey, s));
  HIP_TRY(launch_dep_in_knn(n, k, rank_key, w.minkey, knn_idx, knn_dist, dep, delta, w.ua, w.ucnt, s));

  int32_t *cur = w.ua, *nxt = w.ub;
  int nr = 0;
  if (adj) {
    const int64_t lim = std::min<int64_t>(kdep_cap, n - 1);
    for (int64_t kd = L_d; kd <= lim && nr < 30; kd *= 2, ++nr) {
      SearchParams sp = {};
      sp.rows = rows;
      sp.adj = adj;
      sp.deg = deg;
      sp.R = R;
      sp.n = (int32_t)n;
      sp.items = cur;
      sp.item_count = w.ucnt + nr;
      sp.nitems = 0;
      sp.head = w.ctr + nr;
      sp.starts = nullptr;
      sp.nstarts = 0;
      sp.L = (int32_t)std::max<int64_t>(kd, L_search);
      sp.hbits = hash_bits_for(sp.L);
      sp.mode = MODE_DEP;
      sp.rerank = (int32_t)kd;
      sp.kdep = (int32_t)kd;
      sp.key_in = rank_key;
      sp.dep = dep;
      sp.delta = delta;
      sp.u_out = nxt;
      sp.u_out_count = w.ucnt + nr + 1;
      sp.threshold = threshold;
      {
        PROF(F_SEARCH_DEP, s);
        HIP_TRY(launch_search(dt, S, sp, persistent_grid(n), s));
      }
      std::swap(cur, nxt);
    }
  }
  // final brute force over all of P for the points still unfinished
  HIP_TRY(launch_fill_u64((uint64_t *)w.best, ~0ull, n, s));
  BfDepParams bd = {};
  bd.rows = rows;
  bd.n = (int32_t)n;
  bd.ulist = cur;
  bd.ucount = w.ucnt + nr;
  bd.chunk = 4096;
  bd.nchunks = (int32_t)((n + bd.chunk - 1) / bd.chunk);
  bd.head = w.ctr + 40;
  bd.key = rank_key;
  bd.best = w.best;
  {
    PROF(F_BF_DEP, s);
    HIP_TRY(launch_bf_dep(dt, S, bd, persistent_grid(n * (int64_t)bd.nchunks), s));
  }
  HIP_TRY(launch_bf_dep_finalize(cur, w.ucnt + nr, w.best, ds->metric, dep, delta, (int32_t)n, s));
  if (stats) {
    hipLaunchKernelGGL(dep_stats_kernel, dim3(1), dim3(64), 0, s, w.ucnt, nr, stats);
    HIP_TRY(hipGetLastError());
  }
  return PECANN_OK;
}

// ---------------------------------------------------------------------------
// Cluster
// ---------------------------------------------------------------------------
extern "C" size_t pecann_cluster_workspace_size(int64_t n) {
  if (n < 1) return 0;
  Carver c(nullptr);
  c.take<uint64_t>((size_t)n);
  c.take<int32_t>(64);
  return c.size();
}

extern "C" pecann_status pecann_cluster(int64_t n, const float *rho, const int32_t *dep,
                                        const float *delta, int32_t center_mode, int32_t n_c,
                                        float delta_min, float rho_min, int32_t *labels,
                                        uint8_t *is_center, void *ws, size_t ws_bytes, void *stream) {
  clear_stale_error();
  if (n < 1 || n >= (int64_t)1 << 31) return fail(PECANN_EINVAL, "n out of range");
  if (!rho || !dep || !delta || !labels || !is_center) return fail(PECANN_EINVAL, "pointer is NULL");
  if (center_mode != PECANN_CENTER_PRODUCT && center_mode != PECANN_CENTER_THRESHOLD)
    return fail(PECANN_EINVAL, "center_mode");
  if (center_mode == PECANN_CENTER_PRODUCT && (n_c < 1 || n_c > n))
    return fail(PECANN_EINVAL, "n_c must be in [1, n]");
  const size_t need = pecann_cluster_workspace_size(n);
  if (!ws || ws_bytes < need || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", need, ws_bytes);
  Carver c(ws);
  uint64_t *gkey = c.take<uint64_t>((size_t)n);
  int32_t *flag = c.take<int32_t>(64);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_fill_i32(flag, 0, 1, s));
  PROF(F_CLUSTER, s);
  HIP_TRY(launch_cluster(n, rho, dep, delta, center_mode, n_c, delta_min, rho_min, labels, is_center,
                         gkey, flag, s));
  return PECANN_OK;
}
