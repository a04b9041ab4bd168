// C ABI of libpecann.so: argument validation, prepared-buffer layout, workspace
// carving and the launch sequences of each call (host side only).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "kernels.hpp"
#include "pecann.h"

using namespace pecann;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

// Launch tuning (speed only; see pecann_set_tuning).  Per host thread.
static thread_local pecann_tuning g_tuning = {0, 0, 0, 0, 0};

static pecann_status fail(pecann_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

// Checked builds: after an entry point's launches, wait for them and fail the
// call if a kernel recorded a broken invariant.
static pecann_status check_device(pecann_status st) {
#ifdef PECANN_CHECKED
  if (st != PECANN_OK) return st;
  const hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(PECANN_EHIP, "hipDeviceSynchronize: %s", hipGetErrorString(e));
  using namespace pecann;
  const uint32_t w = check_take_search() | check_take_search_mfma() | check_take_prune() | check_take_misc() |
                     check_take_bruteforce() | check_take_exact() | check_take_nndescent();
  if (w)
    return fail(PECANN_ECHECK, "device invariant check failed: bits 0x%x (1 item, 2 neighbour, 4 beam, "
                "8 instance, 16 prune, 32 reverse edge, 64 chunk, 128 label)", w);
#endif
  return st;
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
    case PECANN_ECHECK: return "device invariant check failed";
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
                                 "exact_mfma", "prepare", "cluster", "nnd_join", "nnd_update",
                                 "nnd_lists", "nnd_prune", "other"};
enum Family { F_SEARCH_BUILD, F_SEARCH_KNN, F_SEARCH_DEP, F_PRUNE_FWD, F_PRUNE_REV, F_REV,
              F_BF_KNN, F_BF_DEP, F_EXACT_MFMA, F_PREPARE, F_CLUSTER, F_NND_JOIN, F_NND_UPDATE,
              F_NND_LISTS, F_NND_PRUNE, F_OTHER, F_COUNT };
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

extern "C" pecann_status pecann_set_tuning(const pecann_tuning *t) {
  clear_stale_error();
  if (!t) {
    g_tuning = pecann_tuning{0, 0, 0, 0, 0};
    return PECANN_OK;
  }
  auto bits_ok = [](int32_t b) { return b == 0 || (b >= 10 && b <= 13); };
  if (!bits_ok(t->hash_bits_build) || !bits_ok(t->hash_bits_search))
    return fail(PECANN_EINVAL, "hash bits must be 0 or in [10, 13]");
  if (t->grid_per_cu != 0 && (t->grid_per_cu < 4 || t->grid_per_cu > 64))
    return fail(PECANN_EINVAL, "grid_per_cu must be 0 or in [4, 64]");
  if (t->scorer < 0 || t->scorer > 2) return fail(PECANN_EINVAL, "scorer must be 0, 1 or 2");
  if (t->prune_steps != 0 && t->prune_steps != 2 && t->prune_steps != 4)
    return fail(PECANN_EINVAL, "prune_steps must be 0, 2 or 4");
  g_tuning = *t;
  return PECANN_OK;
}

extern "C" pecann_status pecann_get_tuning(pecann_tuning *t) {
  if (!t) return fail(PECANN_EINVAL, "tuning is NULL");
  *t = g_tuning;
  return PECANN_OK;
}

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
  const int per_cu = g_tuning.grid_per_cu > 0 ? g_tuning.grid_per_cu : 32;
  int64_t g = (int64_t)cu_count() * per_cu;
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
  size_t off_xg, xg_stride, xg_soff;  // MXFP6 rows: offset, bytes per row, scale words
  size_t off_sqn_g;
  size_t total;
  bool has_xr, has_scale, has_xg;
};

static size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static bool valid_dtype(int32_t t) { return t >= PECANN_F32 && t <= PECANN_MXFP6; }

// Row format of the distance tiles, brute-force scans and fallbacks: MXFP6
// datasets keep an FP8 copy for them.
static int32_t tile_dtype(int32_t sdt) { return sdt == PECANN_MXFP6 ? PECANN_FP8E4M3 : sdt; }

static bool make_layout(int64_t n, int32_t d, int32_t metric, int32_t sdt, Layout *L) {
  if (n < 2 || n >= (int64_t)1 << 31 || d < 1 || d > 4096) return false;
  if (metric != PECANN_L2 && metric != PECANN_COSINE) return false;
  if (!valid_dtype(sdt)) return false;
  if (sdt == PECANN_U8 && metric != PECANN_L2) return false;
  const int32_t tdt = tile_dtype(sdt);
  const size_t bytes = tdt == PECANN_F32 ? 4 : tdt == PECANN_BF16 ? 2 : 1;
  L->off_xs = 0;
  // BF16 / FP8 rows end on a whole matrix-core step of the search's scoring
  // (32 BF16 or 128 FP8 values), zero padded, so its loads need no bounds
  L->xs_stride = up((size_t)d * bytes, tdt == PECANN_BF16 ? 64 : tdt == PECANN_FP8E4M3 ? 128 : 16);
  size_t off = up(L->xs_stride * (size_t)n, 256);
  // MXFP6 rows: per step of 128 values, four 24-byte blocks of 32 packed
  // codes, then one 32-bit word of the four block scales per step; rows padded
  // to 64 bytes
  L->has_xg = sdt == PECANN_MXFP6;
  const size_t steps6 = up((size_t)d, 128) / 128;
  L->xg_soff = 96 * steps6;
  L->xg_stride = up(100 * steps6, 64);
  L->off_xg = off;
  if (L->has_xg) off = up(off + L->xg_stride * (size_t)n, 256);
  L->off_sqn_g = off;
  if (L->has_xg) off = up(off + 4 * (size_t)n, 256);
  L->has_xr = (tdt == PECANN_BF16 || tdt == PECANN_FP8E4M3);
  L->xr_stride = up((size_t)d, 4);
  L->off_xr = off;
  if (L->has_xr) off = up(off + L->xr_stride * 4 * (size_t)n, 256);
  L->has_scale = (tdt == PECANN_FP8E4M3);
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
  r.xg = L.has_xg ? base + L.off_xg : nullptr;
  r.xg_stride = (int64_t)L.xg_stride;
  r.xg_soff = (int32_t)L.xg_soff;
  r.sqn_g = L.has_xg ? (const uint32_t *)(base + L.off_sqn_g) : nullptr;
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
                         L.has_xr ? (float *)(base + L.off_sqn_r) : nullptr,
                         L.has_xg ? base + L.off_xg : nullptr,
                         L.has_xg ? (uint32_t *)(base + L.off_sqn_g) : nullptr, (hipStream_t)stream));
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
// visits some 15 L distinct points), or 10 L for build searches over search
// rows under 512 bytes, between 2^10 and 2^13.  The hash may forget (results
// do not change, only repeated distance evaluations) and a larger table costs
// occupancy; a forgotten point costs a row gather, so short rows favour the
// smaller table.  Measured (build searches): 784-d float32 rows, L = 128:
// 4096 slots 196 ms, 2048 223 ms; 128-d BF16 rows, L = 128: 4096 496 ms, 2048
// 453 ms; 1024-d FP8, L = 200: 4096 and 2048 within 2 %.  The kNN search of
// the 128-d BF16 rows (L = 64) was faster with 2048 slots than with 1024.
// Where the searches score BF16 / FP8 candidates, unless the tuning says
// otherwise: the matrix cores for FP8 rows of 512 bytes or more, whose decode
// dominates on the vector units (1.28M x 1024 FP8 build search: 2,240 ->
// 1,945 ms per step); the vector units for BF16 rows, which unpack with a
// shift (1M x 128: 408 vs 424 ms; 64 instances x 384-d: 1,086 vs 1,407 ms).
static int use_mfma(int32_t sdt, size_t row_bytes) {
  if (sdt == PECANN_MXFP6) return 1;  // scored on the matrix cores only
  if (sdt != PECANN_BF16 && sdt != PECANN_FP8E4M3) return 0;
  if (g_tuning.scorer != 0) return g_tuning.scorer == 2;
  return sdt == PECANN_FP8E4M3 && row_bytes >= 512;
}

static int hash_bits_for(int L, size_t row_bytes, bool build) {
  const int forced = build ? g_tuning.hash_bits_build : g_tuning.hash_bits_search;
  if (forced > 0) return forced;
  const int mult = (build && row_bytes < 512) ? 10 : 20;
  int b = 10;
  while (b < 13 && (1 << b) < mult * L) ++b;
  return b;
}

// ---------------------------------------------------------------------------
// Instances: host spec, validation, device table
// ---------------------------------------------------------------------------
static constexpr int kMaxInstances = 4096;

struct InstSpec {
  std::vector<int64_t> off;  // count + 1
  std::vector<int32_t> k, nc;
  int count() const { return (int)k.size(); }
  int64_t size(int t) const { return off[t + 1] - off[t]; }
  int64_t max_size() const {
    int64_t m = 0;
    for (int t = 0; t < count(); ++t) m = std::max(m, size(t));
    return m;
  }
};

// One instance over all n points.
static InstSpec single_spec(int64_t n, int32_t k, int32_t nc) {
  InstSpec sp;
  sp.off = {0, n};
  sp.k = {k};
  sp.nc = {nc};
  return sp;
}

// Validates the caller's instance table against n points.  k_default /
// nc_default fill tables the caller leaves NULL.
static pecann_status make_spec(int64_t n, const pecann_instances *pi, int32_t k_default,
                               int32_t nc_default, InstSpec *sp) {
  if (!pi) return fail(PECANN_EINVAL, "instances are NULL");
  if (pi->reserved != 0) return fail(PECANN_EINVAL, "instances.reserved must be 0");
  const int I = pi->num_instances;
  if (I < 1 || I > kMaxInstances) return fail(PECANN_EINVAL, "num_instances must be in [1, %d]", kMaxInstances);
  if (!pi->offsets) return fail(PECANN_EINVAL, "instances.offsets is NULL");
  if (pi->offsets[0] != 0 || pi->offsets[I] != n)
    return fail(PECANN_EINVAL, "offsets must start at 0 and end at n = %lld", (long long)n);
  sp->off.assign(pi->offsets, pi->offsets + I + 1);
  sp->k.assign(I, k_default);
  sp->nc.assign(I, nc_default);
  for (int t = 0; t < I; ++t) {
    if (sp->off[t + 1] - sp->off[t] < 2) return fail(PECANN_EINVAL, "instance %d has fewer than 2 points", t);
    if (pi->k) sp->k[t] = pi->k[t];
    if (pi->n_c) sp->nc[t] = pi->n_c[t];
  }
  return PECANN_OK;
}

// k of every instance in [1, min(n_t - 1, kmax)], kmax <= 64.
static pecann_status check_inst_k(const InstSpec &sp, int32_t kmax) {
  if (kmax < 1 || kmax > 64) return fail(PECANN_EINVAL, "k must be in [1, 64]");
  for (int t = 0; t < sp.count(); ++t)
    if (sp.k[t] < 1 || sp.k[t] > kmax || sp.k[t] > sp.size(t) - 1)
      return fail(PECANN_EINVAL, "k of instance %d must be in [1, min(n_t - 1, %d)]", t, kmax);
  return PECANN_OK;
}

struct InstDev {
  int64_t *off;
  int32_t *k, *nc;
};
static void carve_inst(Carver &c, int count, InstDev *d) {
  d->off = c.take<int64_t>((size_t)count + 1);
  d->k = c.take<int32_t>((size_t)count);
  d->nc = c.take<int32_t>((size_t)count);
}
// Device copy of the table through kernel arguments (no host buffer to keep).
static hipError_t upload_inst(const InstSpec &sp, const InstDev &d, hipStream_t s) {
  const int I = sp.count();
  for (int b = 0; b <= I; b += 64) {
    I64Chunk c;
    const int cnt = std::min(64, I + 1 - b);
    for (int j = 0; j < cnt; ++j) c.v[j] = sp.off[b + j];
    hipError_t e = launch_put_i64(c, cnt, d.off + b, s);
    if (e != hipSuccess) return e;
  }
  for (int b = 0; b < I; b += 64) {
    I32Chunk ck, cn;
    const int cnt = std::min(64, I - b);
    for (int j = 0; j < cnt; ++j) { ck.v[j] = sp.k[b + j]; cn.v[j] = sp.nc[b + j]; }
    hipError_t e = launch_put_i32(ck, cnt, d.k + b, s);
    if (e == hipSuccess) e = launch_put_i32(cn, cnt, d.nc + b, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
static InstTable table_of(const InstDev &d, int count) {
  InstTable t;
  t.off = d.off;
  t.k = d.k;
  t.nc = d.nc;
  t.count = count;
  return t;
}

// ---------------------------------------------------------------------------
// Graph build
// ---------------------------------------------------------------------------
// new in-edges a heavy target takes into the LDS at once; a target with more
// is pruned over its sorted candidates in slices of this size
static constexpr int kCapIn = 1024;

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

// One build round: the next batch of every instance that has one.  An
// instance's batches follow the single-instance schedule (DiskANN's two
// passes: the first starts the graph with the instance's first point and
// doubles its batch from 1 up to the cap, the second re-inserts every point in
// full batches).
struct BuildRange { int32_t pbeg, cnt, sbase, ns; };
struct BuildRound {
  int pass;
  std::vector<BuildRange> ranges;
  int64_t total = 0;
  int32_t maxcnt = 0;
};
static std::vector<BuildRound> build_schedule(const InstSpec &sp, const pecann_build_params *bp,
                                              int passes) {
  std::vector<BuildRound> rounds;
  const int I = sp.count();
  std::vector<int64_t> ins(I), bs(I), cap(I);
  for (int t = 0; t < I; ++t) cap[t] = batch_cap(sp.size(t), bp->max_batch);
  for (int pass = 0; pass < passes; ++pass) {
    for (int t = 0; t < I; ++t) {
      ins[t] = pass == 0 ? 1 : 0;
      bs[t] = pass == 0 ? 1 : cap[t];
    }
    for (;;) {
      BuildRound r;
      r.pass = pass;
      for (int t = 0; t < I; ++t) {
        const int64_t nt = sp.size(t);
        if (ins[t] >= nt) continue;
        const int64_t nb = std::min(std::min(bs[t], cap[t]), nt - ins[t]);
        const int64_t in_graph = pass == 0 ? ins[t] : nt;
        BuildRange g;
        g.pbeg = (int32_t)(sp.off[t] + ins[t]);
        g.cnt = (int32_t)nb;
        g.sbase = (int32_t)sp.off[t];
        g.ns = (int32_t)std::min<int64_t>(bp->num_starts, in_graph);
        r.ranges.push_back(g);
        r.total += nb;
        r.maxcnt = std::max(r.maxcnt, g.cnt);
        ins[t] += nb;
        if (bs[t] < cap[t]) bs[t] *= 2;  // stop doubling at the cap (no overflow)
      }
      if (r.ranges.empty()) break;
      rounds.push_back(std::move(r));
    }
  }
  return rounds;
}
static int64_t round_capacity(const InstSpec &sp, int32_t max_batch) {
  int64_t c = 0;
  for (int t = 0; t < sp.count(); ++t) c += batch_cap(sp.size(t), max_batch);
  return c;
}

struct BuildWs {
  int32_t *perm, *ctr, *vis_count, *rcnt, *tidx, *tlist, *tord, *toff, *tcnt, *ticket, *seg;
  int32_t *items, *item_sbase, *item_ns;
  uint64_t *vis;
  uint64_t *akey, *segk;  // keys of the adjacency entries, of the grouped reverse edges
  int32_t *cons;          // entries of each row its last prune selected
};

static void carve_build(Carver &c, int64_t n, int R, int64_t cap, int vcap, BuildWs *w) {
  w->perm = c.take<int32_t>((size_t)n);
  w->ctr = c.take<int32_t>(64);
  w->vis = c.take<uint64_t>((size_t)cap * vcap);
  w->vis_count = c.take<int32_t>((size_t)cap);
  w->items = c.take<int32_t>((size_t)cap);
  w->item_sbase = c.take<int32_t>((size_t)cap);
  w->item_ns = c.take<int32_t>((size_t)cap);
  w->rcnt = c.take<int32_t>((size_t)n);
  w->tidx = c.take<int32_t>((size_t)n);
  const size_t ce = (size_t)cap * R;
  w->tlist = c.take<int32_t>(ce);
  w->tord = c.take<int32_t>(ce);
  w->toff = c.take<int32_t>(ce);
  w->tcnt = c.take<int32_t>(ce);
  w->ticket = c.take<int32_t>(ce);
  w->seg = c.take<int32_t>(ce);
  w->akey = c.take<uint64_t>((size_t)n * R);
  w->segk = c.take<uint64_t>(ce);
  w->cons = c.take<int32_t>((size_t)n);
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

static size_t build_ws_size(const pecann_dataset *ds, const pecann_build_params *bp, const InstSpec &sp) {
  Carver c(nullptr);
  BuildWs w;
  carve_build(c, ds->n, bp->R, round_capacity(sp, bp->max_batch), effective_vcap(bp), &w);
  return c.size();
}

extern "C" size_t pecann_build_graph_workspace_size(const pecann_dataset *ds, const pecann_build_params *bp) {
  Layout L;
  if (check_dataset(ds, &L) != PECANN_OK || check_build(ds, bp) != PECANN_OK) return 0;
  return build_ws_size(ds, bp, single_spec(ds->n, 1, 1));
}

extern "C" size_t pecann_build_graph_batched_workspace_size(const pecann_dataset *ds,
                                                           const pecann_build_params *bp,
                                                           const pecann_instances *inst) {
  Layout L;
  InstSpec sp;
  if (check_dataset(ds, &L) != PECANN_OK || check_build(ds, bp) != PECANN_OK) return 0;
  if (make_spec(ds->n, inst, 1, 1, &sp) != PECANN_OK) return 0;
  return build_ws_size(ds, bp, sp);
}

// SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) driving a Fisher-Yates shuffle.
static uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

#define HIP_TRY_ROUND(expr)                                                                     \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(PECANN_EHIP, "%s: %s (pass %d, round %d, %lld items)", #expr,                \
                  hipGetErrorString(e_), rd.pass, ri, (long long)rd.total);                     \
  } while (0)

static pecann_status build_impl(const pecann_dataset *ds, const pecann_build_params *bp,
                                const InstSpec &spec, const int32_t *perm, uint64_t seed,
                                int32_t *adj, int32_t *deg, uint64_t *counters, void *ws,
                                size_t ws_bytes, void *stream) {
  Layout L;
  pecann_status st = check_dataset(ds, &L);
  if (st != PECANN_OK) return st;
  if ((st = check_build(ds, bp)) != PECANN_OK) return st;
  if (!adj || !deg) return fail(PECANN_EINVAL, "adj/deg are NULL");
  const int64_t n = ds->n;
  const int R = bp->R;
  const int vcap = effective_vcap(bp);
  const int64_t cap = round_capacity(spec, bp->max_batch);
  const int I = spec.count();
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
  const int tdt = tile_dtype(dt);
  const int S = engine_shape(dt, ds->d);
  const int passes = bp->passes == 0 ? 2 : bp->passes;
  const std::vector<BuildRound> sched = build_schedule(spec, bp, passes);

  const int32_t *order = perm;
  if (!order) {
    // instance t: its own seeded shuffle (seed + t) of its points
    std::vector<int32_t> h((size_t)n);
    for (int t = 0; t < I; ++t) {
      const int64_t lo = spec.off[t], nt = spec.size(t);
      for (int64_t i = 0; i < nt; ++i) h[lo + i] = (int32_t)(lo + i);
      uint64_t sm = seed + (uint64_t)t;
      for (int64_t i = nt - 1; i > 0; --i) {
        const int64_t j = (int64_t)(splitmix64(sm) % (uint64_t)(i + 1));
        std::swap(h[lo + i], h[lo + j]);
      }
    }
    HIP_TRY(hipMemcpyAsync(w.perm, h.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // h is pageable and about to go away
    order = w.perm;
  }

  HIP_TRY(launch_fill_i32(adj, -1, n * R, s));
  HIP_TRY(launch_fill_i32(deg, 0, n, s));
  HIP_TRY(launch_fill_i32(w.rcnt, 0, n, s));
  HIP_TRY(launch_fill_i32(w.cons, 0, n, s));

  int32_t *head_search = w.ctr + 0, *head_pf = w.ctr + 1, *head_pr = w.ctr + 2;
  int32_t *ntargets = w.ctr + 3, *cursor = w.ctr + 4;
  int32_t *nlight = w.ctr + 5, *nheavy = w.ctr + 6, *head_ph = w.ctr + 7;

  SearchParams sp = {};
  sp.rows = rows;
  sp.adj = adj;
  sp.deg = deg;
  sp.R = R;
  sp.n = (int32_t)n;
  sp.item_count = nullptr;
  sp.head = head_search;
  sp.starts = order;
  sp.item_sbase = w.item_sbase;
  sp.item_ns = w.item_ns;
  sp.items = w.items;
  sp.L = bp->L;
  sp.hbits = hash_bits_for(bp->L, L.xs_stride, true);
  sp.hid_bits = compact_hash_bits(ds->n, sp.hbits);
  sp.mfma = use_mfma(ds->search_dtype, L.xs_stride);
  sp.mode = MODE_BUILD;
  sp.vis = w.vis;
  sp.vis_count = w.vis_count;
  sp.vcap = vcap;
  sp.counters = (unsigned long long *)counters;

  PruneParams pp = {};
  pp.rows = rows;
  pp.n = (int32_t)n;
  pp.sg = g_tuning.prune_steps;
  pp.R = R;
  pp.adj = adj;
  pp.deg = deg;
  pp.items = w.items;
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
  pp.akey = w.akey;
  pp.segk = w.segk;
  pp.cons = w.cons;
  pp.rcnt = w.rcnt;
  pp.counters = counters ? (unsigned long long *)counters + 4 : nullptr;

  for (int ri = 0; ri < (int)sched.size(); ++ri) {
    const BuildRound &rd = sched[ri];
    // DiskANN's schedule: alpha = 1 first, the given alpha last
    pp.alpha = (passes == 2 && rd.pass == 0) ? 1.0f : bp->alpha;
    const int32_t nb = (int32_t)rd.total;
    for (size_t r0 = 0; r0 < rd.ranges.size(); r0 += 32) {
      RangeChunk ch;
      int cnt = 0;
      int32_t obeg = 0;
      for (size_t j = 0; j < r0; ++j) obeg += rd.ranges[j].cnt;
      for (; cnt < 32 && r0 + cnt < rd.ranges.size(); ++cnt) {
        const BuildRange &g = rd.ranges[r0 + cnt];
        ch.pbeg[cnt] = g.pbeg;
        ch.cnt[cnt] = g.cnt;
        ch.obeg[cnt] = obeg;
        ch.sbase[cnt] = g.sbase;
        ch.ns[cnt] = g.ns;
        obeg += g.cnt;
      }
      HIP_TRY_ROUND(launch_gather_items(ch, cnt, rd.maxcnt, order, w.items, w.item_sbase, w.item_ns, s));
    }
    HIP_TRY_ROUND(launch_fill_i32(w.ctr, 0, 8, s));
    sp.nitems = nb;
    {
      PROF(F_SEARCH_BUILD, s);
      HIP_TRY_ROUND(launch_search(dt, S, sp, persistent_grid(nb), s));
    }
    pp.nb = nb;
    pp.head = head_pf;
    {
      PROF(F_PRUNE_FWD, s);
      HIP_TRY_ROUND(launch_prune_forward(tdt, pp, persistent_grid(nb), s));
    }
    {
      PROF(F_REV, s);
      HIP_TRY_ROUND(launch_rev_count(adj, deg, w.items, nb, R, w.rcnt, ntargets, w.tlist, w.tidx,
                                     w.ticket, s));
      HIP_TRY_ROUND(launch_rev_alloc(w.tlist, ntargets, w.rcnt, w.toff, w.tcnt, cursor, w.tord,
                                     nlight, nheavy, kLightIn, (int32_t)((int64_t)nb * R), s));
      HIP_TRY_ROUND(launch_rev_scatter(adj, deg, w.items, nb, R, w.tidx, w.toff, w.ticket, w.seg,
                                       w.akey, w.segk, s));
    }
    {
      PROF(F_PRUNE_REV, s);
      pp.heavy = 0;
      pp.head = head_pr;
      pp.capin = kLightIn;
      HIP_TRY_ROUND(launch_prune_reverse(tdt, pp, persistent_grid((int64_t)nb * R), s));
      pp.heavy = 1;
      pp.head = head_ph;
      pp.capin = kCapIn;
      const int heavy_grid = (int)std::min<int64_t>((int64_t)nb * R, (int64_t)cu_count() * kHeavyGridPerCu);
      HIP_TRY_ROUND(launch_prune_reverse(tdt, pp, heavy_grid, s));
    }
  }
  return PECANN_OK;
}

// ---------------------------------------------------------------------------
// NN-descent graph
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kNndPropBudget = (int64_t)1 << 32;  // 4 GiB of proposal buffers
constexpr int64_t kNndPropBytes = 4 + 8 + 4 + 8;      // target, key, ticket, grouped key

// Proposals of one local join at most: U and W hold at most 2K members each,
// pairs U x U (unordered) and U x W, each proposed both ways.
int64_t nnd_maxprop(int K) { return 12LL * K * K - 2LL * K; }

int64_t nnd_chunk(const pecann_nnd_params *np, int64_t n) {
  if (np->chunk > 0) return std::min<int64_t>(np->chunk, n);
  const int64_t c = kNndPropBudget / (nnd_maxprop(np->K) * kNndPropBytes);
  return std::max<int64_t>(1, std::min<int64_t>(n, c));
}

struct NndWs {
  uint64_t *keys[2];
  uint8_t *flags[2];
  uint64_t *acc;
  int32_t *rcnt, *roff, *rticket, *rnew, *rold;
  uint64_t *rseg;
  uint8_t *rsegf;
  int32_t *ptgt, *pticket;
  uint64_t *pkey, *pseg;
  int32_t *pcnt, *poff, *ptouch;
  int32_t *pfill;  // slots filled by each join wave
  int32_t *ctr;    // [0] done [1] rcursor [2] join head [3] merge head [5] cursor
                   // [6] targets [7] overflow [8] prune head
  unsigned long long *updates;
  int32_t *rounds;
};

// Join waves of a pass: each owns a segment of at least one worst-case join.
int nnd_join_grid(int64_t n, int64_t chunk) {
  return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)cu_count() * 32, n, chunk}));
}

void carve_nnd(Carver &c, int64_t n, int K, int repeats, int64_t chunk, NndWs *w) {
  const size_t nk = (size_t)(n * K);
  const size_t pc = (size_t)(chunk * nnd_maxprop(K));
  w->keys[0] = c.take<uint64_t>(nk);
  w->keys[1] = c.take<uint64_t>(nk);
  w->flags[0] = c.take<uint8_t>(nk);
  w->flags[1] = c.take<uint8_t>(nk);
  w->acc = repeats > 1 ? c.take<uint64_t>(nk) : nullptr;
  w->rcnt = c.take<int32_t>((size_t)n);
  w->roff = c.take<int32_t>((size_t)n);
  w->rticket = c.take<int32_t>(nk);
  w->rnew = c.take<int32_t>(nk);
  w->rold = c.take<int32_t>(nk);
  w->rseg = c.take<uint64_t>(nk);
  w->rsegf = c.take<uint8_t>(nk);
  w->ptgt = c.take<int32_t>(pc);
  w->pticket = c.take<int32_t>(pc);
  w->pkey = c.take<uint64_t>(pc);
  w->pseg = c.take<uint64_t>(pc);
  w->pcnt = c.take<int32_t>((size_t)n);
  w->poff = c.take<int32_t>((size_t)n);
  w->ptouch = c.take<int32_t>((size_t)n);
  w->pfill = c.take<int32_t>((size_t)cu_count() * 32);
  w->ctr = c.take<int32_t>(16);
  w->updates = c.take<unsigned long long>(1);
  w->rounds = c.take<int32_t>(16);
}

pecann_status check_nnd(const pecann_dataset *ds, const pecann_nnd_params *np) {
  if (!np) return fail(PECANN_EINVAL, "NN-descent params are NULL");
  if (np->K < 1 || np->K > 64) return fail(PECANN_EINVAL, "K must be in [1, 64]");
  if (np->K > ds->n - 1) return fail(PECANN_EINVAL, "K must be <= n - 1");
  if (np->R < 1 || np->R > 128) return fail(PECANN_EINVAL, "R must be in [1, 128]");
  if (!(np->alpha >= 1.0f) || !std::isfinite(np->alpha)) return fail(PECANN_EINVAL, "alpha must be >= 1");
  if (np->max_iters < 0 || np->max_iters > 1000) return fail(PECANN_EINVAL, "max_iters must be in [0, 1000]");
  if (!(np->delta >= 0.0f) || !std::isfinite(np->delta)) return fail(PECANN_EINVAL, "delta must be >= 0");
  if (np->num_repeats < 1 || np->num_repeats > 16) return fail(PECANN_EINVAL, "num_repeats must be in [1, 16]");
  if (np->chunk < 0) return fail(PECANN_EINVAL, "chunk must be >= 0");
  if (np->reserved != 0) return fail(PECANN_EINVAL, "NN-descent params reserved field must be 0");
  if (nnd_chunk(np, ds->n) * nnd_maxprop(np->K) >= ((int64_t)1 << 31))
    return fail(PECANN_EINVAL, "chunk too large: its proposal count must stay below 2^31");
  return PECANN_OK;
}
}  // namespace

extern "C" size_t pecann_build_graph_nndescent_workspace_size(const pecann_dataset *ds,
                                                              const pecann_nnd_params *np) {
  Layout L;
  if (check_dataset(ds, &L) != PECANN_OK || check_nnd(ds, np) != PECANN_OK) return 0;
  Carver c(nullptr);
  NndWs w;
  carve_nnd(c, ds->n, np->K, np->num_repeats, nnd_chunk(np, ds->n), &w);
  return c.size();
}

extern "C" pecann_status pecann_build_graph_nndescent(const pecann_dataset *ds,
                                                      const pecann_nnd_params *np,
                                                      const int32_t *init, int32_t *adj,
                                                      int32_t *deg, int32_t *knn_idx,
                                                      float *knn_dist, int32_t *rounds,
                                                      uint64_t *counters, void *ws,
                                                      size_t ws_bytes, void *stream) {
  clear_stale_error();
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  Layout L;
  pecann_status st = check_dataset(ds, &L);
  if (st != PECANN_OK) return st;
  if ((st = check_nnd(ds, np)) != PECANN_OK) return st;
  if (!init || !adj || !deg) return fail(PECANN_EINVAL, "init/adj/deg are NULL");
  const int64_t n = ds->n;
  const int K = np->K, reps = np->num_repeats;
  const int64_t chunk = nnd_chunk(np, n);
  Carver c0(nullptr);
  NndWs w;
  carve_nnd(c0, n, K, reps, chunk, &w);
  if (!ws || ws_bytes < c0.size() || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", c0.size(), ws_bytes);
  Carver c(ws);
  carve_nnd(c, n, K, reps, chunk, &w);
  hipStream_t s = (hipStream_t)stream;
  const int dt = ds->search_dtype;
  const int tdt = tile_dtype(dt);
  const int cus = cu_count();
  unsigned long long *ctrs = (unsigned long long *)counters;

  NndParams P = {};
  P.rows = rows_of(ds, L);
  P.n = (int32_t)n;
  P.K = K;
  P.done = w.ctr + 0;
  P.rcursor = w.ctr + 1;
  P.pcursor = w.ctr + 5;
  P.ptouch_n = w.ctr + 6;
  P.overflow = w.ctr + 7;
  P.updates = w.updates;
  P.maxprop = nnd_maxprop(K);
  const int jgrid = nnd_join_grid(n, chunk);
  P.seg = chunk * nnd_maxprop(K) / jgrid;
  P.pfill = w.pfill;
  // points a pass joins at least (unless the round's queue runs out)
  const int64_t per_pass = (int64_t)jgrid * (P.seg / P.maxprop);
  P.thr = (long long)std::floor((double)np->delta * (double)n * (double)K);
  P.rcnt = w.rcnt;
  P.roff = w.roff;
  P.rticket = w.rticket;
  P.rseg = w.rseg;
  P.rsegf = w.rsegf;
  P.rnew = w.rnew;
  P.rold = w.rold;
  P.ptgt = w.ptgt;
  P.pkey = w.pkey;
  P.pticket = w.pticket;
  P.pseg = w.pseg;
  P.pcnt = w.pcnt;
  P.poff = w.poff;
  P.ptouch = w.ptouch;
  P.counters = ctrs;
  int32_t *rounds_out = rounds ? rounds : w.rounds;

  HIP_TRY(launch_fill_i32(w.ctr, 0, 16, s));
  HIP_TRY(launch_fill_i32(w.rcnt, 0, n, s));
  HIP_TRY(launch_fill_i32(w.pcnt, 0, n, s));
  HIP_TRY(launch_fill_i32(rounds_out, 0, reps, s));
  HIP_TRY(launch_fill_u64((uint64_t *)w.updates, 0, 1, s));

  const uint64_t *final_keys = nullptr;
  for (int r = 0; r < reps; ++r) {
    P.cur_keys = w.keys[0];
    P.cur_flags = w.flags[0];
    P.nxt_keys = w.keys[1];
    P.nxt_flags = w.flags[1];
    P.rounds = rounds_out + r;
    HIP_TRY(launch_fill_i32(P.done, 0, 1, s));
    {
      PROF(F_NND_LISTS, s);
      HIP_TRY(launch_nnd_init(tdt, P, init + (int64_t)r * n * K, (int)std::min<int64_t>(n, (int64_t)cus * 32), s));
    }
    for (int it = 0; it < np->max_iters; ++it) {
      {
        PROF(F_NND_LISTS, s);
        HIP_TRY(launch_nnd_round_begin(P, cus, s));
        HIP_TRY(launch_nnd_reverse(P, 1, 0, cus, s));
      }
      // passes over the round's queue, enough for per_pass joins each; passes
      // after the queue has drained return at once
      HIP_TRY(launch_fill_i32(w.ctr + 2, 0, 1, s));  // join queue head
      for (int64_t b = 0; b < n; b += per_pass) {
        HIP_TRY(launch_fill_i32(w.ctr + 3, 0, 4, s));  // merge head, (unused), cursor, targets
        P.head = w.ctr + 2;
        {
          PROF(F_NND_JOIN, s);
          HIP_TRY(launch_nnd_join(tdt, P, jgrid, s));
        }
        {
          PROF(F_NND_UPDATE, s);
          HIP_TRY(launch_nnd_proposals(P, jgrid, cus, s));
          P.head = w.ctr + 3;
          HIP_TRY(launch_nnd_merge(P, persistent_grid(n), s));
        }
      }
      {
        PROF(F_NND_LISTS, s);
        HIP_TRY(launch_nnd_round_end(P, cus, s));
      }
      std::swap(P.cur_keys, P.nxt_keys);
      std::swap(P.cur_flags, P.nxt_flags);
    }
    if (reps == 1) {
      final_keys = P.cur_keys;
    } else {
      PROF(F_NND_LISTS, s);
      if (r == 0)
        HIP_TRY(launch_nnd_copy(P.cur_keys, w.acc, n * K, cus, s));
      else
        HIP_TRY(launch_nnd_acc_merge(P, w.acc, P.cur_keys, cus, s));
      final_keys = w.acc;
    }
  }
  // reverse lists of the final lists, then the pruned graph
  NndParams Q = P;
  Q.cur_keys = (uint64_t *)final_keys;
  Q.cur_flags = nullptr;
  {
    PROF(F_NND_LISTS, s);
    HIP_TRY(launch_nnd_reverse(Q, 0, 1, cus, s));
  }
  PruneParams pp = {};
  pp.rows = P.rows;
  pp.n = (int32_t)n;
  pp.sg = g_tuning.prune_steps;
  pp.R = np->R;
  pp.alpha = np->alpha;
  pp.adj = adj;
  pp.deg = deg;
  pp.lists = final_keys;
  pp.rlists = w.rnew;
  pp.lk = K;
  pp.head = w.ctr + 8;
  pp.counters = ctrs ? ctrs + 3 : nullptr;
  {
    PROF(F_NND_PRUNE, s);
    HIP_TRY(launch_prune_lists(tdt, pp, persistent_grid(n), s));
  }
  if (knn_idx || knn_dist) HIP_TRY(launch_nnd_out(P, final_keys, knn_idx, knn_dist, cus, s));
  return check_device(PECANN_OK);
}

extern "C" pecann_status pecann_build_graph(const pecann_dataset *ds, const pecann_build_params *bp,
                                            const int32_t *perm, uint64_t seed, int32_t *adj,
                                            int32_t *deg, uint64_t *counters, void *ws,
                                            size_t ws_bytes, void *stream) {
  clear_stale_error();
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  return check_device(build_impl(ds, bp, single_spec(ds->n, 1, 1), perm, seed, adj, deg, counters, ws, ws_bytes,
                    stream));
}

extern "C" pecann_status pecann_build_graph_batched(const pecann_dataset *ds,
                                                    const pecann_build_params *bp,
                                                    const pecann_instances *inst,
                                                    const int32_t *perm, uint64_t seed,
                                                    int32_t *adj, int32_t *deg,
                                                    uint64_t *counters, void *ws, size_t ws_bytes,
                                                    void *stream) {
  clear_stale_error();
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  InstSpec sp;
  pecann_status st = make_spec(ds->n, inst, 1, 1, &sp);
  if (st != PECANN_OK) return st;
  return check_device(build_impl(ds, bp, sp, perm, seed, adj, deg, counters, ws, ws_bytes, stream));
}

// ---------------------------------------------------------------------------
// kNN + density
// ---------------------------------------------------------------------------
// Exact kNN switches to the matrix-core scan from this many points on (per
// instance).
static constexpr int64_t kExactMfmaMin = 4096;

struct KnnWs {
  int32_t *ctr, *fb, *cand;
  uint64_t *thr;  // exact mode: smallest key each query's scan queues dropped, per part
  float *nmax;
  uint64_t *part;  // exact mode: chunk-local best keys of the split brute force
  InstDev inst;
};
// Exact brute force of the queries the matrix-core scan does not settle (and of
// every query of a small instance): the first kSplitCap of them are scanned
// in chunks of kSplitChunk candidates by separate wavefronts and merged; any
// beyond take one wavefront each.
static constexpr int kSplitCap = 2048;
static constexpr int kSplitChunk = 4096;
static int split_chunks(int64_t max_size) { return (int)((max_size + kSplitChunk - 1) / kSplitChunk); }
static bool any_large(const InstSpec &sp) {
  for (int t = 0; t < sp.count(); ++t)
    if (sp.size(t) >= kExactMfmaMin) return true;
  return false;
}
static void carve_knn(Carver &c, int64_t n, bool exact, bool exact_mfma, int ninst, int64_t max_size,
                      int32_t k, KnnWs *w) {
  w->ctr = c.take<int32_t>(64);
  w->fb = c.take<int32_t>((size_t)n);
  w->nmax = c.take<float>(64);
  w->cand = exact_mfma ? c.take<int32_t>((size_t)n * kExactCand) : nullptr;
  w->thr = exact_mfma ? c.take<uint64_t>((size_t)n * kExactParts) : nullptr;
  w->part = exact ? c.take<uint64_t>((size_t)kSplitCap * split_chunks(max_size) * k) : nullptr;
  carve_inst(c, ninst, &w->inst);
}

extern "C" size_t pecann_knn_density_workspace_size(const pecann_dataset *ds, int32_t k,
                                                    int32_t L_search, int32_t exact) {
  Layout L;
  if (check_dataset(ds, &L) != PECANN_OK) return 0;
  (void)L_search;
  if (k < 1 || k > 64) return 0;
  Carver c(nullptr);
  KnnWs w;
  carve_knn(c, ds->n, exact != 0, exact != 0 && ds->n >= kExactMfmaMin, 1, ds->n, k, &w);
  return c.size();
}

extern "C" size_t pecann_knn_density_batched_workspace_size(const pecann_dataset *ds,
                                                            const pecann_instances *inst,
                                                            int32_t k_max, int32_t L_search,
                                                            int32_t exact) {
  Layout L;
  InstSpec sp;
  if (check_dataset(ds, &L) != PECANN_OK || make_spec(ds->n, inst, k_max, 1, &sp) != PECANN_OK) return 0;
  (void)L_search;
  Carver c(nullptr);
  KnnWs w;
  carve_knn(c, ds->n, exact != 0, exact != 0 && any_large(sp), sp.count(), sp.max_size(), k_max, &w);
  return c.size();
}

// Rows of one instance: row 0 of the view is global row lo.
static RowsDesc shift_rows(RowsDesc r, int64_t lo) {
  r.xs += lo * r.xs_stride;
  if (r.xr) r.xr += lo * r.xr_stride;
  if (r.scale) r.scale += lo;
  r.sqn += lo;
  if (r.sqn_r) r.sqn_r += lo;
  if (r.xg) r.xg += lo * r.xg_stride;
  if (r.sqn_g) r.sqn_g += lo;
  return r;
}

static pecann_status knn_impl(const pecann_dataset *ds, const InstSpec &spec, const int32_t *adj,
                              const int32_t *deg, int32_t R, int32_t k, int32_t L_search,
                              int32_t rerank, int32_t *knn_idx, float *knn_dist, float *rho,
                              uint64_t *rank_key, uint64_t *counters, void *ws, size_t ws_bytes,
                              void *stream) {
  Layout L;
  pecann_status st = check_dataset(ds, &L);
  if (st != PECANN_OK) return st;
  const int64_t n = ds->n;
  if ((st = check_inst_k(spec, k)) != PECANN_OK) return st;
  if (!knn_idx || !knn_dist || !rho || !rank_key) return fail(PECANN_EINVAL, "output pointer is NULL");
  if (adj) {
    if (!deg) return fail(PECANN_EINVAL, "deg is NULL");
    if (R < 1 || R > 128) return fail(PECANN_EINVAL, "R must be in [1, 128]");
    if (L_search < k || L_search > 1024) return fail(PECANN_EINVAL, "L_search must be in [k, 1024]");
    const bool lp = ds->search_dtype == PECANN_BF16 || ds->search_dtype == PECANN_FP8E4M3 ||
                      ds->search_dtype == PECANN_MXFP6;
    if (lp && (rerank < k || rerank > L_search))
      return fail(PECANN_EINVAL, "rerank must be in [k, L_search]");
  }
  const int I = spec.count();
  const bool exact_mfma = !adj && any_large(spec);
  Carver c0(nullptr);
  KnnWs w;
  carve_knn(c0, n, !adj, exact_mfma, I, spec.max_size(), k, &w);
  if (!ws || ws_bytes < c0.size() || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", c0.size(), ws_bytes);
  Carver c(ws);
  carve_knn(c, n, !adj, exact_mfma, I, spec.max_size(), k, &w);
  int32_t *ctr = w.ctr, *fb = w.fb;
  hipStream_t s = (hipStream_t)stream;
  const RowsDesc rows = rows_of(ds, L);
  const int dt = ds->search_dtype;
  const int tdt = tile_dtype(dt);
  const int S = engine_shape(dt, ds->d);
  HIP_TRY(launch_fill_i32(ctr, 0, 8, s));
  HIP_TRY(upload_inst(spec, w.inst, s));
  const InstTable itab = table_of(w.inst, I);

  // exact searches of a list of queries (fb, ctr[1] entries) over their instance
  BfKnnParams bp = {};
  bp.rows = rows;
  bp.n = (int32_t)n;
  bp.k = k;
  bp.kstride = k;
  bp.inst = itab;
  bp.skip_from = INT32_MAX;
  bp.knn_idx = knn_idx;
  bp.knn_dist = knn_dist;
  bp.rho = rho;
  bp.rank_key = rank_key;
  bp.items = fb;
  bp.item_count = ctr + 1;
  bp.nitems = 0;
  bp.head = ctr + 2;

  if (!adj) {
    // large instances: matrix-core scan, then exact re-score; queries whose
    // check fails, and every query of a small instance, go to the list
    for (int t = 0; t < I; ++t) {
      const int64_t lo = spec.off[t], nt = spec.size(t);
      if (nt < kExactMfmaMin) continue;
      ExactMfmaParams ep = {};
      ep.rows = shift_rows(rows, lo);
      ep.n = (int32_t)nt;
      ep.k = spec.k[t];
      ep.kstride = k;
      ep.base = (int32_t)lo;
      ep.cand = w.cand + lo * kExactCand;
      ep.thr = w.thr + lo * kExactParts;
      ep.nmax = w.nmax;
      ep.head = ctr + 0;
      ep.knn_idx = knn_idx + lo * k;
      ep.knn_dist = knn_dist + lo * k;
      ep.rho = rho + lo;
      ep.rank_key = rank_key + lo;
      ep.fb_list = fb;
      ep.fb_count = ctr + 1;
      HIP_TRY(launch_fill_i32(ctr, 0, 1, s));
      PROF(F_EXACT_MFMA, s);
      HIP_TRY(launch_exact_mfma(tdt, S, ep, s));
    }
    HIP_TRY(launch_small_instance_points(n, itab, (int32_t)kExactMfmaMin, fb, ctr + 1, s));
    PROF(F_BF_KNN, s);
    bp.part = w.part;
    bp.split_cap = kSplitCap;
    bp.nchunk = split_chunks(spec.max_size());
    bp.chunk = kSplitChunk;
    bp.kpart = k;
    bp.head = ctr + 3;
    bp.head2 = ctr + 4;
    // grids sized for the queries expected here: every point of an instance
    // below the scan's minimum, plus the few the scan's check sends back (the
    // work queues take any count; mostly empty grids cost launch time: 18k
    // idle waves were 0.9 ms of the 70,000-point uint8 step)
    int64_t small = 0;
    for (int t = 0; t < spec.count(); ++t)
      if (spec.size(t) < kExactMfmaMin) small += spec.size(t);
    const int64_t few = (int64_t)cu_count() * 4;
    const int64_t expect = std::min<int64_t>(kSplitCap, small + few);
    HIP_TRY(launch_bf_knn_split(tdt, S, bp, persistent_grid(expect * bp.nchunk), persistent_grid(expect), s));
    bp.head = ctr + 2;
    bp.item_from = kSplitCap;
    HIP_TRY(launch_bf_knn(tdt, S, bp, persistent_grid(std::max<int64_t>(small - kSplitCap, 0) + few), s));
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
  sp.inst = itab;
  sp.L = L_search;
  sp.hbits = hash_bits_for(L_search, L.xs_stride, false);
  sp.hid_bits = compact_hash_bits(ds->n, sp.hbits);
  sp.mfma = use_mfma(ds->search_dtype, L.xs_stride);
  sp.mode = MODE_KNN;
  sp.rerank = rerank;
  sp.k = k;
  sp.kstride = k;
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
  PROF(F_BF_KNN, s);
  HIP_TRY(launch_bf_knn(tdt, S, bp, cu_count() * 4, s));
  return PECANN_OK;
}

extern "C" pecann_status pecann_knn_density(const pecann_dataset *ds, const int32_t *adj,
                                            const int32_t *deg, int32_t R, int32_t k,
                                            int32_t L_search, int32_t rerank, int32_t *knn_idx,
                                            float *knn_dist, float *rho, uint64_t *rank_key,
                                            uint64_t *counters, void *ws, size_t ws_bytes,
                                            void *stream) {
  clear_stale_error();
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  if (k < 1 || k > 64 || k > ds->n - 1) return fail(PECANN_EINVAL, "k must be in [1, min(n-1, 64)]");
  return check_device(knn_impl(ds, single_spec(ds->n, k, 1), adj, deg, R, k, L_search, rerank, knn_idx, knn_dist,
                  rho, rank_key, counters, ws, ws_bytes, stream));
}

extern "C" pecann_status pecann_knn_density_batched(const pecann_dataset *ds,
                                                    const pecann_instances *inst,
                                                    const int32_t *adj, const int32_t *deg,
                                                    int32_t R, int32_t k_max, int32_t L_search,
                                                    int32_t rerank, int32_t *knn_idx,
                                                    float *knn_dist, float *rho,
                                                    uint64_t *rank_key, uint64_t *counters,
                                                    void *ws, size_t ws_bytes, void *stream) {
  clear_stale_error();
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  InstSpec sp;
  pecann_status st = make_spec(ds->n, inst, k_max, 1, &sp);
  if (st != PECANN_OK) return st;
  return check_device(knn_impl(ds, sp, adj, deg, R, k_max, L_search, rerank, knn_idx, knn_dist, rho, rank_key,
                  counters, ws, ws_bytes, stream));
}

// ---------------------------------------------------------------------------
// Dependent points
// ---------------------------------------------------------------------------
static constexpr int kMaxRounds = 30;

struct DepWs {
  int32_t *ctr, *ucnt, *ua, *ub, *ucnt_inst;
  uint64_t *minkey;
  unsigned long long *best;
  InstDev inst;
};
static void carve_dep(Carver &c, int64_t n, int ninst, DepWs *w) {
  w->ctr = c.take<int32_t>(64);
  w->ucnt = c.take<int32_t>(64);
  w->minkey = c.take<uint64_t>((size_t)ninst);
  w->ua = c.take<int32_t>((size_t)n);
  w->ub = c.take<int32_t>((size_t)n);
  w->best = c.take<unsigned long long>((size_t)n);
  w->ucnt_inst = c.take<int32_t>((size_t)(kMaxRounds + 1) * ninst);
  carve_inst(c, ninst, &w->inst);
}

extern "C" size_t pecann_dependent_search_workspace_size(const pecann_dataset *ds, int32_t kdep_cap,
                                                         int32_t L_search) {
  Layout L;
  if (check_dataset(ds, &L) != PECANN_OK) return 0;
  (void)kdep_cap; (void)L_search;
  Carver c(nullptr);
  DepWs w;
  carve_dep(c, ds->n, 1, &w);
  return c.size();
}

extern "C" size_t pecann_dependent_search_batched_workspace_size(const pecann_dataset *ds,
                                                                 const pecann_instances *inst,
                                                                 int32_t kdep_cap, int32_t L_search) {
  Layout L;
  InstSpec sp;
  if (check_dataset(ds, &L) != PECANN_OK || make_spec(ds->n, inst, 1, 1, &sp) != PECANN_OK) return 0;
  (void)kdep_cap; (void)L_search;
  Carver c(nullptr);
  DepWs w;
  carve_dep(c, ds->n, sp.count(), &w);
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

static pecann_status dep_impl(const pecann_dataset *ds, const InstSpec &spec, const int32_t *adj,
                              const int32_t *deg, int32_t R, const uint64_t *rank_key,
                              const int32_t *knn_idx, const float *knn_dist, int32_t k, int32_t L_d,
                              int32_t L_search, int32_t threshold, int32_t kdep_cap, int32_t *dep,
                              float *delta, int32_t *stats, void *ws, size_t ws_bytes, void *stream) {
  Layout L;
  pecann_status st = check_dataset(ds, &L);
  if (st != PECANN_OK) return st;
  const int64_t n = ds->n;
  if ((st = check_inst_k(spec, k)) != PECANN_OK) return st;
  if (!rank_key || !knn_idx || !knn_dist || !dep || !delta) return fail(PECANN_EINVAL, "pointer is NULL");
  if (threshold < 0) return fail(PECANN_EINVAL, "threshold must be >= 0");
  if (adj) {
    if (!deg) return fail(PECANN_EINVAL, "deg is NULL");
    if (R < 1 || R > 128) return fail(PECANN_EINVAL, "R must be in [1, 128]");
    if (L_d <= k) return fail(PECANN_EINVAL, "L_d must be > k");
    if (kdep_cap < L_d || kdep_cap > 1024) return fail(PECANN_EINVAL, "kdep_cap must be in [L_d, 1024]");
    if (L_search < 1 || L_search > 1024) return fail(PECANN_EINVAL, "L_search must be in [1, 1024]");
  }
  const int I = spec.count();
  Carver c0(nullptr);
  DepWs w;
  carve_dep(c0, n, I, &w);
  if (!ws || ws_bytes < c0.size() || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", c0.size(), ws_bytes);
  Carver c(ws);
  carve_dep(c, n, I, &w);
  hipStream_t s = (hipStream_t)stream;
  const RowsDesc rows = rows_of(ds, L);
  const int dt = ds->search_dtype;
  const int tdt = tile_dtype(dt);
  const int S = engine_shape(dt, ds->d);

  HIP_TRY(launch_fill_i32(w.ctr, 0, 64, s));
  HIP_TRY(launch_fill_i32(w.ucnt, 0, 64, s));
  HIP_TRY(launch_fill_i32(w.ucnt_inst, 0, (int64_t)(kMaxRounds + 1) * I, s));
  HIP_TRY(upload_inst(spec, w.inst, s));
  const InstTable itab = table_of(w.inst, I);
  HIP_TRY(launch_min_key(rank_key, itab, w.minkey, s));
  HIP_TRY(launch_dep_in_knn(n, itab, k, rank_key, w.minkey, knn_idx, knn_dist, dep, delta, w.ua,
                            w.ucnt, w.ucnt_inst, s));

  int32_t *cur = w.ua, *nxt = w.ub;
  int nr = 0;
  if (adj) {
    // rounds while some instance may still double: k_dep <= min(kdep_cap, n_t - 1)
    const int64_t lim = std::min<int64_t>(kdep_cap, spec.max_size() - 1);
    for (int64_t kd = L_d; kd <= lim && nr < kMaxRounds; kd *= 2, ++nr) {
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
      sp.inst = itab;
      sp.L = (int32_t)std::max<int64_t>(kd, L_search);
      sp.hbits = hash_bits_for(sp.L, L.xs_stride, false);
      sp.hid_bits = compact_hash_bits(ds->n, sp.hbits);
      sp.mfma = use_mfma(ds->search_dtype, L.xs_stride);
      sp.mode = MODE_DEP;
      sp.rerank = (int32_t)kd;
      sp.kdep = (int32_t)kd;
      sp.kdep_cap = kdep_cap;
      sp.key_in = rank_key;
      sp.dep = dep;
      sp.delta = delta;
      sp.u_out = nxt;
      sp.u_out_count = w.ucnt + nr + 1;
      sp.ucnt_in = w.ucnt_inst + (int64_t)nr * I;
      sp.ucnt_out = w.ucnt_inst + (int64_t)(nr + 1) * I;
      sp.threshold = threshold;
      {
        PROF(F_SEARCH_DEP, s);
        HIP_TRY(launch_search(dt, S, sp, persistent_grid(n), s));
      }
      std::swap(cur, nxt);
    }
  }
  // final brute force over the instance for the points still unfinished
  HIP_TRY(launch_fill_u64((uint64_t *)w.best, ~0ull, n, s));
  BfDepParams bd = {};
  bd.rows = rows;
  bd.n = (int32_t)n;
  bd.ulist = cur;
  bd.ucount = w.ucnt + nr;
  bd.chunk = 4096;
  bd.nchunks = (int32_t)((spec.max_size() + bd.chunk - 1) / bd.chunk);
  bd.head = w.ctr + 40;
  bd.inst = itab;
  bd.key = rank_key;
  bd.best = w.best;
  {
    PROF(F_BF_DEP, s);
    HIP_TRY(launch_bf_dep(tdt, S, bd, persistent_grid(n * (int64_t)bd.nchunks), s));
  }
  HIP_TRY(launch_bf_dep_finalize(cur, w.ucnt + nr, w.best, ds->metric, dep, delta, (int32_t)n, s));
  if (stats) {
    hipLaunchKernelGGL(dep_stats_kernel, dim3(1), dim3(64), 0, s, w.ucnt, nr, stats);
    HIP_TRY(hipGetLastError());
  }
  return PECANN_OK;
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
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  if (k < 1 || k > 64 || k > ds->n - 1) return fail(PECANN_EINVAL, "k must be in [1, min(n-1, 64)]");
  return check_device(dep_impl(ds, single_spec(ds->n, k, 1), adj, deg, R, rank_key, knn_idx, knn_dist, k, L_d,
                  L_search, threshold, kdep_cap, dep, delta, stats, ws, ws_bytes, stream));
}

extern "C" pecann_status pecann_dependent_search_batched(const pecann_dataset *ds,
                                                         const pecann_instances *inst,
                                                         const int32_t *adj, const int32_t *deg,
                                                         int32_t R, const uint64_t *rank_key,
                                                         const int32_t *knn_idx,
                                                         const float *knn_dist, int32_t k_max,
                                                         int32_t L_d, int32_t L_search,
                                                         int32_t threshold, int32_t kdep_cap,
                                                         int32_t *dep, float *delta, int32_t *stats,
                                                         void *ws, size_t ws_bytes, void *stream) {
  clear_stale_error();
  if (!ds) return fail(PECANN_EINVAL, "dataset is NULL");
  InstSpec sp;
  pecann_status st = make_spec(ds->n, inst, k_max, 1, &sp);
  if (st != PECANN_OK) return st;
  return check_device(dep_impl(ds, sp, adj, deg, R, rank_key, knn_idx, knn_dist, k_max, L_d, L_search, threshold,
                  kdep_cap, dep, delta, stats, ws, ws_bytes, stream));
}

// ---------------------------------------------------------------------------
// Cluster
// ---------------------------------------------------------------------------
static size_t cluster_ws_size(int64_t n, int ninst) {
  Carver c(nullptr);
  c.take<uint64_t>((size_t)n);
  c.take<int32_t>(64);
  c.take<uint32_t>(kSelWords);
  InstDev d;
  carve_inst(c, ninst, &d);
  return c.size();
}

extern "C" size_t pecann_cluster_workspace_size(int64_t n) {
  if (n < 1) return 0;
  return cluster_ws_size(n, 1);
}

extern "C" size_t pecann_cluster_batched_workspace_size(int64_t n, const pecann_instances *inst) {
  InstSpec sp;
  if (n < 2 || make_spec(n, inst, 1, 1, &sp) != PECANN_OK) return 0;
  return cluster_ws_size(n, sp.count());
}

static pecann_status cluster_impl(int64_t n, const InstSpec &spec, const float *rho, const int32_t *dep,
                                  const float *delta, int32_t center_mode, float delta_min,
                                  float rho_min, int32_t *labels, uint8_t *is_center, void *ws,
                                  size_t ws_bytes, void *stream) {
  if (n < 1 || n >= (int64_t)1 << 31) return fail(PECANN_EINVAL, "n out of range");
  if (!rho || !dep || !delta || !labels || !is_center) return fail(PECANN_EINVAL, "pointer is NULL");
  if (center_mode != PECANN_CENTER_PRODUCT && center_mode != PECANN_CENTER_THRESHOLD &&
      center_mode != PECANN_CENTER_GIVEN)
    return fail(PECANN_EINVAL, "center_mode");
  if (center_mode == PECANN_CENTER_PRODUCT)
    for (int t = 0; t < spec.count(); ++t)
      if (spec.nc[t] < 1 || spec.nc[t] > spec.size(t))
        return fail(PECANN_EINVAL, "n_c of instance %d must be in [1, n_t]", t);
  const size_t need = cluster_ws_size(n, spec.count());
  if (!ws || ws_bytes < need || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", need, ws_bytes);
  Carver c(ws);
  uint64_t *gkey = c.take<uint64_t>((size_t)n);
  int32_t *flag = c.take<int32_t>(64);
  uint32_t *sel = c.take<uint32_t>(kSelWords);  // wide center-select state
  InstDev d;
  carve_inst(c, spec.count(), &d);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_fill_i32(flag, 0, 1, s));
  HIP_TRY(upload_inst(spec, d, s));
  PROF(F_CLUSTER, s);
  HIP_TRY(launch_cluster(n, table_of(d, spec.count()), rho, dep, delta, center_mode, delta_min,
                         rho_min, labels, is_center, gkey, flag, sel, s));
  return PECANN_OK;
}

extern "C" pecann_status pecann_cluster(int64_t n, const float *rho, const int32_t *dep,
                                        const float *delta, int32_t center_mode, int32_t n_c,
                                        float delta_min, float rho_min, int32_t *labels,
                                        uint8_t *is_center, void *ws, size_t ws_bytes, void *stream) {
  clear_stale_error();
  if (n < 1 || n >= (int64_t)1 << 31) return fail(PECANN_EINVAL, "n out of range");
  if (center_mode == PECANN_CENTER_PRODUCT && (n_c < 1 || n_c > n))
    return fail(PECANN_EINVAL, "n_c must be in [1, n]");
  return check_device(cluster_impl(n, single_spec(n, 1, n_c), rho, dep, delta, center_mode, delta_min, rho_min,
                      labels, is_center, ws, ws_bytes, stream));
}

extern "C" pecann_status pecann_cluster_batched(int64_t n, const pecann_instances *inst,
                                                const float *rho, const int32_t *dep,
                                                const float *delta, int32_t center_mode,
                                                int32_t n_c, float delta_min, float rho_min,
                                                int32_t *labels, uint8_t *is_center, void *ws,
                                                size_t ws_bytes, void *stream) {
  clear_stale_error();
  if (n < 2 || n >= (int64_t)1 << 31) return fail(PECANN_EINVAL, "n out of range");
  InstSpec sp;
  pecann_status st = make_spec(n, inst, 1, n_c, &sp);
  if (st != PECANN_OK) return st;
  return check_device(cluster_impl(n, sp, rho, dep, delta, center_mode, delta_min, rho_min, labels, is_center, ws,
                      ws_bytes, stream));
}

// ---------------------------------------------------------------------------
// pecann_cluster without a workspace argument.  Its scratch (the gamma keys,
// the pointer-jumping flag, the wide select's state, a one-instance table)
// lives in a file-scope
// device array: every GPU the library runs on holds its own copy until the
// process ends.  The array's name is a host-side stand-in in host code, so the
// device address is looked up once per device and only that address is used.
// ---------------------------------------------------------------------------
static constexpr int64_t kNoAllocMaxN = (int64_t)1 << 21;
static constexpr size_t kScratchBytes = (size_t)kNoAllocMaxN * 8 + 4096;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static pecann_status scratch_of_current_device(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PECANN_EUNSUPPORTED, "device %d is beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PECANN_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PECANN_OK;
}

extern "C" pecann_status pecann_cluster_noalloc(int64_t n, const float *rho, const int32_t *dep,
                                                const float *delta, int32_t center_mode, int32_t n_c,
                                                float delta_min, float rho_min, int32_t *labels,
                                                uint8_t *is_center, void *stream) {
  clear_stale_error();
  if (n < 1 || n > kNoAllocMaxN)
    return fail(PECANN_EINVAL, "n must be in [1, %lld] (the no-allocation entry point's fixed scratch)",
                (long long)kNoAllocMaxN);
  if (!rho || !dep || !delta || !labels || !is_center) return fail(PECANN_EINVAL, "pointer is NULL");
  if (center_mode != PECANN_CENTER_PRODUCT && center_mode != PECANN_CENTER_THRESHOLD &&
      center_mode != PECANN_CENTER_GIVEN)
    return fail(PECANN_EINVAL, "center_mode");
  if (center_mode == PECANN_CENTER_PRODUCT && (n_c < 1 || n_c > n))
    return fail(PECANN_EINVAL, "n_c must be in [1, n]");
  void *base = nullptr;
  pecann_status st = scratch_of_current_device(&base);
  if (st != PECANN_OK) return st;
  Carver c(base);
  uint64_t *gkey = c.take<uint64_t>((size_t)n);
  int32_t *flag = c.take<int32_t>(64);
  uint32_t *sel = c.take<uint32_t>(kSelWords);  // wide center-select state
  InstDev d;
  carve_inst(c, 1, &d);
  if (c.size() > kScratchBytes) return fail(PECANN_EWORKSPACE, "scratch layout exceeds the array");
  hipStream_t s = (hipStream_t)stream;
  // the table of one instance goes through kernel arguments (no host buffer)
  I64Chunk off;
  off.v[0] = 0;
  off.v[1] = n;
  I32Chunk kk, nc;
  kk.v[0] = 1;
  nc.v[0] = n_c;
  HIP_TRY(launch_fill_i32(flag, 0, 1, s));  // left set by the last call
  HIP_TRY(launch_put_i64(off, 2, d.off, s));
  HIP_TRY(launch_put_i32(kk, 1, d.k, s));
  HIP_TRY(launch_put_i32(nc, 1, d.nc, s));
  HIP_TRY(launch_cluster(n, table_of(d, 1), rho, dep, delta, center_mode, delta_min, rho_min, labels,
                         is_center, gkey, flag, sel, s));
  return PECANN_OK;
}

// ---------------------------------------------------------------------------
// Other density functions and local centers (epilogues over the kNN lists)
// ---------------------------------------------------------------------------
static size_t table_ws_size(int ninst) {
  Carver c(nullptr);
  InstDev d;
  carve_inst(c, ninst, &d);
  return c.size();
}

// inst NULL: one instance of n points with the call's k.
static pecann_status spec_or_single(int64_t n, const pecann_instances *inst, int32_t k, InstSpec *sp) {
  if (n < 2 || n >= (int64_t)1 << 31) return fail(PECANN_EINVAL, "n out of range");
  if (!inst) {
    *sp = single_spec(n, k, 1);
    return PECANN_OK;
  }
  return make_spec(n, inst, k, 1, sp);
}

extern "C" size_t pecann_density_workspace_size(int64_t n, const pecann_instances *inst) {
  InstSpec sp;
  if (spec_or_single(n, inst, 1, &sp) != PECANN_OK) return 0;
  return table_ws_size(sp.count());
}

extern "C" pecann_status pecann_density(int64_t n, const pecann_instances *inst, int32_t k,
                                        int32_t density_fn, const int32_t *knn_idx,
                                        const float *knn_dist, float *rho, uint64_t *rank_key,
                                        void *ws, size_t ws_bytes, void *stream) {
  clear_stale_error();
  InstSpec sp;
  pecann_status st = spec_or_single(n, inst, k, &sp);
  if (st != PECANN_OK) return st;
  if ((st = check_inst_k(sp, k)) != PECANN_OK) return st;
  if (density_fn < PECANN_DENSITY_KTH || density_fn > PECANN_DENSITY_SUM)
    return fail(PECANN_EINVAL, "density_fn");
  if (!knn_idx || !knn_dist || !rho || !rank_key) return fail(PECANN_EINVAL, "pointer is NULL");
  const size_t need = table_ws_size(sp.count());
  if (!ws || ws_bytes < need || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", need, ws_bytes);
  Carver c(ws);
  InstDev d;
  carve_inst(c, sp.count(), &d);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(upload_inst(sp, d, s));
  PROF(F_OTHER, s);
  HIP_TRY(launch_density(n, table_of(d, sp.count()), k, density_fn, knn_idx, knn_dist, rho, rank_key, s));
  return PECANN_OK;
}

extern "C" size_t pecann_local_centers_workspace_size(int64_t n, const pecann_instances *inst) {
  return pecann_density_workspace_size(n, inst);
}

extern "C" pecann_status pecann_local_centers(int64_t n, const pecann_instances *inst, int32_t k,
                                              const int32_t *knn_idx, const uint64_t *rank_key,
                                              const float *rho, float rho_min, uint8_t *is_center,
                                              void *ws, size_t ws_bytes, void *stream) {
  clear_stale_error();
  InstSpec sp;
  pecann_status st = spec_or_single(n, inst, k, &sp);
  if (st != PECANN_OK) return st;
  if ((st = check_inst_k(sp, k)) != PECANN_OK) return st;
  if (!knn_idx || !rank_key || !rho || !is_center) return fail(PECANN_EINVAL, "pointer is NULL");
  const size_t need = table_ws_size(sp.count());
  if (!ws || ws_bytes < need || !aligned(ws, 256))
    return fail(PECANN_EWORKSPACE, "workspace needs %zu bytes (256-aligned), got %zu", need, ws_bytes);
  Carver c(ws);
  InstDev d;
  carve_inst(c, sp.count(), &d);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(upload_inst(sp, d, s));
  PROF(F_CLUSTER, s);
  HIP_TRY(launch_local_centers(n, table_of(d, sp.count()), k, knn_idx, rank_key, rho, rho_min,
                               is_center, s));
  return PECANN_OK;
}

// ---------------------------------------------------------------------------
// Measurement aid
// ---------------------------------------------------------------------------
extern "C" pecann_status pecann_read_probe(const void *buf, size_t bytes, int32_t passes,
                                           uint32_t key, uint32_t *sink, void *stream) {
  clear_stale_error();
  if (!buf || !sink) return fail(PECANN_EINVAL, "buf/sink are NULL");
  if (bytes == 0 || bytes % 16 != 0 || !aligned(buf, 16))
    return fail(PECANN_EINVAL, "bytes must be a positive multiple of 16 and buf 16-byte aligned");
  if (passes < 1) return fail(PECANN_EINVAL, "passes must be >= 1");
  HIP_TRY(launch_read_probe(buf, (int64_t)bytes, passes, key, sink, cu_count() * 16,
                            (hipStream_t)stream));
  return PECANN_OK;
}
