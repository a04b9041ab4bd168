// K8/K9 RobustPrune of DiskANN (the Vamana pruning rule the paper adopts,
// Sec. 3.2), one wavefront per pruned point:
//   sort the candidates by (D(p, c), c), drop p, duplicates and -1;
//   repeatedly move the closest surviving candidate c* to the output (stop at
//   R) and drop every surviving c with alpha * D(c*, c) <= D(p, c)
//   (alpha^2 * D^2 <= D^2 for L2 measures, which are squared distances).
// prune_forward: Nout(p) = RobustPrune(p, V_p u Nout(p)) for each point of a batch.
// prune_reverse: for each target q of the batch's reverse edges, append the
//   new sources not yet present (ascending index) if they fit in R, else
//   Nout(q) = RobustPrune(q, Nout(q) u sources).
#include "beam.hpp"

namespace pecann {

namespace {

struct PruneLds {
  int32_t *ids;    // candidates [ccap]
  uint64_t *k0;    // keys [ccap]
  uint64_t *k1;    // sorted keys [ccap]
  int32_t *list;   // compacted survivor positions [ccap]
  int32_t *sel;    // selected [R]
  uint8_t *alive;  // [ccap]
};

__device__ __forceinline__ PruneLds carve_prune(uint8_t *smem, int ccap, int R) {
  PruneLds s;
  s.k0 = (uint64_t *)smem;
  s.k1 = s.k0 + ccap;
  s.ids = (int32_t *)(s.k1 + ccap);
  s.list = s.ids + ccap;
  s.sel = s.list + ccap;
  s.alive = (uint8_t *)(s.sel + ((R + 3) & ~3));
  return s;
}

// Stable rank sort of cnt keys that may repeat.
__device__ __forceinline__ void rank_sort_dups(const uint64_t *src, uint64_t *dst, int cnt) {
  for (int j = lane_id(); j < cnt; j += kWave) {
    const uint64_t key = src[j];
    int r = 0;
    for (int t = 0; t < cnt; ++t) {
      const uint64_t o = src[t];
      r += (o < key) | ((o == key) & (t < j));
    }
    dst[r] = key;
  }
  wave_lds_sync();
}

// RobustPrune of point pt over s.ids[0..nc); writes Nout(pt) into adj/deg.
// Returns the number of rows gathered for distances.
template <int DT, int G>
__device__ int robust_prune_wave(const PruneParams &p, Engine<DT, G> &eng, PruneLds &s, int32_t pt,
                                 int nc) {
  constexpr int NPL = Engine<DT, G>::NPL;
  const int l = lane_id();
  const int grp = l / G;
  const bool leader = (l % G) == 0;
  const float a2 = p.rows.metric == PECANN_L2 ? p.alpha * p.alpha : p.alpha;

  eng.load_query(p.rows, pt);
  for (int base = 0; base < nc; base += NPL) {
    const int ci = base + grp;
    int32_t id = ci < nc ? s.ids[ci] : -1;
    if (id == pt) id = -1;
    const float m = eng.measure(p.rows, id);
    if (leader && ci < nc) s.k0[ci] = id >= 0 ? make_key(m, id) : kNoKey;
  }
  wave_lds_sync();
  rank_sort_dups(s.k0, s.k1, nc);
  for (int j = l; j < nc; j += kWave) {
    const uint64_t key = s.k1[j];
    s.alive[j] = (key != kNoKey) && (j == 0 || s.k1[j - 1] != key);
  }
  wave_lds_sync();

  int nsel = 0;
  int from = 0;
  int rows = nc;
  while (nsel < p.R) {
    // first survivor at or after `from`
    int j = -1;
    for (int base = from; base < nc; base += kWave) {
      const int u = base + l;
      const uint64_t bm = ballot(u < nc && s.alive[u]);
      if (bm) { j = base + __builtin_ctzll(bm); break; }
    }
    if (j < 0) break;
    const int32_t cstar = key_id(s.k1[j]);
    if (l == 0) { s.sel[nsel] = cstar; s.alive[j] = 0; }
    ++nsel;
    wave_lds_sync();
    if (nsel == p.R) break;
    // survivors after j
    int cnt = 0;
    for (int base = j + 1; base < nc; base += kWave) {
      const int u = base + l;
      const bool a = u < nc && s.alive[u];
      const uint64_t bm = ballot(a);
      if (a) s.list[cnt + lanes_below(bm)] = u;
      cnt += __popcll(bm);
    }
    wave_lds_sync();
    if (cnt > 0) {
      rows += cnt;
      eng.load_query(p.rows, cstar);
      for (int base = 0; base < cnt; base += NPL) {
        const int ci = base + grp;
        const int u = ci < cnt ? s.list[ci] : -1;
        const int32_t row = u >= 0 ? key_id(s.k1[u]) : -1;
        const float m = eng.measure(p.rows, row);
        if (leader && u >= 0 && a2 * m <= key_measure(s.k1[u])) s.alive[u] = 0;
      }
      wave_lds_sync();
    }
    from = j + 1;
  }
  int32_t *row = p.adj + (int64_t)pt * p.R;
  for (int e = l; e < p.R; e += kWave) row[e] = e < nsel ? s.sel[e] : -1;
  if (l == 0) p.deg[pt] = nsel;
  return rows;
}

}  // namespace

template <int DT, int G>
__global__ __launch_bounds__(64) void prune_forward_kernel(PruneParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int ccap = p.vcap + p.R;
  PruneLds s = carve_prune(smem, ccap, p.R);
  Engine<DT, G> eng;
  const int l = lane_id();
  for (;;) {
    const int t = next_item(p.head);
    if (t >= p.nb) break;
    const int32_t pt = p.perm[p.b0 + t];
    // candidates: the visited set V_p, then the current out-neighbours Nout(p)
    const int nv = min(p.vis_count[t], p.vcap);
    const uint64_t *v = p.vis + (int64_t)t * p.vcap;
    for (int j = l; j < nv; j += kWave) s.ids[j] = key_id(v[j]);
    const int dp = min(p.deg[pt], p.R);
    const int32_t *row = p.adj + (int64_t)pt * p.R;
    for (int j = l; j < dp; j += kWave) s.ids[nv + j] = row[j];
    wave_lds_sync();
    const int rows = robust_prune_wave<DT, G>(p, eng, s, pt, nv + dp);
    if (p.counters && l == 0) atomicAdd(p.counters + 0, (unsigned long long)rows);
    wave_lds_sync();
  }
}

template <int DT, int G>
__global__ __launch_bounds__(64) void prune_reverse_kernel(PruneParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int ccap = p.R + p.capin;
  PruneLds s = carve_prune(smem, ccap, p.R);
  Engine<DT, G> eng;
  const int l = lane_id();
  const int nt = *p.ntargets;
  for (;;) {
    const int u = next_item(p.head);
    if (u >= nt) break;
    const int32_t q = p.tlist[u];
    int cnt = p.tcnt[u];
    if (cnt > p.capin) {
      if (l == 0) atomicAdd(p.overflow, 1);
      cnt = p.capin;
    }
    const int32_t *src = p.seg + p.toff[u];
    const int dq = min(p.deg[q], p.R);
    int32_t *row = p.adj + (int64_t)q * p.R;
    // current out-neighbours, then the new sources in ascending index order,
    // leaving out sources already among the out-neighbours
    for (int j = l; j < dq; j += kWave) s.ids[j] = row[j];
    for (int j = l; j < cnt; j += kWave) {
      const int32_t v = src[j];
      int r = 0;
      for (int t = 0; t < cnt; ++t) r += src[t] < v;
      bool present = false;
      for (int t = 0; t < dq; ++t) present |= (row[t] == v);
      s.list[r] = present ? -1 : v;
    }
    wave_lds_sync();
    int nnew = 0;
    for (int base = 0; base < cnt; base += kWave) {
      const int j = base + l;
      const int32_t v = j < cnt ? s.list[j] : -1;
      const uint64_t bm = ballot(v >= 0);
      if (v >= 0) s.ids[dq + nnew + lanes_below(bm)] = v;
      nnew += __popcll(bm);
    }
    wave_lds_sync();
    if (dq + nnew <= p.R) {
      for (int j = l; j < nnew; j += kWave) row[dq + j] = s.ids[dq + j];
      if (l == 0) p.deg[q] = dq + nnew;
      if (p.counters && l == 0) atomicAdd(p.counters + 3, 1ull);
    } else {
      const int rows = robust_prune_wave<DT, G>(p, eng, s, q, dq + nnew);
      if (p.counters && l == 0) {
        atomicAdd(p.counters + 1, (unsigned long long)rows);
        atomicAdd(p.counters + 2, 1ull);
      }
    }
    if (l == 0) p.rcnt[q] = 0;
    wave_lds_sync();
  }
}

size_t prune_lds_bytes(int ccap, int R) {
  return (size_t)ccap * (8 + 8 + 4 + 4 + 1) + 4 * (size_t)((R + 3) & ~3) + 16;
}

template <int DT, int G>
static hipError_t launch_pf_t(const PruneParams &p, int grid, hipStream_t st) {
  hipLaunchKernelGGL((prune_forward_kernel<DT, G>), dim3(grid), dim3(64),
                     prune_lds_bytes(p.vcap + p.R, p.R), st, p);
  return hipGetLastError();
}
template <int DT, int G>
static hipError_t launch_pr_t(const PruneParams &p, int grid, hipStream_t st) {
  hipLaunchKernelGGL((prune_reverse_kernel<DT, G>), dim3(grid), dim3(64),
                     prune_lds_bytes(p.R + p.capin, p.R), st, p);
  return hipGetLastError();
}

#define PECANN_DISPATCH_G(FN, DT, ...)                      \
  switch (G) {                                              \
    case 4: return FN<DT, 4>(__VA_ARGS__);                  \
    case 8: return FN<DT, 8>(__VA_ARGS__);                  \
    case 16: return FN<DT, 16>(__VA_ARGS__);                \
    case 32: return FN<DT, 32>(__VA_ARGS__);                \
    case 64: return FN<DT, 64>(__VA_ARGS__);                \
    default: return hipErrorInvalidValue;                   \
  }

hipError_t launch_prune_forward(int32_t dt, int G, const PruneParams &p, int grid, hipStream_t st) {
  switch (dt) {
    case PECANN_F32: PECANN_DISPATCH_G(launch_pf_t, PECANN_F32, p, grid, st)
    case PECANN_U8: PECANN_DISPATCH_G(launch_pf_t, PECANN_U8, p, grid, st)
    case PECANN_BF16: PECANN_DISPATCH_G(launch_pf_t, PECANN_BF16, p, grid, st)
    case PECANN_FP8E4M3: PECANN_DISPATCH_G(launch_pf_t, PECANN_FP8E4M3, p, grid, st)
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_prune_reverse(int32_t dt, int G, const PruneParams &p, int grid, hipStream_t st) {
  switch (dt) {
    case PECANN_F32: PECANN_DISPATCH_G(launch_pr_t, PECANN_F32, p, grid, st)
    case PECANN_U8: PECANN_DISPATCH_G(launch_pr_t, PECANN_U8, p, grid, st)
    case PECANN_BF16: PECANN_DISPATCH_G(launch_pr_t, PECANN_BF16, p, grid, st)
    case PECANN_FP8E4M3: PECANN_DISPATCH_G(launch_pr_t, PECANN_FP8E4M3, p, grid, st)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pecann
