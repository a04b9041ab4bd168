// Exact (brute-force) kernels, float32 (or exact uint8) distances:
//   K1 bf_knn  -- exact k nearest neighbours of a list of queries over all points
//                 of their instance (the paper's BruteForce index, Sec. 4.1; also
//                 the fallback when a graph search returns fewer than k points),
//                 one wavefront per query, or split: a wavefront per (query,
//                 chunk of candidates) and a merge of the chunks' best keys, so
//                 that a short list of queries over many points is not one
//                 long serial scan per query;
//   K7 bf_dep  -- DPBruteForce(x_i, P) of Alg. 3 for the unfinished points: the
//                 closest point of strictly smaller rank key, split into chunks
//                 of candidates whose partial argmins meet in a 64-bit atomic min.
#include <type_traits>

#include "beam.hpp"

namespace pecann {

template <int DT, int S>
__global__ __launch_bounds__(64) void bf_knn_kernel(BfKnnParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int kp = (p.k + 15) & ~15;  // p.k: the largest k of any instance
  SortedList top;
  top.a = (uint64_t *)smem;
  top.b = top.a + kp;
  top.tmp = top.b + kp;
  uint64_t *kb = top.tmp + 64;  // keys of the current 64 candidates
  top.fa = (uint8_t *)(kb + 64);
  top.fb = top.fa + kp;
  ExactEngine<DT, S> eng;
  const int l = lane_id();
  const int count = p.item_count ? *p.item_count : p.nitems;
  for (;;) {
    const int it = next_item(p.head) + p.item_from;
    if (it >= count) break;
    const int32_t qid = p.items ? p.items[it] : it;
    const int ti = find_instance(p.inst, qid);
    const int32_t lo = (int32_t)p.inst.off[ti], hi = (int32_t)p.inst.off[ti + 1];
    if (hi - lo >= p.skip_from) continue;  // searched by another path
    const int k = p.inst.k[ti];
    top.cap = k;
    eng.load_query(p.rows, qid);
    top.reset();
    wave_lds_sync();
    for (int base = lo; base < hi; base += kWave) {
      const int c = min(kWave, hi - base);
      score_keys(eng, p.rows, c, [&](int i) { return base + i == qid ? -1 : base + i; }, kb);
      wave_lds_sync();
      const uint64_t key = l < c ? kb[l] : kNoKey;
      wave_lds_sync();
      top.merge(key);
    }
    const int64_t o = (int64_t)qid * p.kstride;
    for (int t = l; t < p.kstride; t += kWave) {
      const uint64_t kt = t < k ? top.a[t] : kNoKey;
      p.knn_idx[o + t] = t < k ? key_id(kt) : -1;
      p.knn_dist[o + t] = t < k ? measure_to_dist(key_measure(kt), p.rows.metric)
                                : __int_as_float(0x7f800000);
    }
    if (l == 0) {
      const uint64_t kk = top.a[k - 1];
      p.rho[qid] = 1.0f / measure_to_dist(key_measure(kk), p.rows.metric);
      p.rank_key[qid] = (kk & 0xffffffff00000000ull) | (uint32_t)qid;
    }
    wave_lds_sync();
  }
}

// The writes of one query's k best keys (and its density and rank key) from a
// sorted list holding at least k of them.
__device__ __forceinline__ void write_knn(const BfKnnParams &p, const SortedList &top, int32_t qid, int k) {
  const int l = lane_id();
  const int64_t o = (int64_t)qid * p.kstride;
  for (int t = l; t < p.kstride; t += kWave) {
    const uint64_t kt = t < k ? top.a[t] : kNoKey;
    p.knn_idx[o + t] = t < k ? key_id(kt) : -1;
    p.knn_dist[o + t] = t < k ? measure_to_dist(key_measure(kt), p.rows.metric) : __int_as_float(0x7f800000);
  }
  if (l == 0) {
    const uint64_t kk = top.a[k - 1];
    p.rho[qid] = 1.0f / measure_to_dist(key_measure(kk), p.rows.metric);
    p.rank_key[qid] = (kk & 0xffffffff00000000ull) | (uint32_t)qid;
  }
}

// Split path, part 1: the k best keys of one chunk of one query's candidates.
template <int DT, int S>
__global__ __launch_bounds__(64) void bf_knn_chunk_kernel(BfKnnParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int kp = (p.k + 15) & ~15;
  SortedList top;
  top.a = (uint64_t *)smem;
  top.b = top.a + kp;
  top.tmp = top.b + kp;
  uint64_t *kb = top.tmp + 64;
  top.fa = (uint8_t *)(kb + 64);
  top.fb = top.fa + kp;
  ExactEngine<DT, S> eng;
  const int l = lane_id();
  const int count = min(p.item_count ? *p.item_count : p.nitems, p.split_cap);
  const int total = count * p.nchunk;
  for (;;) {
    const int it = next_item(p.head);
    if (it >= total) break;
    const int slot = it / p.nchunk, ch = it - slot * p.nchunk;
    const int32_t qid = p.items ? p.items[slot] : slot;
    const int ti = find_instance(p.inst, qid);
    const int32_t lo = (int32_t)p.inst.off[ti], hi = (int32_t)p.inst.off[ti + 1];
    const int32_t c0 = lo + ch * p.chunk, c1 = min(hi, c0 + p.chunk);
    top.cap = p.inst.k[ti];
    top.reset();
    wave_lds_sync();
    if (c0 < c1) {
      eng.load_query(p.rows, qid);
      for (int base = c0; base < c1; base += kWave) {
        const int c = min(kWave, c1 - base);
        score_keys(eng, p.rows, c, [&](int i) { return base + i == qid ? -1 : base + i; }, kb);
        wave_lds_sync();
        const uint64_t key = l < c ? kb[l] : kNoKey;
        wave_lds_sync();
        top.merge(key);
      }
    }
    uint64_t *out = p.part + ((int64_t)slot * p.nchunk + ch) * p.kpart;
    for (int t = l; t < p.kpart; t += kWave) out[t] = t < top.m ? top.a[t] : kNoKey;
    wave_lds_sync();
  }
}

// Split path, part 2: one wavefront per query merges its chunks' keys (the
// candidates of different chunks are different points, so the keys are
// distinct) and writes the query's k nearest neighbours.
__global__ __launch_bounds__(64) void bf_knn_merge_kernel(BfKnnParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int kp = (p.k + 15) & ~15;
  SortedList top;
  top.a = (uint64_t *)smem;
  top.b = top.a + kp;
  top.tmp = top.b + kp;
  top.fa = (uint8_t *)(top.tmp + 128);
  top.fb = top.fa + kp;
  const int l = lane_id();
  const int count = min(p.item_count ? *p.item_count : p.nitems, p.split_cap);
  const int tot = p.nchunk * p.kpart;
  for (;;) {
    const int slot = next_item(p.head2);
    if (slot >= count) break;
    const int32_t qid = p.items ? p.items[slot] : slot;
    const int ti = find_instance(p.inst, qid);
    const int k = p.inst.k[ti];
    top.cap = k;
    top.reset();
    wave_lds_sync();
    const uint64_t *src = p.part + (int64_t)slot * tot;
    for (int base = 0; base < tot; base += kWave) {
      const uint64_t key = base + l < tot ? src[base + l] : kNoKey;
      top.merge(key);
    }
    write_knn(p, top, qid, k);
    wave_lds_sync();
  }
}

size_t bf_knn_lds_bytes(int k) {
  const size_t kp = (size_t)((k + 15) & ~15);
  return 8 * (2 * kp + 128) + 2 * kp;
}

template <int DT, int S>
__global__ __launch_bounds__(64) void bf_dep_kernel(BfDepParams p) {
  __shared__ int32_t cidx[64];
  __shared__ uint64_t kb[64];
  ExactEngine<DT, S> eng;
  const int l = lane_id();
  const int count = *p.ucount;
  const int total = count * p.nchunks;
  for (;;) {
    const int it = next_item(p.head);
    if (it >= total) break;
    const int u = it / p.nchunks;
    const int ch = it - u * p.nchunks;
    const int32_t qid = p.ulist[u];
    PECANN_CHECK(qid >= 0 && qid < p.n, CK_ITEM);
    const int ti = find_instance(p.inst, qid);
    const int32_t lo = (int32_t)p.inst.off[ti], hi = (int32_t)p.inst.off[ti + 1];
    PECANN_CHECK(lo <= qid && qid < hi, CK_INSTANCE);
    const int j0 = lo + ch * p.chunk;
    if (j0 >= hi) continue;  // beyond this instance
    const int j1 = min(hi, j0 + p.chunk);
    const uint64_t ki = p.key[qid];
    eng.load_query(p.rows, qid);
    uint64_t best = kNoKey;
    for (int base = j0; base < j1; base += kWave) {
      const int j = base + l;
      const bool ok = j < j1 && p.key[j] < ki;
      const uint64_t bm = ballot(ok);
      if (bm == 0) continue;
      const int c = __popcll(bm);
      if (ok) cidx[lanes_below(bm)] = j;
      wave_lds_sync();
      score_keys(eng, p.rows, c, [&](int i) { return cidx[i]; }, kb);
      wave_lds_sync();
      if (l < c && kb[l] < best) best = kb[l];
      wave_lds_sync();
    }
    best = wave_min_u64(best);
    if (l == 0 && best != kNoKey) atomicMin(&p.best[u], (unsigned long long)best);
  }
}

template <int DT, int S>
static hipError_t launch_bf_knn_t(const BfKnnParams &p, int grid, hipStream_t st) {
  if constexpr (S > max_shape(DT)) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((bf_knn_kernel<DT, S>), dim3(grid), dim3(64), bf_knn_lds_bytes(p.k), st, p);
    return hipGetLastError();
  }
}
template <int DT, int S>
static hipError_t launch_bf_dep_t(const BfDepParams &p, int grid, hipStream_t st) {
  if constexpr (S > max_shape(DT)) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((bf_dep_kernel<DT, S>), dim3(grid), dim3(64), 0, st, p);
    return hipGetLastError();
  }
}

hipError_t launch_bf_knn(int32_t dt, int S, const BfKnnParams &p, int grid, hipStream_t st) {
  PECANN_DISPATCH_SHAPE(launch_bf_knn_t, dt, S, p, grid, st)
}

template <int DT, int S>
static hipError_t launch_bf_knn_split_t(const BfKnnParams &p, int grid_chunks, int grid_merge,
                                        hipStream_t st) {
  if constexpr (S > max_shape(DT)) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((bf_knn_chunk_kernel<DT, S>), dim3(grid_chunks), dim3(64), bf_knn_lds_bytes(p.k), st,
                       p);
    hipLaunchKernelGGL(bf_knn_merge_kernel, dim3(grid_merge), dim3(64), bf_knn_lds_bytes(p.k), st, p);
    return hipGetLastError();
  }
}

hipError_t launch_bf_knn_split(int32_t dt, int S, const BfKnnParams &p, int grid_chunks, int grid_merge,
                               hipStream_t st) {
  PECANN_DISPATCH_SHAPE(launch_bf_knn_split_t, dt, S, p, grid_chunks, grid_merge, st)
}

hipError_t launch_bf_dep(int32_t dt, int S, const BfDepParams &p, int grid, hipStream_t st) {
  PECANN_DISPATCH_SHAPE(launch_bf_dep_t, dt, S, p, grid, st)
}

PECANN_CHECK_READER(bruteforce)

}  // namespace pecann
