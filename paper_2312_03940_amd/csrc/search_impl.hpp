// K2 greedy beam search (Alg. 1), one wavefront per query, persistent over a
// device work queue (shared by search.hip and search_mfma.hip, which
// instantiate the vector-unit and the matrix-core scoring variants).  Three epilogues share the walk:
//   MODE_KNN   kNN + kth density of a point (Alg. 2 Find-Knn / F_density),
//   MODE_DEP   one doubling round of ComputeDepPts (Alg. 3),
//   MODE_BUILD the search of a batched Vamana insertion (visited set V).
//
// LDS per wavefront: two beam buffers of L keys + flags, 64 keys of merge
// scratch, 64 ids of distance work, the visited hash and, for BF16/FP8 rows,
// the two parts of the query the matrix cores multiply.
//
// Candidates are scored on the vector units (one fused difference-square per
// element, after a decode for BF16 / FP8 rows) or, for BF16 and FP8 rows, on
// the matrix cores (mfma_score.hpp, template flag MF), where the vector units
// would spend most of their issue slots on decoding and multiply-adds over
// long rows.
#pragma once

#include <type_traits>

#include "beam.hpp"
#include "mfma_score.hpp"

namespace pecann {

namespace {

struct Lds {
  SortedList beam;
  IdHash hash;
  int32_t *cid;  // 64 ids awaiting distances
  uint8_t *qp;   // query parts of the matrix-core scorer (BF16/FP8 rows)
  // wave-uniform work tallies of the current query
  unsigned long long n_exp, n_ids, n_rows;
};

__device__ __forceinline__ Lds carve(uint8_t *smem, int L, int hbits, int hid_bits) {
  Lds s;
  uint64_t *p = (uint64_t *)smem;
  s.beam.a = p;
  s.beam.b = p + L;
  s.beam.tmp = p + 2 * L;
  s.cid = (int32_t *)(p + 2 * L + 64);
  uint8_t *f = (uint8_t *)(s.cid + 64);
  const int Lp = (L + 15) & ~15;
  s.beam.fa = f;
  s.beam.fb = f + Lp;
  s.hash.slot = (int32_t *)(f + 2 * Lp);
  s.hash.bits = hbits;
  if (hid_bits) {
    s.hash.rb = hid_bits - (hbits - 2);
    s.hash.kmask = hid_bits >= 32 ? ~0u : (1u << hid_bits) - 1u;
  }
  s.qp = (uint8_t *)s.hash.slot + (hid_bits ? 2 : 4) * (1 << hbits);
  s.beam.cap = L;
  s.beam.reset();
  s.n_exp = s.n_ids = s.n_rows = 0;
  return s;
}

// Distances for the ids given one per lane (-1 = none), then merge into the beam.
// score(c, id_of, out) writes the keys of candidates id_of(0 .. c) to out.
template <class F>
__device__ __forceinline__ void score_and_merge(F &score, Lds &s, int32_t myid) {
  const int l = lane_id();
  const uint64_t bm = ballot(myid >= 0);
  const int c = __popcll(bm);
  if (c == 0) return;
  s.n_rows += c;
  if (myid >= 0) s.cid[lanes_below(bm)] = myid;
  wave_lds_sync();
  score(c, [&](int i) { return s.cid[i]; }, s.beam.tmp);
  wave_lds_sync();
  const uint64_t key = l < c ? s.beam.tmp[l] : kNoKey;
  wave_lds_sync();
  s.beam.merge(key);
}

// Add the out-neighbours of point v to the beam (ids seen before are skipped).
template <class F>
__device__ __forceinline__ void expand(F &score, const SearchParams &p, Lds &s, int32_t v) {
  const int32_t *row = p.adj + (int64_t)v * p.R;
  // the degree and the first 64 entries of the row are loaded together (the
  // row always has R entries), so the expansion costs one memory round trip
  const int e_first = lane_id();
  const int32_t nb_first = e_first < p.R ? row[e_first] : -1;
  PECANN_CHECK(p.deg[v] >= 0 && p.deg[v] <= p.R, CK_NEIGHBOUR);
  const int dg = min(p.deg[v], p.R);
  s.n_exp += 1;
  s.n_ids += dg;
  for (int e0 = 0; e0 < dg; e0 += kWave) {
    const int e = e0 + lane_id();
    int32_t nb = e < dg ? (e0 == 0 ? nb_first : row[e]) : -1;
    PECANN_CHECK(nb < p.n, CK_NEIGHBOUR);
    if (nb >= p.n) nb = -1;  // ids outside the point set are ignored
    if (nb >= 0 && !s.hash.insert(nb)) nb = -1;
    score_and_merge(score, s, nb);
  }
}

// The expanded points of an insertion's search (V_p), at most `cap` of them:
// once the slot is full, a newly expanded point replaces the farthest kept one
// when it is closer, so the slot ends with the `cap` closest by (D, index).
// (An expanded point is never expanded again: it either stays in the beam or
// was pushed out by closer keys and can never re-enter, so the keys are
// distinct.)  Entry e is written and read by lane e % 64 only, so each lane
// reads back its own stores.
struct VisitedSlot {
  uint64_t *v;
  int cap;
  int n;        // points expanded so far (may exceed cap)
  uint64_t mx;  // largest kept key, once the slot is full
  int mpos;     // its entry

  __device__ __forceinline__ void find_max() {
    const int l = lane_id();
    uint64_t best = 0;
    int bp = -1;
    for (int e = l; e < cap; e += kWave) {
      const uint64_t k = v[e];
      if (bp < 0 || k > best) { best = k; bp = e; }
    }
    mx = ~wave_min_u64(~best);
    const uint64_t who = ballot(bp >= 0 && best == mx);
    mpos = __shfl(bp, __builtin_ctzll(who));
  }

  // every lane calls with the same key
  __device__ __forceinline__ void add(uint64_t key) {
    const int l = lane_id();
    if (n < cap) {
      if (l == (n & (kWave - 1))) v[n] = key;
      if (++n == cap) find_max();
      return;
    }
    ++n;
    if (key >= mx) return;
    if (l == (mpos & (kWave - 1))) v[mpos] = key;
    find_max();
  }
};

// Re-score the first r beam entries from float32 rows and sort them (into beam.a).
template <int SR>
__device__ __forceinline__ void rerank_beam(const SearchParams &p, Lds &s, int32_t qid, int r) {
  Engine32<SR> e32;
  e32.load_query(p.rows, qid);
  const uint64_t *a = s.beam.a;
  score_keys(e32, p.rows, r, [&](int i) { return key_id(a[i]); }, s.beam.b);
  wave_lds_sync();
  lds_rank_sort(s.beam.b, s.beam.a, r);
}

}  // namespace

template <int DT, int S, int MODE, bool MF>
__device__ __forceinline__ void search_body(const SearchParams &p) {
  extern __shared__ __align__(16) uint8_t smem[];
  Lds s = carve(smem, p.L, p.hbits, p.hid_bits);
  const int l = lane_id();
  const int count = p.item_count ? *p.item_count : p.nitems;
  constexpr bool kNeedRerank = (DT == PECANN_BF16 || DT == PECANN_FP8E4M3 || DT == PECANN_MXFP6);
  // MXFP6 rows are scored on the matrix cores only; the vector-unit types below
  // are then those of the FP8 copy and go unused
  constexpr int DTE = DT == PECANN_MXFP6 ? PECANN_FP8E4M3 : DT;


  // build searches over float32 rows of 64 chunks or more run at most two
  // waves per SIMD anyway (their beam and visited hash fill the LDS), so they
  // spend the spare registers on twice the row loads in flight (784-d rows:
  // 190 -> 186 ms per step; the FP8 and BF16 builds, whose time goes to
  // decoding and FMAs, gained nothing)
  constexpr int kLc = (DT == PECANN_F32 && MODE == MODE_BUILD && S >= 64) ? 32 : 0;
  Engine<DTE, S, false, kLc> eng;
  constexpr bool kMfma = MF && (DT == PECANN_BF16 || DT == PECANN_FP8E4M3 || DT == PECANN_MXFP6);
  static_assert(DT != PECANN_MXFP6 || kMfma, "MXFP6 rows need the matrix-core scorer");
  using Scorer = typename std::conditional<kMfma, MfmaScorer<kMfma ? DT : PECANN_BF16, S>, int>::type;
  Scorer msc{};
  if constexpr (kMfma) msc.qp = s.qp;
  auto score = [&](int c, auto id_of, uint64_t *out) {
    if constexpr (kMfma) msc.score(p.rows, c, id_of, out);
    else score_keys(eng, p.rows, c, id_of, out);
  };
  constexpr int SR = RerankShape<DTE, S>::v;
  for (;;) {
    const int it = next_item(p.head);
    if (it >= count) break;
    const int32_t qid = p.items ? p.items[it] : it;
    PECANN_CHECK(qid >= 0 && qid < p.n, CK_ITEM);
    int ti = 0;  // the query's instance
    if (MODE != MODE_BUILD) {
      ti = find_instance(p.inst, qid);
      PECANN_CHECK(p.inst.off[ti] <= qid && qid < p.inst.off[ti + 1], CK_INSTANCE);
    }
    if (MODE == MODE_DEP) {
      // this instance's doubling has ended (few enough points left, or k_dep
      // beyond its limit): carry the point over to the next list unchanged
      const int64_t nt = p.inst.off[ti + 1] - p.inst.off[ti];
      const int64_t lim = min((int64_t)p.kdep_cap, nt - 1);
      if (p.ucnt_in[ti] <= p.threshold || p.kdep > lim) {
        if (l == 0) {
          p.u_out[atomicAdd(p.u_out_count, 1)] = qid;
          atomicAdd(p.ucnt_out + ti, 1);
        }
        continue;
      }
    }

    s.hash.clear();
    s.beam.reset();
    wave_lds_sync();
    if constexpr (kMfma) msc.prepare(p.rows, qid);
    else eng.load_query(p.rows, qid);
    if (l == 0) s.hash.insert(qid);  // the query never takes a beam slot
    wave_lds_sync();

    // S = {query} u starts, or S = starts for an insertion.  A query that is
    // itself a start is expanded at once (it never takes a beam slot).
    const int32_t *starts = p.item_sbase ? p.starts + p.item_sbase[it] : p.starts;
    const int nstarts = p.item_ns ? p.item_ns[it] : p.nstarts;
    bool self_start = (MODE != MODE_BUILD);
    for (int s0 = 0; s0 < nstarts && !self_start; s0 += kWave)
      self_start = ballot(s0 + l < nstarts && starts[s0 + l] == qid) != 0;
    if (self_start) expand(score, p, s, qid);
    for (int s0 = 0; s0 < nstarts; s0 += kWave) {
      int32_t id = s0 + l < nstarts ? starts[s0 + l] : -1;
      if (id >= 0 && !s.hash.insert(id)) id = -1;
      score_and_merge(score, s, id);
    }

    VisitedSlot vs{MODE == MODE_BUILD ? p.vis + (int64_t)it * p.vcap : nullptr, p.vcap, 0, 0, 0};
    for (;;) {
      uint64_t kj = kNoKey;
      const int j = s.beam.first_unflagged(kj);
      if (j < 0) break;
      if (l == 0) s.beam.fa[j] = 1;
      if (MODE == MODE_BUILD) vs.add(kj);
      wave_lds_sync();
      expand(score, p, s, key_id(kj));
    }
    const int nv = vs.n;

    const int m = s.beam.m;
#ifdef PECANN_CHECKED
    // the beam holds at most L keys, strictly increasing
    PECANN_CHECK(m <= s.beam.cap, CK_BEAM);
    for (int j = l; j + 1 < m; j += kWave) PECANN_CHECK(s.beam.a[j] < s.beam.a[j + 1], CK_BEAM);
#endif
    unsigned long long n_rerank = 0;
    if (MODE == MODE_BUILD) {
      if (l == 0) p.vis_count[it] = nv;
      n_rerank = nv > p.vcap;  // build counter [3]: searches whose V_p was capped
    } else if (MODE == MODE_KNN) {
      const int k = p.inst.k[ti];
      int mm = m;
      if (kNeedRerank && m > 0) {
        mm = min(m, p.rerank);
        rerank_beam<SR>(p, s, qid, mm);
        n_rerank = mm;
      }
      if (mm < k) {
        if (l == 0) {
          const int slot = atomicAdd(p.fb_count, 1);
          p.fb_list[slot] = qid;
        }
      } else {
        const int64_t o = (int64_t)qid * p.kstride;
        for (int t = l; t < p.kstride; t += kWave) {
          const uint64_t kt = t < k ? s.beam.a[t] : kNoKey;
          p.knn_idx[o + t] = t < k ? key_id(kt) : -1;
          p.knn_dist[o + t] = t < k ? measure_to_dist(key_measure(kt), p.rows.metric)
                                    : __int_as_float(0x7f800000);
        }
        if (l == 0) {
          const uint64_t kk = s.beam.a[k - 1];
          const float dk = measure_to_dist(key_measure(kk), p.rows.metric);
          p.rho[qid] = 1.0f / dk;
          p.rank_key[qid] = (kk & 0xffffffff00000000ull) | (uint32_t)qid;
        }
      }
    } else {  // MODE_DEP
      int c = min(m, p.kdep);
      if (kNeedRerank && c > 0) {
        rerank_beam<SR>(p, s, qid, c);
        n_rerank = c;
      }
      const uint64_t ki = p.key_in[qid];
      uint64_t best = kNoKey;
      for (int t = l; t < c; t += kWave) {
        const uint64_t kt = s.beam.a[t];
        if (p.key_in[key_id(kt)] < ki && kt < best) best = kt;
      }
      best = wave_min_u64(best);
      if (l == 0) {
        if (best != kNoKey) {
          p.dep[qid] = key_id(best);
          p.delta[qid] = measure_to_dist(key_measure(best), p.rows.metric);
        } else {
          const int slot = atomicAdd(p.u_out_count, 1);
          p.u_out[slot] = qid;
          atomicAdd(p.ucnt_out + ti, 1);
        }
      }
    }
    if (p.counters && l == 0) {
      atomicAdd(p.counters + 0, s.n_exp);
      atomicAdd(p.counters + 1, s.n_ids);
      atomicAdd(p.counters + 2, s.n_rows);
      atomicAdd(p.counters + 3, n_rerank);
    }
    s.n_exp = s.n_ids = s.n_rows = 0;
    wave_lds_sync();
  }
}

// Three waves per SIMD for the narrow row formats (at most 168 VGPRs, no
// spills): with the compact visited hash their LDS holds about eleven waves per
// CU, and the compiler's own choice (170 VGPRs) would allow only two per SIMD
// (1.28M x 1024 FP8 build search 1,621 -> 1,480 ms per step).  Build searches
// scored on the matrix cores over short rows (at most 16 lanes per row) have
// LDS for about twenty waves per CU and ask for five per SIMD (96 VGPRs, a few
// bytes spilled; 1M x 128 BF16 build search 356 -> 344 ms per step).  Float32
// rows keep the compiler's choice (about 250 VGPRs for 784-d rows).
template <int DT, int S, int MODE, bool MF>
constexpr int search_waves_per_simd() {
  if (DT == PECANN_F32) return 1;
  if (MF && MODE == MODE_BUILD && S <= 16) return 5;
  return 3;
}
template <int DT, int S, int MODE, bool MF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(search_waves_per_simd<DT, S, MODE, MF>()))) void search_kernel(SearchParams p) {
  search_body<DT, S, MODE, MF>(p);
}
// The kNN search with a register budget for three waves per SIMD (168 VGPRs):
// there the extra wave hides more gather latency than the few spilled
// registers cost (measured); the build and doubling searches gained nothing.
template <int DT, int S, bool MF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void search_knn_kernel(SearchParams p) {
  search_body<DT, S, MODE_KNN, MF>(p);
}

template <int DT, int S, bool MF>
constexpr int scorer_lds_bytes() {
  if constexpr (MF && (DT == PECANN_BF16 || DT == PECANN_FP8E4M3 || DT == PECANN_MXFP6))
    return MfmaScorer<DT, S>::LDS_BYTES;
  else return 0;
}

template <int DT, int S, bool MF>
static hipError_t launch_search_t(const SearchParams &p, int grid, hipStream_t st) {
  if constexpr (S > max_shape(DT)) {
    return hipErrorInvalidValue;
  } else {
    const size_t lds = search_lds_bytes(p.L, p.hbits, p.hid_bits) + scorer_lds_bytes<DT, S, MF>();
    switch (p.mode) {
      case MODE_KNN:
        hipLaunchKernelGGL((search_knn_kernel<DT, S, MF>), dim3(grid), dim3(64), lds, st, p);
        break;
      case MODE_DEP:
        hipLaunchKernelGGL((search_kernel<DT, S, MODE_DEP, MF>), dim3(grid), dim3(64), lds, st, p);
        break;
      case MODE_BUILD:
        hipLaunchKernelGGL((search_kernel<DT, S, MODE_BUILD, MF>), dim3(grid), dim3(64), lds, st, p);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
}

}  // namespace pecann
