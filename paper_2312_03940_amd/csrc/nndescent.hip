// NN-descent graph construction: the PyNNDescent index offered beside Vamana
// (Sec. 4.1; the graph comparison of Sec. 6 prunes both with alpha).  The paper
// does not print the construction; this is Dong, Charikar and Li's NN-descent
// in synchronous rounds.  Every point keeps K neighbour keys (distance
// measure, index) in ascending order, each flagged new or old.  A round reads
// the lists as they were when it began:
//   reverse lists   for each point, the K closest sources whose list holds it
//                   flagged new, and the K closest flagged old;
//   local join      for each point i, U = its new entries and new reverse
//                   sources, W = its old entries and old reverse sources not
//                   in U; every pair of U x U and U x W is scored on the matrix
//                   cores and each member is proposed to the other when it
//                   beats that point's current K-th key;
//   update          the next list of a point is the K smallest keys of its list
//                   and its proposals; entries that were not in the list are
//                   flagged new.
// The next list is a function of sets (the K smallest of a union), so neither
// the order of the joins nor the chunking of the proposal buffer changes it.
// A device flag ends the rounds once a round leaves at most the stop level of
// new entries; later rounds then only copy the lists, so the host never waits.
#include "beam.hpp"
#include "claim.hpp"
#include "kernels.hpp"
#include "tiles.hpp"

namespace pecann {

namespace {

constexpr int kBlock = 256;       // threads per block of the element-wise kernels
constexpr int kJoinHashBits = 10; // members of one join: at most 4K <= 256 ids

__device__ __forceinline__ int wave_incl_sum(int v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(v, off);
    if (l >= off) v += y;
  }
  return v;
}

// A SortedList of capacity K over LDS at p (2K keys, 64 keys of scratch, 2K
// flag bytes); returns the bytes it takes.
__device__ __forceinline__ size_t carve_list(SortedList &sl, uint8_t *p, int K) {
  const int Kp = (K + 15) & ~15;
  sl.a = (uint64_t *)p;
  sl.b = sl.a + K;
  sl.tmp = sl.b + K;
  sl.fa = (uint8_t *)(sl.tmp + 64);
  sl.fb = sl.fa + Kp;
  sl.cap = K;
  sl.reset();
  return 8 * (2 * (size_t)K + 64) + 2 * (size_t)Kp;
}

// Merge keys given one per lane, possibly repeated within the call, into the
// list (bitonic path, which drops repeats).
__device__ __forceinline__ void merge_any(SortedList &sl, uint64_t key) {
  if (sl.m == sl.cap && key >= sl.tail) key = kNoKey;
  if (ballot(key != kNoKey)) sl.merge_sorted(key);
}

__device__ __forceinline__ void load_list(SortedList &sl, const uint64_t *keys, const uint8_t *flags,
                                          int K) {
  const int l = lane_id();
  int m = 0;
  for (int j0 = 0; j0 < K; j0 += kWave) {
    const int j = j0 + l;
    uint64_t k = kNoKey;
    if (j < K) k = keys[j];
    // the sorted list's flag marks an entry as old (flag 1 of the list = new)
    if (j < K) { sl.a[j] = k; sl.fa[j] = flags ? (flags[j] ? 0 : 1) : 1; }
    m += __popcll(ballot(j < K && k != kNoKey));
  }
  wave_lds_sync();
  sl.m = m;
  sl.hint = 0;
  sl.tail = m > 0 ? sl.a[m - 1] : kNoKey;
}

__device__ __forceinline__ void store_list(const SortedList &sl, uint64_t *keys, uint8_t *flags, int K) {
  for (int j = lane_id(); j < K; j += kWave) {
    const bool in = j < sl.m;
    keys[j] = in ? sl.a[j] : kNoKey;
    if (flags) flags[j] = in && sl.fa[j] == 0 ? 1 : 0;
  }
}

}  // namespace

// First lists: the measures to the K given ids, sorted; every entry new.  Ids
// outside [0, n) or equal to the point itself give empty entries.
template <int DT>
__global__ __launch_bounds__(64) void nnd_init_kernel(NndParams p, const int32_t *init) {
  __shared__ uint64_t k0[64], k1[64];
  const int l = lane_id(), col = l & 15, g = l >> 4;
  const int K = p.K;
  for (int64_t u = blockIdx.x; u < p.n; u += gridDim.x) {
    int32_t id = l < K ? init[u * K + l] : -1;
    if (id < 0 || id >= p.n || id == u) id = -1;
    int32_t rj[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) rj[t] = __shfl(id, 16 * t + col);
    v4f tt[4];
    dot_tiles<DT, 4>(p.rows, col == 0 ? (int32_t)u : -1, rj, tt);  // A row 0 holds u
    if (g == 0) {
      const uint32_t nu = p.rows.sqn[u];
      const float su = (DT == PECANN_FP8E4M3) ? fp8_row_scale(p.rows, u) : 1.0f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint64_t key = kNoKey;
        if (rj[t] >= 0) {
          const float sc = (DT == PECANN_FP8E4M3) ? fp8_row_scale(p.rows, rj[t]) : 1.0f;
          key = make_key(pair_measure<DT>(tt[t][0], nu, p.rows.sqn[rj[t]], su, sc, p.rows.metric),
                         rj[t]);
        }
        k0[16 * t + col] = key;
      }
    }
    wave_lds_sync();
    // stable rank sort of the K keys (repeated ids keep both copies)
    if (l < K) {
      const uint64_t key = k0[l];
      int r = 0;
      for (int t = 0; t < K; ++t) {
        const uint64_t o = k0[t];
        r += (o < key) | ((o == key) & (t < l));
      }
      k1[r] = key;
    }
    wave_lds_sync();
    if (l < K) {
      p.cur_keys[u * K + l] = k1[l];
      p.cur_flags[u * K + l] = k1[l] != kNoKey ? 1 : 0;
    }
    wave_lds_sync();
  }
}

// Round start: next = cur with every entry old.  Runs even after the stop
// flag is set, so that the last lists always end in the same buffer.
__global__ void nnd_round_begin_kernel(NndParams p) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nk = (int64_t)p.n * p.K;
  for (int64_t e = e0; e < nk; e += (int64_t)gridDim.x * blockDim.x) {
    p.nxt_keys[e] = p.cur_keys[e];
    p.nxt_flags[e] = 0;
  }
}

// Reverse entries grouped by target: count, place, scatter (key = the source's
// measure to the target and the source's index; flag = the entry's flag).
__global__ void nnd_rev_count_kernel(NndParams p, int32_t ignore_done) {
  if (!ignore_done && *p.done) return;
  const int64_t nk = (int64_t)p.n * p.K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t id = key_id(p.cur_keys[e]);
    p.rticket[e] = id >= 0 ? atomicAdd(p.rcnt + id, 1) : -1;
  }
}

// Segment offsets per block (block_claim), the loop's trip count uniform in the block.
__global__ void nnd_rev_alloc_kernel(NndParams p, int32_t ignore_done) {
  if (!ignore_done && *p.done) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < p.n; t0 += stride) {
    const int64_t t = t0 + threadIdx.x;
    const int c = t < p.n ? p.rcnt[t] : 0;
    const int incl = wave_prefix_sum(c);
    const int cnt[1] = {__shfl(incl, kWave - 1)};
    int32_t *const ctr[1] = {p.rcursor};
    int base[1];
    block_claim<1>(cnt, ctr, base);
    if (t < p.n) p.roff[t] = base[0] + incl - c;
  }
}

__global__ void nnd_rev_scatter_kernel(NndParams p, int32_t ignore_done) {
  if (!ignore_done && *p.done) return;
  const int64_t nk = (int64_t)p.n * p.K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t tk = p.rticket[e];
    if (tk < 0) continue;
    const uint64_t key = p.cur_keys[e];
    const int64_t pos = (int64_t)p.roff[key_id(key)] + tk;
    p.rseg[pos] = (key & 0xffffffff00000000ull) | (uint32_t)(e / p.K);
    p.rsegf[pos] = p.cur_flags ? p.cur_flags[e] : 1;
  }
}

// Per target: the K closest new sources (rnew) and the K closest old ones
// (rold); with split = 0 every source goes to rnew.  Resets the target's count.
__global__ __launch_bounds__(64) void nnd_rev_select_kernel(NndParams p, int32_t split,
                                                            int32_t ignore_done) {
  if (!ignore_done && *p.done) return;
  extern __shared__ __align__(16) uint8_t smem[];
  SortedList ln, lo;
  const size_t b = carve_list(ln, smem, p.K);
  carve_list(lo, smem + b, p.K);
  const int l = lane_id();
  for (int64_t t = blockIdx.x; t < p.n; t += gridDim.x) {
    ln.reset();
    lo.reset();
    const int cnt = p.rcnt[t];
    const int64_t off = p.roff[t];
    for (int c0 = 0; c0 < cnt; c0 += kWave) {
      uint64_t key = kNoKey;
      bool fnew = true;
      if (c0 + l < cnt) {
        key = p.rseg[off + c0 + l];
        fnew = !split || p.rsegf[off + c0 + l];
      }
      ln.merge(fnew ? key : kNoKey);  // the sources of one target are distinct
      if (split) lo.merge(fnew ? kNoKey : key);
    }
    for (int j = l; j < p.K; j += kWave) {
      p.rnew[t * p.K + j] = j < ln.m ? key_id(ln.a[j]) : -1;
      if (split) p.rold[t * p.K + j] = j < lo.m ? key_id(lo.a[j]) : -1;
    }
    if (l == 0) p.rcnt[t] = 0;
    wave_lds_sync();
  }
}

// Local joins: proposals (target, key) into the pass's buffer, in which wave
// (block) w owns the segment [w * seg, (w + 1) * seg).  A wave takes the next
// point of the round's queue while its segment still has room for the
// worst-case proposal count of one join, so with no shared counter a pass
// covers at least floor(seg / worst) points per wave unless the queue runs
// out; the wave records its segment's fill when it stops.  Members: U (new
// entries, then new reverse sources) and W (old entries, then old reverse
// sources), deduplicated through an LDS hash (one it forgets costs a repeated
// pair, never a wrong one: self pairs are skipped and the merge drops repeated
// keys).  Tiles: row block b of U against U blocks b.. (upper triangle on the
// diagonal) and every W block, four at a time.  A proposal to t is kept only
// if it beats the K-th key of t's next list as it stands after the previous
// passes: that list only improves, so nothing dropped could enter it.
template <int DT>
__global__ __launch_bounds__(64) void nnd_join_kernel(NndParams p) {
  if (*p.done) return;
  extern __shared__ __align__(16) uint8_t smem[];
  const int K = p.K, M = 4 * K;
  int32_t *mem = (int32_t *)smem;         // [M] member ids
  uint64_t *wk = (uint64_t *)(mem + M);   // [M] member's current K-th key
  uint32_t *cn = (uint32_t *)(wk + M);    // [M] squared norms
  float *cs = (float *)(cn + M);          // [M] row scales
  IdHash h;
  h.slot = (int32_t *)(cs + M);
  h.bits = kJoinHashBits;
  const int l = lane_id(), col = l & 15, g = l >> 4;
  unsigned long long n_tiles = 0, n_prop = 0;
  const int64_t sbase = (int64_t)blockIdx.x * p.seg;
  int64_t fill = 0;
  for (;;) {
    if (fill + p.maxprop > p.seg) break;
    const int it = next_item(p.head);
    const int64_t i = it;
    if (i >= p.n) break;
    h.clear();
    wave_lds_sync();
    int cnt = 0, nu = 0;
    for (int src = 0; src < 4; ++src) {
      for (int j0 = 0; j0 < K; j0 += kWave) {
        const int j = j0 + l;
        int32_t id = -1;
        if (j < K) {
          if (src == 0 || src == 2) {
            const uint64_t key = p.cur_keys[i * K + j];
            const bool fnew = p.cur_flags[i * K + j] != 0;
            if (key != kNoKey && fnew == (src == 0)) id = key_id(key);
          } else {
            id = (src == 1 ? p.rnew : p.rold)[i * K + j];
          }
        }
        if (id >= p.n || id == i) id = -1;
        if (id >= 0 && !h.insert(id)) id = -1;
        const uint64_t bm = ballot(id >= 0);
        if (id >= 0) mem[cnt + lanes_below(bm)] = id;
        cnt += __popcll(bm);
      }
      if (src == 1) nu = cnt;
    }
    const int nw = cnt - nu;
    wave_lds_sync();
    for (int j = l; j < cnt; j += kWave) {
      const int32_t id = mem[j];
      wk[j] = p.nxt_keys[(int64_t)id * K + K - 1];
      cn[j] = p.rows.sqn[id];
      cs[j] = (DT == PECANN_FP8E4M3) ? fp8_row_scale(p.rows, id) : 1.0f;
    }
    wave_lds_sync();
    const int nub = (nu + 15) >> 4, nwb = (nw + 15) >> 4;
    for (int b1 = 0; b1 < nub; ++b1) {
      const int ncb = (nub - b1) + nwb;  // column blocks: U b1.., then W
      const int ai0 = 16 * b1;
      const int32_t ar = ai0 + col < nu ? mem[ai0 + col] : -1;
      for (int cb0 = 0; cb0 < ncb; cb0 += 4) {
        int32_t br[4];
        int cbase[4], clim[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int cb = cb0 + t;
          cbase[t] = -1;
          clim[t] = 0;
          br[t] = -1;
          if (cb < ncb) {
            const bool inU = cb < nub - b1;
            cbase[t] = inU ? 16 * (b1 + cb) : nu + 16 * (cb - (nub - b1));
            clim[t] = inU ? nu : cnt;
            const int j = cbase[t] + col;
            br[t] = j < clim[t] ? mem[j] : -1;
          }
        }
        v4f tt[4];
        dot_tiles<DT, 4>(p.rows, ar, br, tt);
        n_tiles += min(4, ncb - cb0);
        // proposals of this lane: bit 2 (4 t + r) + dir (0: c to a, 1: a to c)
        uint32_t pm = 0;
        float mv[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            mv[t][r] = 0.f;
            const int ai = ai0 + 4 * g + r, ci = cbase[t] + col;
            const bool diag = cb0 + t == 0;  // U block b1 against itself
            if (cbase[t] < 0 || ai >= nu || ci >= clim[t] || (diag && 4 * g + r >= col)) continue;
            const int32_t a = mem[ai], c = mem[ci];
            if (a == c) continue;
            const float m = pair_measure<DT>(tt[t][r], cn[ai], cn[ci], cs[ai], cs[ci], p.rows.metric);
            mv[t][r] = m;
            if (make_key(m, c) < wk[ai]) pm |= 1u << (2 * (4 * t + r));
            if (make_key(m, a) < wk[ci]) pm |= 1u << (2 * (4 * t + r) + 1);
          }
        }
        const int mine = __popc(pm);
        const int incl = wave_incl_sum(mine);
        const int total = __shfl(incl, kWave - 1);
        if (total == 0) continue;
        if (fill + total > p.seg) {  // cannot happen: a join never exceeds maxprop
          if (l == 0) atomicAdd(p.overflow, 1);
          continue;
        }
        int64_t o = sbase + fill + incl - mine;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint32_t two = (pm >> (2 * (4 * t + r))) & 3u;
            if (!two) continue;
            const int ai = ai0 + 4 * g + r, ci = cbase[t] + col;
            const int32_t a = mem[ai], c = mem[ci];
            if (two & 1u) { p.ptgt[o] = a; p.pkey[o] = make_key(mv[t][r], c); ++o; }
            if (two & 2u) { p.ptgt[o] = c; p.pkey[o] = make_key(mv[t][r], a); ++o; }
          }
        }
        n_prop += total;
        fill += total;
      }
    }
    wave_lds_sync();
  }
  if (l == 0) p.pfill[blockIdx.x] = (int32_t)fill;
  if (p.counters && l == 0) {
    atomicAdd(p.counters + 0, n_prop);
    atomicAdd(p.counters + 1, n_tiles);
  }
}

// Proposals grouped by target: count (and list each target once), place,
// scatter.  Block b walks the filled part of join segment b.
__global__ void nnd_prop_count_kernel(NndParams p) {
  if (*p.done) return;
  const int64_t base = (int64_t)blockIdx.x * p.seg;
  const int nf = p.pfill[blockIdx.x];
  for (int j0 = 0; j0 < nf; j0 += blockDim.x) {
    const int j = j0 + threadIdx.x;
    int32_t t = -1;
    int tk = -1;
    if (j < nf) {
      const int64_t e = base + j;
      t = p.ptgt[e];
      tk = atomicAdd(p.pcnt + t, 1);
      p.pticket[e] = tk;
    }
    // first proposals to a target list it once; slots handed out per block
    const uint64_t fm = ballot(tk == 0);
    const int cnt[1] = {(int)__popcll(fm)};
    int32_t *const ctr[1] = {p.ptouch_n};
    int b[1];
    block_claim<1>(cnt, ctr, b);
    if (tk == 0) p.ptouch[b[0] + lanes_below(fm)] = t;
  }
}

__global__ void nnd_prop_alloc_kernel(NndParams p) {
  if (*p.done) return;
  const int nt = *p.ptouch_n;
  for (int j0 = blockIdx.x * blockDim.x; j0 < nt; j0 += gridDim.x * blockDim.x) {
    const int j = j0 + threadIdx.x;
    int32_t t = -1;
    int c = 0;
    if (j < nt) {
      t = p.ptouch[j];
      c = p.pcnt[t];
    }
    const int incl = wave_prefix_sum(c);
    const int cnt[1] = {__shfl(incl, kWave - 1)};
    int32_t *const ctr[1] = {p.pcursor};
    int b[1];
    block_claim<1>(cnt, ctr, b);
    if (j < nt) p.poff[t] = b[0] + incl - c;
  }
}

__global__ void nnd_prop_scatter_kernel(NndParams p) {
  if (*p.done) return;
  const int64_t base = (int64_t)blockIdx.x * p.seg;
  const int nf = p.pfill[blockIdx.x];
  for (int j = threadIdx.x; j < nf; j += blockDim.x) {
    const int64_t e = base + j;
    p.pseg[(int64_t)p.poff[p.ptgt[e]] + p.pticket[e]] = p.pkey[e];
  }
}

// Per proposed-to point: next list = the K smallest of it and its proposals.
__global__ __launch_bounds__(64) void nnd_merge_kernel(NndParams p) {
  if (*p.done) return;
  extern __shared__ __align__(16) uint8_t smem[];
  SortedList sl;
  carve_list(sl, smem, p.K);
  const int l = lane_id();
  const int nt = *p.ptouch_n;
  unsigned long long merged = 0;
  for (;;) {
    const int it = next_item(p.head);
    if (it >= nt) break;
    ++merged;
    const int32_t t = p.ptouch[it];
    const int64_t o = (int64_t)t * p.K;
    load_list(sl, p.nxt_keys + o, p.nxt_flags + o, p.K);
    const int cnt = p.pcnt[t];
    const int64_t off = p.poff[t];
    for (int c0 = 0; c0 < cnt; c0 += kWave)
      merge_any(sl, c0 + l < cnt ? p.pseg[off + c0 + l] : kNoKey);
    store_list(sl, p.nxt_keys + o, p.nxt_flags + o, p.K);
    if (l == 0) p.pcnt[t] = 0;
    wave_lds_sync();
  }
  if (p.counters && l == 0 && merged) atomicAdd(p.counters + 2, merged);
}

// New entries of the next lists (one 64-bit atomic per wave).
__global__ void nnd_count_new_kernel(NndParams p) {
  if (*p.done) return;
  const int64_t nk = (int64_t)p.n * p.K;
  unsigned long long c = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nk;
       e += (int64_t)gridDim.x * blockDim.x)
    c += p.nxt_flags[e] != 0;
  for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_down(c, off);
  if (lane_id() == 0 && c) atomicAdd(p.updates, c);
}

__global__ void nnd_round_end_kernel(NndParams p) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!*p.done) {
    *p.rounds += 1;
    if ((long long)*p.updates <= p.thr) *p.done = 1;
  }
  *p.updates = 0;
}

// acc = the K smallest of acc and src (lists of two repeats).
__global__ __launch_bounds__(64) void nnd_acc_merge_kernel(NndParams p, uint64_t *acc,
                                                           const uint64_t *src) {
  extern __shared__ __align__(16) uint8_t smem[];
  SortedList sl;
  carve_list(sl, smem, p.K);
  const int l = lane_id();
  for (int64_t t = blockIdx.x; t < p.n; t += gridDim.x) {
    const int64_t o = t * p.K;
    load_list(sl, acc + o, nullptr, p.K);
    for (int c0 = 0; c0 < p.K; c0 += kWave)
      merge_any(sl, c0 + l < p.K ? src[o + c0 + l] : kNoKey);
    store_list(sl, acc + o, nullptr, p.K);
    wave_lds_sync();
  }
}

__global__ void nnd_out_kernel(NndParams p, const uint64_t *keys, int32_t *idx, float *dist) {
  const int64_t nk = (int64_t)p.n * p.K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[e];
    const bool in = k != kNoKey;
    if (idx) idx[e] = in ? key_id(k) : -1;
    if (dist) dist[e] = in ? measure_to_dist(key_measure(k), p.rows.metric) : __int_as_float(0x7f800000);
  }
}

__global__ void nnd_copy_u64_kernel(const uint64_t *src, uint64_t *dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int elem_grid(int64_t items, int cus) {
  const int64_t g = (items + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, (int64_t)cus * 16));
}

size_t nnd_list_lds_bytes(int K) {
  const size_t Kp = (size_t)((K + 15) & ~15);
  return 8 * (2 * (size_t)K + 64) + 2 * Kp;
}
size_t nnd_join_lds_bytes(int K) {
  return (size_t)4 * K * (4 + 8 + 4 + 4) + 4 * ((size_t)1 << kJoinHashBits);
}

template <int DT>
static hipError_t launch_nnd_init_t(const NndParams &p, const int32_t *init, int grid, hipStream_t s) {
  hipLaunchKernelGGL((nnd_init_kernel<DT>), dim3(grid), dim3(64), 0, s, p, init);
  return hipGetLastError();
}
template <int DT>
static hipError_t launch_nnd_join_t(const NndParams &p, int grid, hipStream_t s) {
  hipLaunchKernelGGL((nnd_join_kernel<DT>), dim3(grid), dim3(64), nnd_join_lds_bytes(p.K), s, p);
  return hipGetLastError();
}

#define NND_DT_SWITCH(fn, ...)                                        \
  switch (dt) {                                                       \
    case PECANN_F32: return fn<PECANN_F32>(__VA_ARGS__);              \
    case PECANN_U8: return fn<PECANN_U8>(__VA_ARGS__);                \
    case PECANN_BF16: return fn<PECANN_BF16>(__VA_ARGS__);            \
    case PECANN_FP8E4M3: return fn<PECANN_FP8E4M3>(__VA_ARGS__);      \
    default: return hipErrorInvalidValue;                             \
  }

hipError_t launch_nnd_init(int32_t dt, const NndParams &p, const int32_t *init, int grid, hipStream_t s) {
  NND_DT_SWITCH(launch_nnd_init_t, p, init, grid, s)
}

hipError_t launch_nnd_join(int32_t dt, const NndParams &p, int grid, hipStream_t s) {
  NND_DT_SWITCH(launch_nnd_join_t, p, grid, s)
}

hipError_t launch_nnd_round_begin(const NndParams &p, int cus, hipStream_t s) {
  hipLaunchKernelGGL(nnd_round_begin_kernel, dim3(elem_grid((int64_t)p.n * p.K, cus)), dim3(kBlock), 0,
                     s, p);
  return hipGetLastError();
}

hipError_t launch_nnd_reverse(const NndParams &p, int32_t split, int32_t ignore_done, int cus,
                              hipStream_t s) {
  const int64_t nk = (int64_t)p.n * p.K;
  hipError_t e = launch_fill_i32(p.rcursor, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nnd_rev_count_kernel, dim3(elem_grid(nk, cus)), dim3(kBlock), 0, s, p, ignore_done);
  hipLaunchKernelGGL(nnd_rev_alloc_kernel, dim3(elem_grid(p.n, cus)), dim3(kBlock), 0, s, p, ignore_done);
  hipLaunchKernelGGL(nnd_rev_scatter_kernel, dim3(elem_grid(nk, cus)), dim3(kBlock), 0, s, p, ignore_done);
  const size_t lds = 2 * nnd_list_lds_bytes(p.K);
  const int grid = (int)std::min<int64_t>(p.n, (int64_t)cus * 32);
  hipLaunchKernelGGL(nnd_rev_select_kernel, dim3(grid), dim3(64), lds, s, p, split, ignore_done);
  return hipGetLastError();
}

hipError_t launch_nnd_proposals(const NndParams &p, int join_grid, int cus, hipStream_t s) {
  hipLaunchKernelGGL(nnd_prop_count_kernel, dim3(join_grid), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(nnd_prop_alloc_kernel, dim3(cus * 16), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(nnd_prop_scatter_kernel, dim3(join_grid), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_nnd_merge(const NndParams &p, int grid, hipStream_t s) {
  hipLaunchKernelGGL(nnd_merge_kernel, dim3(grid), dim3(64), nnd_list_lds_bytes(p.K), s, p);
  return hipGetLastError();
}

hipError_t launch_nnd_round_end(const NndParams &p, int cus, hipStream_t s) {
  hipLaunchKernelGGL(nnd_count_new_kernel, dim3(elem_grid((int64_t)p.n * p.K, cus)), dim3(kBlock), 0,
                     s, p);
  hipLaunchKernelGGL(nnd_round_end_kernel, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_nnd_acc_merge(const NndParams &p, uint64_t *acc, const uint64_t *src, int cus,
                                hipStream_t s) {
  const int grid = (int)std::min<int64_t>(p.n, (int64_t)cus * 32);
  hipLaunchKernelGGL(nnd_acc_merge_kernel, dim3(grid), dim3(64), nnd_list_lds_bytes(p.K), s, p, acc, src);
  return hipGetLastError();
}

hipError_t launch_nnd_out(const NndParams &p, const uint64_t *keys, int32_t *idx, float *dist, int cus,
                          hipStream_t s) {
  hipLaunchKernelGGL(nnd_out_kernel, dim3(elem_grid((int64_t)p.n * p.K, cus)), dim3(kBlock), 0, s, p,
                     keys, idx, dist);
  return hipGetLastError();
}

hipError_t launch_nnd_copy(const uint64_t *src, uint64_t *dst, int64_t n, int cus, hipStream_t s) {
  hipLaunchKernelGGL(nnd_copy_u64_kernel, dim3(elem_grid(n, cus)), dim3(kBlock), 0, s, src, dst, n);
  return hipGetLastError();
}

PECANN_CHECK_READER(nndescent)

}  // namespace pecann
