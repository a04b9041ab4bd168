// K8/K9 RobustPrune of DiskANN (the Vamana pruning rule the paper adopts,
// Sec. 3.2), one wavefront per pruned point:
//   sort the candidates by (D(p, c), c), drop p, duplicates and -1;
//   repeatedly move the closest surviving candidate c* to the output (stop at
//   R) and drop every surviving c with alpha * D(c*, c) <= D(p, c)
//   (alpha^2 * D^2 <= D^2 for L2 measures, which are squared distances).
// Distances between candidates come from dense 16 x 16 dot-product tiles on
// the matrix cores (f32, i8, bf16 or fp8 MFMA by row format), turned into
// distances with the rows' stored norms.  Distances to p are not formed again
// in the graph build: the search hands over D(p, v) of the visited set, every
// adjacency entry keeps the key (D(p, u), u) it was selected or appended with,
// and a reverse edge p -> q carries D(p, q) as D(q, p).  After each
// block of 16 the surviving candidates are compacted, so every later tile is
// dense in live candidates; column tiles go four at a time to keep several row
// loads in flight per lane.
// prune_forward: Nout(p) = RobustPrune(p, V_p u Nout(p)) for each point of a batch.
// prune_reverse: for each target q of the batch's reverse edges, append the
//   new sources not yet present (ascending index) if they fit in R, else
//   Nout(q) = RobustPrune(q, Nout(q) u sources).
#include "beam.hpp"
#include "tiles.hpp"

namespace pecann {

namespace {

struct PruneLds {
  int32_t *ids;    // candidates [ccap]
  uint64_t *k0;    // keys [ccap]
  uint64_t *k1;    // sorted keys [ccap]
  uint64_t *sel;   // keys of the selected [R]
  uint32_t *cn;    // squared norm of each sorted candidate [ccap] (L2 only)
  float *cs;       // row scale of each sorted candidate [ccap] (FP8 L2 only)
  uint8_t *alive;  // [ccap]
  // a candidate's norm and scale: cosine measures need no norm, and cosine FP8
  // rows share one scale, so those arrays are left out of the LDS
  __device__ __forceinline__ uint32_t norm(int j) const { return cn ? cn[j] : 0u; }
  __device__ __forceinline__ float scl(int j) const { return cs ? cs[j] : 1.0f / kFp8UnitInv; }
};

__host__ __device__ __forceinline__ bool prune_has_norms(int metric) { return metric == PECANN_L2; }
__host__ __device__ __forceinline__ bool prune_has_scales(int dt, int metric) {
  return dt == PECANN_FP8E4M3 && metric == PECANN_L2;
}

template <int DT>
__device__ __forceinline__ PruneLds carve_prune(uint8_t *smem, int ccap, int R, int metric) {
  PruneLds s;
  s.k0 = (uint64_t *)smem;
  s.k1 = s.k0 + ccap;
  s.sel = s.k1 + ccap;
  s.ids = (int32_t *)(s.sel + R);
  uint8_t *q = (uint8_t *)(s.ids + ccap);
  s.cn = prune_has_norms(metric) ? (uint32_t *)q : nullptr;
  if (s.cn) q += 4 * (size_t)ccap;
  s.cs = prune_has_scales(DT, metric) ? (float *)q : nullptr;
  if (s.cs) q += 4 * (size_t)ccap;
  s.alive = q;
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

// Compacts the live entries of the sorted list [from, mv) toward `from`, keeping
// their order; returns the new end.  Entries move only to lower positions and
// every chunk is read before any lane writes, so the pass works in place.
__device__ __forceinline__ int compact_live(PruneLds &s, int from, int mv) {
  const int l = lane_id();
  int out = from;
  for (int j0 = from; j0 < mv; j0 += kWave) {
    const int j = j0 + l;
    const bool live = j < mv && s.alive[j];
    uint64_t key = 0;
    uint32_t cn = 0;
    float cs = 0.f;
    if (live) {
      key = s.k1[j];
      if (s.cn) cn = s.cn[j];
      if (s.cs) cs = s.cs[j];
    }
    const uint64_t bm = ballot(live);
    wave_lds_sync();
    if (live) {
      const int o = out + lanes_below(bm);
      s.k1[o] = key;
      if (s.cn) s.cn[o] = cn;
      if (s.cs) s.cs[o] = cs;
      s.alive[o] = 1;
    }
    out += __popcll(bm);
    wave_lds_sync();
  }
  return out;
}

// Selections of the block of 16 candidates starting at o, in order, from the
// block's own tile (register r of lane l: entries o + 4 (l / 16) + r and
// o + l % 16).  Each lane works out which earlier entries of its column's
// candidate would drop it (alpha^2 D^2(i, j) <= D^2(p, j) for i < j), the masks
// are transposed with ballots, and the greedy pass runs on wave-uniform masks:
// no LDS round trip per step.  Appends the selected keys to s.sel and returns
// the mask of selected block entries; block entries end not alive.
template <int DT>
__device__ __forceinline__ uint32_t select_block(const PruneParams &p, PruneLds &s, const v4f &tile,
                                                 int o, int mv, float a2, int &nsel) {
  const int l = lane_id();
  const int col = l & 15, g = l >> 4;
  const int j = o + col;
  uint32_t kb = 0;
  if (j < mv) {
    const float dpj = key_measure(s.k1[j]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * g + r;
      if (i < col) {
        const float m = pair_measure<DT>(tile[r], s.norm(o + i), s.norm(j), s.scl(o + i), s.scl(j),
                                         p.rows.metric);
        if (a2 * m <= dpj) kb |= 1u << i;
      }
    }
  }
  kb |= __shfl_xor(kb, 16);
  kb |= __shfl_xor(kb, 32);
  uint32_t alive = (uint32_t)ballot(l < 16 && j < mv && s.alive[j]) & 0xffffu;
  uint32_t sel = 0;
  const int nsel0 = nsel;
#pragma unroll 1
  for (int i = 0; i < 16; ++i) {
    if (!((alive >> i) & 1u)) continue;
    sel |= 1u << i;
    alive &= ~(1u << i);
    if (++nsel == p.R) break;
    alive &= ~((uint32_t)ballot(l < 16 && ((kb >> i) & 1u)) & 0xffffu);
  }
  if (l < 16 && j < mv) {
    if ((sel >> l) & 1u) s.sel[nsel0 + __popc(sel & ((1u << l) - 1u))] = s.k1[j];
    s.alive[j] = 0;
  }
  wave_lds_sync();
  return sel;
}

// A lone 16 x 16 tile (a block's own tile, or the last tile of a row of
// tiles) has registers for twice the steps per memory round trip of a group
// of four: half the round trips for the same row bytes.  The products are
// accumulated in the same step order, so the results are the same (reverse
// prune per step: 70,000 x 784 float32 rows 39.0 -> 36.1 ms, 1.28M x 1024 FP8
// 282.0 -> 278.4 ms, 64 instances BF16 142.3 -> 138.1 ms).
template <int SG>
constexpr int lone_tile_steps() { return SG < 4 ? 4 : SG; }

// Short lists (at most kSmallBlocks blocks of 16 live candidates): block B's
// tiles against itself and every later block are formed in one round (rows
// already dropped are not loaded), then the block's selections and kills are
// settled from them -- one memory round trip per block instead of two or three.
constexpr int kSmallBlocks = 5;

template <int DT, int B, int SG>
__device__ __forceinline__ void short_block(const PruneParams &p, PruneLds &s, int mv, float a2,
                                            int &nsel) {
  if (16 * B >= mv || nsel >= p.R) return;
  constexpr int NT = kSmallBlocks - B;
  const int l = lane_id();
  const int col = l & 15, g = l >> 4;
  const int o = 16 * B;
  int32_t br[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = o + 16 * t + col;
    br[t] = (j < mv && s.alive[j]) ? key_id(s.k1[j]) : -1;
  }
  v4f tt[NT];
  dot_tiles<DT, NT, NT == 1 ? lone_tile_steps<SG>() : SG>(p.rows, br[0], br, tt);
  // (a) the block's own tile -> its selections, in order
  const uint32_t selmask = select_block<DT>(p, s, tt[0], o, mv, a2, nsel);
  if (nsel == p.R) return;
  // (b) the block's selected points drop later candidates
#pragma unroll
  for (int t = 1; t < NT; ++t) {
    const int j = o + 16 * t + col;
    bool kill = false;
    if (j < mv) {
      const float dpc = key_measure(s.k1[j]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * g + r;
        if ((selmask >> i) & 1u) {
          const float m = pair_measure<DT>(tt[t][r], s.norm(o + i), s.norm(j), s.scl(o + i), s.scl(j),
                                           p.rows.metric);
          kill |= a2 * m <= dpc;
        }
      }
    }
    const uint64_t km = ballot(kill);
    const uint32_t k16 = (uint32_t)((km | (km >> 16) | (km >> 32) | (km >> 48)) & 0xffffu);
    if (l < 16 && ((k16 >> l) & 1u)) s.alive[o + 16 * t + l] = 0;
  }
  wave_lds_sync();
}

// Nout(pt) from the selected keys: ids into adj, the keys beside them (when
// kept), the count into deg.
__device__ __forceinline__ void write_nout(const PruneParams &p, const PruneLds &s, int32_t pt,
                                           int nsel) {
  const int l = lane_id();
  PECANN_CHECK(nsel >= 0 && nsel <= p.R, CK_PRUNE);
  PECANN_CHECK(pt >= 0 && pt < p.n, CK_ITEM);
  int32_t *row = p.adj + (int64_t)pt * p.R;
  for (int e = l; e < p.R; e += kWave) row[e] = e < nsel ? (int32_t)key_id(s.sel[e]) : -1;
  if (p.akey)
    for (int e = l; e < nsel; e += kWave) p.akey[(int64_t)pt * p.R + e] = s.sel[e];
  if (l == 0) {
    p.deg[pt] = nsel;
    if (p.cons) p.cons[pt] = nsel;
  }
}

// The selected points of block b (selmask; A rows ra) drop later candidates of
// the NT tiles from column j0: each lane tests the 4 rows of its accumulator
// against its column.  Returns the tiles formed.
template <int DT, int NT, int SG>
__device__ __forceinline__ int kill_tiles(const PruneParams &p, PruneLds &s, int32_t ra, int b,
                                          uint32_t selmask, int j0, int mv, float a2) {
  const int l = lane_id();
  const int col = l & 15, g = l >> 4;
  int32_t rj[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = j0 + 16 * t + col;
    rj[t] = j < mv ? key_id(s.k1[j]) : -1;
  }
  v4f tt[NT];
  dot_tiles<DT, NT, SG>(p.rows, ra, rj, tt);
  int tiles = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = j0 + 16 * t + col;
    bool kill = false;
    if (j < mv) {
      const float dpc = key_measure(s.k1[j]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * g + r;
        if ((selmask >> i) & 1u) {
          const float m = pair_measure<DT>(tt[t][r], s.norm(b + i), s.norm(j), s.scl(b + i), s.scl(j),
                                           p.rows.metric);
          kill |= a2 * m <= dpc;
        }
      }
    }
    const uint64_t km = ballot(kill);
    const uint32_t k16 = (uint32_t)((km | (km >> 16) | (km >> 32) | (km >> 48)) & 0xffffu);
    if (l < 16 && ((k16 >> l) & 1u)) s.alive[j0 + 16 * t + l] = 0;
    tiles += j0 + 16 * t < mv;
  }
  wave_lds_sync();
  return tiles;
}

// RobustPrune of point pt over s.ids[0..nc); writes Nout(pt) into adj/deg.
// The first npre candidates come with their keys (D(pt, c), c) already in s.k0.
// Candidates are sorted by (D(pt, c), c), and empty entries and repeats are
// dropped.  D(pt, c) comes from tiles whose A row 0 holds pt (rows 1-15 are
// zeros), 64 candidates per round; lanes 0-15 read their column's value in
// accumulator register 0.  The greedy pass then walks the live
// list in blocks of 16: one matrix-core tile gives the block's own pairwise
// distances, which settle the block's selections in order; the block's selected
// points then drop later candidates tile by tile (each lane testing the 4 rows
// of its accumulator against its column), and the survivors are compacted.
// Returns the number of 16 x 16 tiles formed.
template <int DT, int SG>
__device__ __forceinline__ int robust_prune_tiles(const PruneParams &p, PruneLds &s, int32_t pt, int nc, int npre = 0) {
  constexpr int NT = 4;  // tiles in flight
  const int l = lane_id();
  const int col = l & 15, g = l >> 4;
  const float a2 = p.rows.metric == PECANN_L2 ? p.alpha * p.alpha : p.alpha;

  {
    const uint32_t npt = p.rows.sqn[pt];
    const float spt = (DT == PECANN_FP8E4M3) ? fp8_row_scale(p.rows, pt) : 1.0f;
    for (int base = npre; base < nc; base += 16 * NT) {
      int32_t rj[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int j = base + 16 * t + col;
        const int32_t id = j < nc ? s.ids[j] : -1;
        rj[t] = id == pt ? -1 : id;
      }
      v4f tt[NT];
      dot_tiles<DT, NT, SG>(p.rows, col == 0 ? pt : -1, rj, tt);  // A row 0 holds pt, rows 1-15 zeros
      if (g == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int j = base + 16 * t + col;
          if (j < nc) {
            uint64_t key = kNoKey;
            if (rj[t] >= 0) {
              const float sc = (DT == PECANN_FP8E4M3) ? fp8_row_scale(p.rows, rj[t]) : 1.0f;
              key = make_key(pair_measure<DT>(tt[t][0], npt, p.rows.sqn[rj[t]], spt, sc,
                                              p.rows.metric), rj[t]);
            }
            s.k0[j] = key;
          }
        }
      }
    }
  }
  wave_lds_sync();
  rank_sort_dups(s.k0, s.k1, nc);
  for (int j0 = 0; j0 < nc; j0 += kWave) {
    const int j = j0 + l;
    if (j < nc) {
      const uint64_t key = s.k1[j];
      const bool live = key != kNoKey && (j == 0 || s.k1[j - 1] != key);
      s.alive[j] = live;
      if (live) {
        const int32_t id = key_id(key);
        if (s.cn) s.cn[j] = p.rows.sqn[id];
        if (s.cs) s.cs[j] = fp8_row_scale(p.rows, id);
      }
    }
  }
  wave_lds_sync();
  int mv = compact_live(s, 0, nc);

  int nsel = 0, tiles = nc > npre ? (nc - npre + 15) / 16 : 0;
  if (mv <= 16 * kSmallBlocks) {
    const int nb = (mv + 15) / 16;
    short_block<DT, 0, SG>(p, s, mv, a2, nsel);
    short_block<DT, 1, SG>(p, s, mv, a2, nsel);
    short_block<DT, 2, SG>(p, s, mv, a2, nsel);
    short_block<DT, 3, SG>(p, s, mv, a2, nsel);
    short_block<DT, 4, SG>(p, s, mv, a2, nsel);
    tiles += nb * kSmallBlocks - nb * (nb - 1) / 2;
    write_nout(p, s, pt, nsel);
    return tiles;
  }
  for (int b = 0; b < mv && nsel < p.R; b += 16) {
    // (a) the block's own 16 x 16 tile (every entry of the block is live)
    const int32_t rb = b + col < mv ? key_id(s.k1[b + col]) : -1;
    uint32_t selmask;
    {
      const int32_t br[1] = {rb};
      v4f t[1];
      dot_tiles<DT, 1, lone_tile_steps<SG>()>(p.rows, rb, br, t);
      ++tiles;
      // (b) selections of this block, in order
      selmask = select_block<DT>(p, s, t[0], b, mv, a2, nsel);
    }
    if (nsel == p.R) break;
    // (c) the block's selected points drop later candidates, NT tiles at a time;
    // A rows of block entries that were not selected are not loaded (zeros:
    // their accumulator rows are never read)
    const int32_t ra = ((selmask >> col) & 1u) ? rb : -1;
    for (int j0 = b + 16; j0 < mv; j0 += 16 * NT) {
      if (mv - j0 <= 16) tiles += kill_tiles<DT, 1, lone_tile_steps<SG>()>(p, s, ra, b, selmask, j0, mv, a2);
      else tiles += kill_tiles<DT, NT, SG>(p, s, ra, b, selmask, j0, mv, a2);
    }
    // (d) survivors after this block move up behind it
    mv = compact_live(s, b + 16, mv);
  }
  write_nout(p, s, pt, nsel);
  return tiles;
}

// RobustPrune of pt over the keys s.k0[0..mv) (all known, distinct, none of
// them pt) whose first c entries are the output of pt's previous prune: no
// selected entry drops a later one, so none of them drops another here either
// (the same keys, the same measures, and alpha never decreases -- measures are
// at least 0, so a larger alpha drops less).  Only pairs with a member of
// U = the other mv - c candidates can drop anything, and the greedy pass is
// settled from the U x all tiles alone:
//   kU[j] = U members before j that would drop j,
//   cU[j] = U members after j that j would drop (j outside U),
// then a walk over U in key order decides each member from the selected
// entries before it.  The result is the full greedy pass's, with nu/16 rows of
// tiles instead of the pairwise triangle.  Returns the tiles formed, or -1 when
// the shape does not fit (more than kMaxU members of U or 3 * 64 candidates).
constexpr int kMaxU = 32;

// The tiles of U block ub (A rows aid; the block's members at sorted positions
// pr with measures dr) against the NT column tiles from c0: bits of U members
// before a column that would drop it go to kU, bits of U members after a
// column that it would drop go to cU.  Returns the tiles formed.
template <int DT, int NT, int SG>
__device__ __forceinline__ int u_tiles(const PruneParams &p, const PruneLds &s, int32_t aid, const int (&pr)[4],
                                       const float (&dr)[4], int ub, int c0, int mv, float a2, uint32_t *kU,
                                       uint32_t *cU) {
  const int l = lane_id();
  const int col = l & 15, g = l >> 4;
  int32_t bj[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int jc = c0 + 16 * t + col;
    bj[t] = jc < mv ? (int32_t)key_id(s.k1[jc]) : -1;
  }
  v4f tt[NT];
  dot_tiles<DT, NT, SG>(p.rows, aid, bj, tt);
  int tiles = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int jc = c0 + 16 * t + col;
    uint32_t kk = 0, cc = 0;
    if (jc < mv) {
      const float dc = key_measure(s.k1[jc]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pu = pr[r];
        if (pu >= 0 && pu != jc) {
          const float m = pair_measure<DT>(tt[t][r], s.norm(pu), s.norm(jc), s.scl(pu), s.scl(jc),
                                           p.rows.metric);
          const uint32_t bit = 1u << (ub * 16 + 4 * g + r);
          if (pu < jc) {
            if (a2 * m <= dc) kk |= bit;
          } else if (a2 * m <= dr[r]) {
            cc |= bit;
          }
        }
      }
    }
    kk |= __shfl_xor(kk, 16);
    kk |= __shfl_xor(kk, 32);
    cc |= __shfl_xor(cc, 16);
    cc |= __shfl_xor(cc, 32);
    if (l < 16 && jc < mv) {
      kU[jc] |= kk;
      cU[jc] |= cc;
    }
    tiles += c0 + 16 * t < mv;
  }
  return tiles;
}

template <int DT, int SG>
__device__ __forceinline__ int prune_with_prefix(const PruneParams &p, PruneLds &s, int32_t pt, int mv, int c) {
  constexpr int NT = 4;
  const int nu = mv - c;
  if (nu < 1 || nu > kMaxU || mv > 3 * kWave) return -1;
  const int l = lane_id();
  const int col = l & 15, g = l >> 4;
  const float a2 = p.rows.metric == PECANN_L2 ? p.alpha * p.alpha : p.alpha;
  // (1) sort by key (keys are distinct), marking the members of U
  for (int j = l; j < mv; j += kWave) {
    const uint64_t key = s.k0[j];
    int r = 0;
    for (int t = 0; t < mv; ++t) r += s.k0[t] < key;
    s.k1[r] = key;
    s.alive[r] = j >= c;
    const int32_t id = key_id(key);
    if (s.cn) s.cn[r] = p.rows.sqn[id];
    if (s.cs) s.cs[r] = fp8_row_scale(p.rows, id);
  }
  wave_lds_sync();
  // (2) positions of U in key order (s.ids), each member's index + 1 in alive
  uint32_t *kU = (uint32_t *)s.k0;
  uint32_t *cU = kU + mv;
  int32_t *upos = s.ids;
  for (int base = 0, cnt = 0; base < mv; base += kWave) {
    const int jp = base + l;
    const bool u = jp < mv && s.alive[jp];
    const uint64_t bm = ballot(u);
    if (u) {
      const int ui = cnt + lanes_below(bm);
      upos[ui] = jp;
      s.alive[jp] = (uint8_t)(1 + ui);
    }
    if (jp < mv) {
      kU[jp] = 0;
      cU[jp] = 0;
    }
    cnt += __popcll(bm);
  }
  wave_lds_sync();
  // (3) U x all tiles: A rows are U members, lanes 0-15 of each 16-group hold
  // column j, register r of lane l row 4 (l / 16) + r
  int tiles = 0;
  for (int ub = 0; ub * 16 < nu; ++ub) {
    const int ua = ub * 16 + col;
    const int32_t aid = ua < nu ? (int32_t)key_id(s.k1[upos[ua]]) : -1;
    int pr[4];
    float dr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ui = ub * 16 + 4 * g + r;
      pr[r] = ui < nu ? upos[ui] : -1;
      dr[r] = pr[r] >= 0 ? key_measure(s.k1[pr[r]]) : 0.f;
    }
    for (int c0 = 0; c0 < mv; c0 += 16 * NT) {
      if (mv - c0 <= 16) tiles += u_tiles<DT, 1, lone_tile_steps<SG>()>(p, s, aid, pr, dr, ub, c0, mv, a2, kU, cU);
      else tiles += u_tiles<DT, NT, SG>(p, s, aid, pr, dr, ub, c0, mv, a2, kU, cU);
    }
  }
  wave_lds_sync();
  // (4) the walk: member t of U is dropped by a selected U member before it
  // (kU of its position) or by a selected entry j outside U before it (j is
  // selected when no selected U member before j drops it)
  uint32_t rk[3], rc[3];
  bool rin[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int jp = l + kWave * i;
    rin[i] = jp < mv && s.alive[jp] == 0;
    rk[i] = rin[i] ? kU[jp] : 0u;
    rc[i] = rin[i] ? cU[jp] : 0u;
  }
  uint32_t selU = 0;
#pragma unroll 1
  for (int t = 0; t < nu; ++t) {
    const int pu = upos[t];
    bool dead = (kU[pu] & selU) != 0;
    if (!dead) {
      bool hit = false;
#pragma unroll
      for (int i = 0; i < 3; ++i)
        hit |= rin[i] && l + kWave * i < pu && !(rk[i] & selU) && ((rc[i] >> t) & 1u);
      dead = ballot(hit) != 0;
    }
    if (!dead) selU |= 1u << t;
  }
  // (5) the selected entries in key order, at most R of them
  int nsel = 0;
  for (int base = 0; base < mv && nsel < p.R; base += kWave) {
    const int jp = base + l;
    bool sel = false;
    if (jp < mv) {
      const int a = s.alive[jp];
      sel = a ? ((selU >> (a - 1)) & 1u) != 0 : (kU[jp] & selU) == 0;
    }
    const uint64_t bm = ballot(sel);
    if (sel) {
      const int o = nsel + lanes_below(bm);
      if (o < p.R) s.sel[o] = s.k1[jp];
    }
    nsel = min(p.R, nsel + __popcll(bm));
  }
  wave_lds_sync();
  write_nout(p, s, pt, nsel);
  return tiles;
}

}  // namespace

// Register targets (arch and accumulation registers share one file, so the 20
// accumulators count): the forward prune over BF16/u8 rows runs four waves per
// SIMD with a few spilled bytes (1M x 128 BF16 build: 58.1 -> 52.6 ms per step);
// over float32 rows the spills cost more than the extra wave, and FP8 builds
// with their wide visited sets are held below three waves by the LDS.
template <int DT, int SG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(DT == PECANN_BF16 || DT == PECANN_U8 ? 4 : 1))) void prune_forward_kernel(PruneParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int ccap = p.vcap + p.R;
  PruneLds s = carve_prune<DT>(smem, ccap, p.R, p.rows.metric);
  const int l = lane_id();
  for (;;) {
    const int t = next_item(p.head);
    if (t >= p.nb) break;
    const int32_t pt = p.items[t];
    // candidates: the visited set V_p, whose keys (D(p, v), v) the search has
    // already formed, then the current out-neighbours Nout(p) that are not in
    // V_p with their kept keys (R <= 128, two per lane): no distance is formed
    // before the greedy pass
    const int nv = min(p.vis_count[t], p.vcap);
    const uint64_t *v = p.vis + (int64_t)t * p.vcap;
    for (int j = l; j < nv; j += kWave) {
      const uint64_t kv = v[j];
      s.k0[j] = kv;
      s.ids[j] = key_id(kv);
    }
    const int dp = min(p.deg[pt], p.R);
    const int32_t *row = p.adj + (int64_t)pt * p.R;
    const uint64_t *krow = p.akey + (int64_t)pt * p.R;
    int32_t e0 = l < dp ? row[l] : -1;
    int32_t e1 = l + kWave < dp ? row[l + kWave] : -1;
    const uint64_t ke0 = l < dp ? krow[l] : kNoKey;
    const uint64_t ke1 = l + kWave < dp ? krow[l + kWave] : kNoKey;
    wave_lds_sync();
    if (dp > 0) {
      for (int j = 0; j < nv; ++j) {
        const int32_t vj = s.ids[j];
        if (vj == e0) e0 = -1;
        if (vj == e1) e1 = -1;
      }
    }
    const uint64_t m0 = ballot(e0 >= 0), m1 = ballot(e1 >= 0);
    if (e0 >= 0) {
      const int o = nv + lanes_below(m0);
      s.ids[o] = e0;
      s.k0[o] = ke0;
    }
    if (e1 >= 0) {
      const int o = nv + __popcll(m0) + lanes_below(m1);
      s.ids[o] = e1;
      s.k0[o] = ke1;
    }
    const int nout = __popcll(m0) + __popcll(m1);
    wave_lds_sync();
    const int rows = 32 * robust_prune_tiles<DT, SG>(p, s, pt, nv + nout, nv + nout);
    if (p.counters && l == 0) atomicAdd(p.counters + 0, (unsigned long long)rows);
    wave_lds_sync();
  }
}

// A target with more new sources than the launch's capacity (capin): the
// greedy pass of RobustPrune visits the candidates in key order and only the
// points it selects drop later ones, so it can run over the sorted candidate
// list in consecutive slices -- slice t is pruned together with the points
// selected so far, which come first in key order and drop none of each other
// again -- until R points are selected or the list ends.  The result equals one
// pass over all candidates.  A slice is the capin smallest keys not yet taken,
// bounded by bisection over the key space; the candidates are Nout(q) (two
// per lane) and the sources not already in it, whose keys stay in the
// target's segment (a source already present has its key cleared there;
// entry j of the segment is only read and written by lane j % 64).
template <int DT, int SG>
__device__ __forceinline__ int prune_reverse_sliced(const PruneParams &p, PruneLds &s, int32_t q,
                                                 uint64_t *srck, int cnt, int dq) {
  const int l = lane_id();
  const int32_t *row = p.adj + (int64_t)q * p.R;
  const uint64_t *krow = p.akey + (int64_t)q * p.R;
  const uint64_t ke0 = l < dq ? krow[l] : kNoKey;
  const uint64_t ke1 = l + kWave < dq ? krow[l + kWave] : kNoKey;
  for (int j = l; j < dq; j += kWave) s.ids[j] = row[j];
  wave_lds_sync();
  for (int j = l; j < cnt; j += kWave) {
    const int32_t v = key_id(srck[j]);
    bool present = false;
    for (int t = 0; t < dq; ++t) present |= (s.ids[t] == v);
    if (present) srck[j] = kNoKey;
  }
  wave_lds_sync();
  constexpr uint64_t kTop = kNoKey - 1;  // largest key a candidate can hold
  // candidates with keys in [lo, hi]
  auto count_in = [&](uint64_t lo, uint64_t hi) {
    int c = (ke0 >= lo && ke0 <= hi) + (ke1 >= lo && ke1 <= hi);
    for (int j = l; j < cnt; j += kWave) {
      const uint64_t k = srck[j];
      c += k >= lo && k <= hi;
    }
    return wave_sum_i32(c);
  };
  int nsel = 0, tiles = 0;
  uint64_t lo = 0;
  for (;;) {
    const int rem = count_in(lo, kTop);
    if (rem == 0) break;
    uint64_t hi = kTop;
    if (rem > p.capin) {
      uint64_t a = lo, b = kTop;  // count_in(lo, b) >= capin throughout
      while (a < b) {
        const uint64_t mid = a + (b - a) / 2;
        if (count_in(lo, mid) >= p.capin) b = mid; else a = mid + 1;
      }
      hi = b;
    }
    // the points selected so far, then the slice
    for (int j = l; j < nsel; j += kWave) {
      const uint64_t k = s.sel[j];
      s.k0[j] = k;
      s.ids[j] = key_id(k);
    }
    int m = nsel;
    {
      const bool in0 = ke0 >= lo && ke0 <= hi, in1 = ke1 >= lo && ke1 <= hi;
      const uint64_t b0 = ballot(in0), b1 = ballot(in1);
      if (in0) { const int o = m + lanes_below(b0); s.k0[o] = ke0; s.ids[o] = key_id(ke0); }
      if (in1) {
        const int o = m + __popcll(b0) + lanes_below(b1);
        s.k0[o] = ke1;
        s.ids[o] = key_id(ke1);
      }
      m += __popcll(b0) + __popcll(b1);
    }
    for (int j0 = 0; j0 < cnt; j0 += kWave) {
      const int j = j0 + l;
      const uint64_t k = j < cnt ? srck[j] : kNoKey;
      const bool in = k >= lo && k <= hi;
      const uint64_t bm = ballot(in);
      if (in) { const int o = m + lanes_below(bm); s.k0[o] = k; s.ids[o] = key_id(k); }
      m += __popcll(bm);
    }
    wave_lds_sync();
    tiles += robust_prune_tiles<DT, SG>(p, s, q, m, m);
    int v = 0;
    if (l == 0) v = p.deg[q];  // written by lane 0 in write_nout
    nsel = __shfl(v, 0);
    wave_lds_sync();
    if (nsel >= p.R || hi == kTop) break;
    lo = hi + 1;
  }
  return tiles;
}

// Three waves per SIMD for every row format but float32, with no spills: the
// compiler then gives up the accumulation registers (1M x 128 BF16 build:
// reverse prune 142.7 -> 112.9 ms per step; 1.28M x 1024 FP8: 332 -> 282 ms).
// Float32 would spill and ran slower.
template <int DT, int SG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(DT == PECANN_F32 ? 1 : 3))) void prune_reverse_kernel(PruneParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int ccap = p.R + p.capin;
  PruneLds s = carve_prune<DT>(smem, ccap, p.R, p.rows.metric);
  const int l = lane_id();
  const int nt = *p.ntargets;
  const int items = p.heavy ? *p.nheavy : *p.nlight;
  // light targets are many and short: a wave takes kLightChunk of them per
  // queue atomic so that the queue head is not the serialising point
  constexpr int kLightChunk = 8;
  const int chunk = p.heavy ? 1 : kLightChunk;
  int it = 0, end = 0, base = 0;
  // light chunks: lane i holds target base + i's list entry, node, source count,
  // segment offset and degree, all loaded at once when the chunk is taken (the
  // targets of a launch are distinct, so no earlier item changes them)
  int32_t pf_q = 0, pf_cnt = 0, pf_off = 0, pf_deg = 0;
  for (;;) {
    if (it >= end) {
      int v = 0;
      if (l == 0) v = atomicAdd(p.head, chunk);
      it = __shfl(v, 0);
      if (it >= items) break;
      end = min(items, it + chunk);
      base = it;
      if (!p.heavy && l < end - base) {
        const int32_t uu = p.tord[base + l];
        pf_q = p.tlist[uu];
        pf_cnt = p.tcnt[uu];
        pf_off = p.toff[uu];
        pf_deg = p.deg[pf_q];
      }
    }
    int32_t q, cnt, off, dg;
    if (!p.heavy) {
      const int i = it - base;
      q = __builtin_amdgcn_readlane(pf_q, i);
      cnt = __builtin_amdgcn_readlane(pf_cnt, i);
      off = __builtin_amdgcn_readlane(pf_off, i);
      dg = __builtin_amdgcn_readlane(pf_deg, i);
    } else {
      const int u = p.tord[nt - 1 - it];
      q = p.tlist[u];
      cnt = p.tcnt[u];
      off = p.toff[u];
      dg = p.deg[q];
    }
    ++it;
    // each source p arrives with its key (D(p, q), p) and each out-neighbour
    // with its kept key, so neither an append nor a prune forms a distance to q
    const int32_t *src = p.seg + off;
    const uint64_t *srck = p.segk + off;
    const int dq = min(dg, p.R);
    PECANN_CHECK(q >= 0 && q < p.n && dg >= 0 && dg <= p.R, CK_PRUNE);
    PECANN_CHECK(p.heavy || cnt <= p.capin, CK_PRUNE);  // light targets fit the LDS
    if (cnt > p.capin) {
      // more sources than the LDS holds (heavy list only: light targets have
      // at most capin by construction); more than capin - R of them are new,
      // so the target is always pruned
      const int rows = 32 * prune_reverse_sliced<DT, SG>(p, s, q, p.segk + off, cnt, dq);
      if (p.counters && l == 0) {
        atomicAdd(p.counters + 1, (unsigned long long)rows);
        atomicAdd(p.counters + 2, 1ull);
      }
      if (l == 0) p.rcnt[q] = 0;
      wave_lds_sync();
      continue;
    }
    int32_t *row = p.adj + (int64_t)q * p.R;
    uint64_t *krow = p.akey + (int64_t)q * p.R;
    int nnew = 0;
    if (!p.heavy) {
      // at most 64 sources (one per lane) and R <= 128 out-neighbours (two per
      // lane): membership and ascending order come from ballots and lane reads,
      // and an append never touches the LDS
      const uint64_t kv = l < cnt ? srck[l] : kNoKey;
      const int32_t v = l < cnt ? (int32_t)key_id(kv) : -1;
      const int32_t e0 = l < dq ? row[l] : -1;
      const int32_t e1 = l + kWave < dq ? row[l + kWave] : -1;
      uint64_t pres = 0;
      for (int t = 0; t < cnt; ++t) {
        const int32_t vt = __builtin_amdgcn_readlane(v, t);
        if (ballot(e0 == vt || e1 == vt)) pres |= 1ull << t;
      }
      const bool keep = l < cnt && !((pres >> l) & 1ull);
      const uint64_t km = ballot(keep);
      int r = 0;  // rank among the kept sources by index
      for (uint64_t m = km; m; m &= m - 1)
        r += __builtin_amdgcn_readlane(v, __builtin_ctzll(m)) < v;
      nnew = __popcll(km);
      if (dq + nnew <= p.R) {
        if (keep) {
          row[dq + r] = v;
          krow[dq + r] = kv;
        }
      } else {
        if (l < dq) {
          s.ids[l] = e0;
          s.k0[l] = krow[l];
        }
        if (l + kWave < dq) {
          s.ids[l + kWave] = e1;
          s.k0[l + kWave] = krow[l + kWave];
        }
        if (keep) {
          s.ids[dq + r] = v;
          s.k0[dq + r] = kv;
        }
      }
    } else {
      // current out-neighbours, then the new sources in ascending index order,
      // leaving out sources already among the out-neighbours (the sources of
      // one batch are distinct; their ids are staged in s.k0, free until the
      // keys are gathered, and ranked there, and their keys land in s.k1 at
      // their rank)
      int32_t *stage = (int32_t *)s.k0;
      for (int j = l; j < dq; j += kWave) s.ids[j] = row[j];
      for (int j = l; j < cnt; j += kWave) stage[j] = src[j];
      wave_lds_sync();
      for (int j = l; j < cnt; j += kWave) {
        const int32_t v = stage[j];
        int r = 0;
        for (int t = 0; t < cnt; ++t) r += stage[t] < v;
        bool present = false;
        for (int t = 0; t < dq; ++t) present |= (s.ids[t] == v);
        s.k1[r] = present ? kNoKey : srck[j];
      }
      wave_lds_sync();
      for (int base = 0; base < cnt; base += kWave) {
        const int j = base + l;
        const uint64_t kv = j < cnt ? s.k1[j] : kNoKey;
        const uint64_t bm = ballot(kv != kNoKey);
        if (kv != kNoKey) {
          const int o = dq + nnew + lanes_below(bm);
          s.ids[o] = (int32_t)key_id(kv);
          s.k0[o] = kv;
        }
        nnew += __popcll(bm);
      }
      wave_lds_sync();
      if (dq + nnew <= p.R) {
        for (int j = l; j < nnew; j += kWave) {
          row[dq + j] = s.ids[dq + j];
          krow[dq + j] = s.k0[dq + j];
        }
      } else {
        for (int j = l; j < dq; j += kWave) s.k0[j] = krow[j];
      }
    }
    wave_lds_sync();
    if (dq + nnew <= p.R) {
      if (l == 0) p.deg[q] = dq + nnew;
      if (p.counters && l == 0) atomicAdd(p.counters + 3, 1ull);
    } else {
      // the leading entries that q's last prune selected need no tiles among themselves
      int tiles = -1;
      if (!p.heavy) tiles = prune_with_prefix<DT, SG>(p, s, q, dq + nnew, min(p.cons[q], dq));
      if (tiles < 0) tiles = robust_prune_tiles<DT, SG>(p, s, q, dq + nnew, dq + nnew);
      const int rows = 32 * tiles;
      if (p.counters && l == 0) {
        atomicAdd(p.counters + 1, (unsigned long long)rows);
        atomicAdd(p.counters + 2, 1ull);
      }
    }
    if (l == 0) p.rcnt[q] = 0;
    wave_lds_sync();
  }
}

// NN-descent graph: Nout(i) = RobustPrune(i, list_i u rev_i) for every point.
template <int DT>
__global__ __launch_bounds__(64) void prune_lists_kernel(PruneParams p) {
  extern __shared__ __align__(16) uint8_t smem[];
  PruneLds s = carve_prune<DT>(smem, 2 * p.lk, p.R, p.rows.metric);
  const int l = lane_id();
  for (;;) {
    const int u = next_item(p.head);
    if (u >= p.n) break;
    for (int j = l; j < p.lk; j += kWave) {
      const uint64_t k = p.lists[(int64_t)u * p.lk + j];
      s.ids[j] = k == kNoKey ? -1 : key_id(k);
      s.ids[p.lk + j] = p.rlists[(int64_t)u * p.lk + j];
    }
    wave_lds_sync();
    const int rows = 32 * robust_prune_tiles<DT, tile_steps_rule<DT>()>(p, s, u, 2 * p.lk);
    if (p.counters && l == 0) atomicAdd(p.counters + 0, (unsigned long long)rows);
    wave_lds_sync();
  }
}

size_t prune_lds_bytes(int ccap, int R, int dt, int metric) {
  const size_t per = 8 + 8 + 4 + 1 + (prune_has_norms(metric) ? 4 : 0) + (prune_has_scales(dt, metric) ? 4 : 0);
  return (size_t)ccap * per + 8 * (size_t)R + 16;
}

// The tile steps per memory round trip: the tuning's (2 or 4), else the rule.
template <int DT>
static hipError_t launch_pf_t(const PruneParams &p, int grid, hipStream_t st) {
  const size_t lds = prune_lds_bytes(p.vcap + p.R, p.R, DT, p.rows.metric);
  if ((p.sg ? p.sg : tile_steps_rule<DT>()) == 4)
    hipLaunchKernelGGL((prune_forward_kernel<DT, 4>), dim3(grid), dim3(64), lds, st, p);
  else
    hipLaunchKernelGGL((prune_forward_kernel<DT, 2>), dim3(grid), dim3(64), lds, st, p);
  return hipGetLastError();
}
template <int DT>
static hipError_t launch_pr_t(const PruneParams &p, int grid, hipStream_t st) {
  const size_t lds = prune_lds_bytes(p.R + p.capin, p.R, DT, p.rows.metric);
  if ((p.sg ? p.sg : tile_steps_rule<DT>()) == 4)
    hipLaunchKernelGGL((prune_reverse_kernel<DT, 4>), dim3(grid), dim3(64), lds, st, p);
  else
    hipLaunchKernelGGL((prune_reverse_kernel<DT, 2>), dim3(grid), dim3(64), lds, st, p);
  return hipGetLastError();
}

template <int DT>
static hipError_t launch_pl_t(const PruneParams &p, int grid, hipStream_t st) {
  hipLaunchKernelGGL((prune_lists_kernel<DT>), dim3(grid), dim3(64), prune_lds_bytes(2 * p.lk, p.R, DT, p.rows.metric), st,
                     p);
  return hipGetLastError();
}

hipError_t launch_prune_lists(int32_t dt, const PruneParams &p, int grid, hipStream_t st) {
  switch (dt) {
    case PECANN_F32: return launch_pl_t<PECANN_F32>(p, grid, st);
    case PECANN_U8: return launch_pl_t<PECANN_U8>(p, grid, st);
    case PECANN_BF16: return launch_pl_t<PECANN_BF16>(p, grid, st);
    case PECANN_FP8E4M3: return launch_pl_t<PECANN_FP8E4M3>(p, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prune_forward(int32_t dt, const PruneParams &p, int grid, hipStream_t st) {
  switch (dt) {
    case PECANN_F32: return launch_pf_t<PECANN_F32>(p, grid, st);
    case PECANN_U8: return launch_pf_t<PECANN_U8>(p, grid, st);
    case PECANN_BF16: return launch_pf_t<PECANN_BF16>(p, grid, st);
    case PECANN_FP8E4M3: return launch_pf_t<PECANN_FP8E4M3>(p, grid, st);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_prune_reverse(int32_t dt, const PruneParams &p, int grid, hipStream_t st) {
  switch (dt) {
    case PECANN_F32: return launch_pr_t<PECANN_F32>(p, grid, st);
    case PECANN_U8: return launch_pr_t<PECANN_U8>(p, grid, st);
    case PECANN_BF16: return launch_pr_t<PECANN_BF16>(p, grid, st);
    case PECANN_FP8E4M3: return launch_pr_t<PECANN_FP8E4M3>(p, grid, st);
    default: return hipErrorInvalidValue;
  }
}

PECANN_CHECK_READER(prune)

}  // namespace pecann
