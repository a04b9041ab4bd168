// K8/K9 RobustPrune of DiskANN (the Vamana pruning rule the paper adopts,
// Sec. 3.2), one wavefront per pruned point:
//   sort the candidates by (D(p, c), c), drop p, duplicates and -1;
//   repeatedly move the closest surviving candidate c* to the output (stop at
//   R) and drop every surviving c with alpha * D(c*, c) <= D(p, c)
//   (alpha^2 * D^2 <= D^2 for L2 measures, which are squared distances).
// Candidate-pair distances are dense 16 x 16 dot-product tiles on the matrix
// cores (f32, i8, bf16 or fp8 MFMA by row format), turned into distances with
// the rows' stored norms; distances to p are direct differences.
// prune_forward: Nout(p) = RobustPrune(p, V_p u Nout(p)) for each point of a batch.
// prune_reverse: for each target q of the batch's reverse edges, append the
//   new sources not yet present (ascending index) if they fit in R, else
//   Nout(q) = RobustPrune(q, Nout(q) u sources).
#include "beam.hpp"

namespace pecann {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct PruneLds {
  int32_t *ids;    // candidates [ccap]
  uint64_t *k0;    // keys [ccap]
  uint64_t *k1;    // sorted keys [ccap]
  uint32_t *cn;    // squared norm of each sorted candidate [ccap]
  float *cs;       // row scale of each sorted candidate (FP8) [ccap]
  float *dg;       // 16 x 16 measures of the current diagonal tile
  int32_t *sel;    // selected [R]
  uint8_t *alive;  // [ccap]
};

__device__ __forceinline__ PruneLds carve_prune(uint8_t *smem, int ccap, int R) {
  PruneLds s;
  s.k0 = (uint64_t *)smem;
  s.k1 = s.k0 + ccap;
  s.ids = (int32_t *)(s.k1 + ccap);
  s.cn = (uint32_t *)(s.ids + ccap);
  s.cs = (float *)(s.cn + ccap);
  s.dg = s.cs + ccap;
  s.sel = (int32_t *)(s.dg + 256);
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

// 16 x 16 tile of dot products between search rows on the matrix cores.  Lane
// l contributes row (l % 16) of the A tile (arow) and of the B tile (brow);
// at step s it loads 16-byte chunk (l / 16) + 4 s of each.  The result is the
// MFMA accumulator layout: register r of lane l holds A-row 4 (l / 16) + r
// against B-row l % 16.  U8 rows are shifted to signed (x - 128) so that the
// integer dot is exact.  Missing rows (-1) contribute zeros.
template <int DT>
__device__ __forceinline__ v4f dot_tile(const Rows &r, int32_t arow, int32_t brow) {
  const int g = lane_id() >> 4;
  const uint8_t *pa = r.xs + (int64_t)(arow < 0 ? 0 : arow) * r.xs_stride;
  const uint8_t *pb = r.xs + (int64_t)(brow < 0 ? 0 : brow) * r.xs_stride;
  const int steps = (r.nch + 3) >> 2;
  v4f accf = {0.f, 0.f, 0.f, 0.f};
  v4i acci = {0, 0, 0, 0};
  for (int st = 0; st < steps; ++st) {
    const int q = g + 4 * st;
    uint4 a = make_uint4(0, 0, 0, 0), b = make_uint4(0, 0, 0, 0);
    if (q < r.nch) {
      if (arow >= 0) a = *(const uint4 *)(pa + 16 * q);
      if (brow >= 0) b = *(const uint4 *)(pb + 16 * q);
      if (DT == PECANN_U8) {
        if (arow >= 0) { a.x ^= 0x80808080u; a.y ^= 0x80808080u; a.z ^= 0x80808080u; a.w ^= 0x80808080u; }
        if (brow >= 0) { b.x ^= 0x80808080u; b.y ^= 0x80808080u; b.z ^= 0x80808080u; b.w ^= 0x80808080u; }
      }
    }
    if (DT == PECANN_F32) {
      accf = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), accf, 0, 0, 0);
      accf = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), accf, 0, 0, 0);
      accf = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), accf, 0, 0, 0);
      accf = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), accf, 0, 0, 0);
    } else if (DT == PECANN_U8) {
      const v4i ai = {(int)a.x, (int)a.y, (int)a.z, (int)a.w};
      const v4i bi = {(int)b.x, (int)b.y, (int)b.z, (int)b.w};
      acci = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai, bi, acci, 0, 0, 0);
    } else if (DT == PECANN_BF16) {
      const v8bf ab = __builtin_bit_cast(v8bf, a);
      const v8bf bb = __builtin_bit_cast(v8bf, b);
      accf = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, accf, 0, 0, 0);
    } else {  // FP8 e4m3: two 8-byte halves
      const long a0 = (long)(((uint64_t)a.y << 32) | a.x), a1 = (long)(((uint64_t)a.w << 32) | a.z);
      const long b0 = (long)(((uint64_t)b.y << 32) | b.x), b1 = (long)(((uint64_t)b.w << 32) | b.z);
      accf = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, accf, 0, 0, 0);
      accf = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, accf, 0, 0, 0);
    }
  }
  if (DT == PECANN_U8) {
    // keep the exact integer dot in the float lanes' bits
    return v4f{__int_as_float(acci[0]), __int_as_float(acci[1]), __int_as_float(acci[2]),
               __int_as_float(acci[3])};
  }
  return accf;
}

// Measure (squared L2, or cosine distance) from a dot product and the two rows'
// norms / scales, as the search keys define it.
template <int DT>
__device__ __forceinline__ float pair_measure(float dotv, uint32_t na, uint32_t nb, float sa, float sb,
                                              int metric) {
  if (DT == PECANN_U8) {
    const int d2 = (int)na + (int)nb - 2 * __float_as_int(dotv);
    return (float)(d2 < 0 ? 0 : d2);
  }
  const float dt = (DT == PECANN_FP8E4M3) ? dotv * sa * sb : dotv;
  if (metric == PECANN_L2) return fmaxf(0.f, __uint_as_float(na) + __uint_as_float(nb) - 2.0f * dt);
  return fmaxf(0.f, 1.0f - dt);
}

// RobustPrune of point pt over s.ids[0..nc); writes Nout(pt) into adj/deg.
// Candidates are sorted by (D(pt, c), c) from direct-difference distances.  The
// greedy pass then walks them in blocks of 16: one matrix-core tile gives the
// block's own pairwise distances, which settle the block's selections in
// order; the block's selected points then drop later candidates tile by tile,
// each lane testing the 4 rows of its accumulator against its column.
// Returns the number of 16 x 16 tiles formed.
template <int DT, int G>
__device__ int robust_prune_tiles(const PruneParams &p, Engine<DT, G> &eng, PruneLds &s, int32_t pt,
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
  int mv = 0;  // valid (non-empty) sorted entries
  for (int j0 = 0; j0 < nc; j0 += kWave) {
    const int j = j0 + l;
    const uint64_t key = j < nc ? s.k1[j] : kNoKey;
    const bool valid = key != kNoKey;
    if (j < nc) {
      s.alive[j] = valid && (j == 0 || s.k1[j - 1] != key);
      if (valid) {
        const int32_t id = key_id(key);
        s.cn[j] = p.rows.sqn[id];
        s.cs[j] = (DT == PECANN_FP8E4M3) ? p.rows.scale[id] : 1.0f;
      }
    }
    mv += __popcll(ballot(valid));
  }
  wave_lds_sync();

  const int col = l & 15, g = l >> 4;
  int nsel = 0, tiles = 0;
  for (int b = 0; b < mv && nsel < p.R; b += 16) {
    if (ballot(col + b < mv && l < 16 && s.alive[b + col]) == 0) continue;
    // (a) the block's own 16 x 16 tile
    const int32_t rb = b + col < mv ? key_id(s.k1[b + col]) : -1;
    v4f t = dot_tile<DT>(p.rows, rb, rb);
    ++tiles;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * g + r;
      float m = 0.f;
      if (b + i < mv && b + col < mv)
        m = pair_measure<DT>(t[r], s.cn[b + i], s.cn[b + col], s.cs[b + i], s.cs[b + col],
                             p.rows.metric);
      s.dg[i * 16 + col] = m;
    }
    wave_lds_sync();
    // (b) selections of this block, in order
    uint32_t selmask = 0;
    for (int i = 0; i < 16 && b + i < mv; ++i) {
      if (!s.alive[b + i]) continue;
      if (l == 0) { s.sel[nsel] = key_id(s.k1[b + i]); s.alive[b + i] = 0; }
      selmask |= 1u << i;
      ++nsel;
      if (nsel == p.R) break;
      if (l > i && l < 16 && b + l < mv && s.alive[b + l] &&
          a2 * s.dg[i * 16 + l] <= key_measure(s.k1[b + l]))
        s.alive[b + l] = 0;
      wave_lds_sync();
    }
    wave_lds_sync();
    if (nsel == p.R) break;
    // (c) the block's selected points drop later candidates
    const int32_t ra = rb;
    for (int j0 = b + 16; j0 < mv; j0 += 16) {
      if (ballot(l < 16 && j0 + l < mv && s.alive[j0 + l]) == 0) continue;
      const int32_t rj = j0 + col < mv ? key_id(s.k1[j0 + col]) : -1;
      v4f tt = dot_tile<DT>(p.rows, ra, rj);
      ++tiles;
      bool kill = false;
      if (j0 + col < mv) {
        const float dpc = key_measure(s.k1[j0 + col]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * g + r;
          if ((selmask >> i) & 1u) {
            const float m = pair_measure<DT>(tt[r], s.cn[b + i], s.cn[j0 + col], s.cs[b + i],
                                             s.cs[j0 + col], p.rows.metric);
            kill |= a2 * m <= dpc;
          }
        }
      }
      const uint64_t km = ballot(kill);
      const uint32_t k16 = (uint32_t)((km | (km >> 16) | (km >> 32) | (km >> 48)) & 0xffffu);
      if (l < 16 && ((k16 >> l) & 1u)) s.alive[j0 + l] = 0;
      wave_lds_sync();
    }
  }
  int32_t *row = p.adj + (int64_t)pt * p.R;
  for (int e = l; e < p.R; e += kWave) row[e] = e < nsel ? s.sel[e] : -1;
  if (l == 0) p.deg[pt] = nsel;
  return tiles;
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
    const int rows = nv + dp + 32 * robust_prune_tiles<DT, G>(p, eng, s, pt, nv + dp);
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
      ((int32_t *)s.k0)[r] = present ? -1 : v;
    }
    wave_lds_sync();
    int nnew = 0;
    for (int base = 0; base < cnt; base += kWave) {
      const int j = base + l;
      const int32_t v = j < cnt ? ((const int32_t *)s.k0)[j] : -1;
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
      const int rows = dq + nnew + 32 * robust_prune_tiles<DT, G>(p, eng, s, q, dq + nnew);
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
  return (size_t)ccap * (8 + 8 + 4 + 4 + 4 + 1) + 4 * 256 + 4 * (size_t)((R + 3) & ~3) + 16;
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
