// Exact kNN on the matrix cores (the BruteForce index of Sec. 4.1 at scale).
//
// scan:   a workgroup of 4 wavefronts takes 64 queries (16 per wavefront) and
//         streams one of kParts consecutive parts of the points past them in
//         blocks of 64 candidates, each block in rounds of kSPB 64-byte steps.  A round's candidate chunks are
//         staged through a double-buffered LDS tile; the loads of the next
//         round (candidate chunks, the wavefront's query chunks, the block's
//         norms) are issued before the products of the current one, so the
//         memory latency of a round hides behind the matrix work of the one
//         before.  Each wavefront forms a 16 x 64 block of dot products (f32
//         16x16x4, or i8 16x16x64 on uint8 rows shifted to x - 128, which is
//         exact) and turns them into distance measures with the stored row
//         norms.  Every lane keeps, for each of its 4 query rows, the kKQ
//         smallest (measure, index) pairs of its column stream in registers.
// rerank: one wavefront per query re-scores the kParts x 16 x kKQ kept candidates by
//         direct differences -- the same float32 arithmetic as the brute-force
//         kernel -- and keeps the k best.  A candidate the scan dropped had a
//         matrix-core measure >= thr (the smallest value any queue dropped), so
//         its exact measure is >= thr - E, with E a bound on the rounding of
//         |a|^2 + |b|^2 - 2 a.b; if the k-th re-scored measure is < thr - E the
//         answer is exact, otherwise the query goes to the brute-force kernel.
//         uint8 measures are exact integers on both sides (E = 0), so there the
//         (measure, index) keys are compared: a tie with a dropped candidate
//         of larger index is no reason to fall back.
#include "beam.hpp"

namespace pecann {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kQT = 64;   // queries per workgroup
constexpr int kCT = 64;   // candidates per block
// The points are scanned in kParts parts by separate workgroups, each keeping
// its own queues: twice the workgroups of one full scan, so that the last
// wave of workgroups fills the GPU better (70,000 points: 2,188 workgroups
// over 768 resident at three waves per SIMD, against 1,094), and half the
// queue length per lane for the same kExactCand kept candidates per query.
// Measured on 70,000 x 784 rows: uint8 scan 20.3 -> 17.9 ms, float32 94.7 ->
// 82.6 ms (plus 1.4 ms of brute force for the queries whose shorter queues
// fail the exactness check); four waves per SIMD (1,024 resident, a short
// last wave) made the uint8 scan slower, 24.7 ms.
constexpr int kParts = kExactParts;
// queue length per lane and query row (a lane's stream is one sixteenth of a
// part); the inserts of a wave are divergent, so a shorter queue is also a
// cheaper one.  With one part, four per lane sent ~0.3 % of the 70,000-point
// uint8 queries to the brute force (a lane holding five of a query's ten
// nearest); two parts give each query 32 streams of four.
constexpr int kKQ = kExactCand / (16 * kParts);
constexpr int kSPB = 4;   // 64-byte steps per round
constexpr int kCand = kExactCand;

struct ScanRows {
  const uint8_t *rows;
  int64_t stride;          // bytes
  int32_t nch;             // 16-byte chunks per row
  const uint32_t *norms;   // float bits (F32) or int32 (U8)
};


__device__ __forceinline__ uint4 shift_u8(uint4 v) {
  v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
  return v;
}

// The global loads of one round: this thread's candidate chunks (row
// tid / 4, chunks tid % 4 + 4 step), its lane's query chunks (row of A: the
// lane's query, chunks g + 4 step) and, with a block's first round, the norm
// of candidate tid.  Loads are not guarded by branches (indices are clamped;
// chunks past the row are zeroed after all loads are out), so they issue back
// to back.
template <int SDT>
struct Round {
  uint4 b[kSPB], a[kSPB];
  uint32_t nrm;
  __device__ __forceinline__ void load(const ScanRows &sr, int32_t n, int tid, int g, int qa, int cb,
                                       int step0, bool first) {
    const int br = min(cb + (tid >> 2), n - 1);
    const uint8_t *pb = sr.rows + (int64_t)br * sr.stride;
    const uint8_t *pa = sr.rows + (int64_t)min(qa, n - 1) * sr.stride;
    int cbq[kSPB], caq[kSPB];
#pragma unroll
    for (int u = 0; u < kSPB; ++u) {
      cbq[u] = (tid & 3) + 4 * (step0 + u);
      caq[u] = g + 4 * (step0 + u);
      b[u] = *(const uint4 *)(pb + 16 * min(cbq[u], sr.nch - 1));
      a[u] = *(const uint4 *)(pa + 16 * min(caq[u], sr.nch - 1));
    }
    nrm = (first && tid < kCT) ? sr.norms[min(cb + tid, n - 1)] : 0u;
    // uint8 rows are shifted to signed first; chunks past the row are zero
    // after the shift (they add nothing to a dot product)
#pragma unroll
    for (int u = 0; u < kSPB; ++u) {
      if (SDT == PECANN_U8) {
        b[u] = shift_u8(b[u]);
        a[u] = shift_u8(a[u]);
      }
      if (cbq[u] >= sr.nch) b[u] = make_uint4(0, 0, 0, 0);
      if (caq[u] >= sr.nch) a[u] = make_uint4(0, 0, 0, 0);
    }
  }
};

template <int SDT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void exact_scan_kernel(ScanRows sr, int32_t n, int32_t metric,
                                                         int32_t *cand, uint64_t *thr) {
  __shared__ uint4 bs[2][kCT][4 * kSPB + 1];
  __shared__ uint32_t bn[2][kCT];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  const int q0 = blockIdx.x * kQT + 16 * w;  // this wavefront's first query
  const int qa = q0 + c16;                    // the query row this lane feeds as A
  const int steps = (sr.nch + 3) >> 2;
  const int rpb = (steps + kSPB - 1) / kSPB;  // rounds per block
  // this workgroup's part: candidate blocks [b0, b1) (possibly none)
  const int part = blockIdx.y;
  const int nblk = (n + kCT - 1) / kCT;
  const int b0 = (int)((int64_t)nblk * part / kParts), b1 = (int)((int64_t)nblk * (part + 1) / kParts);
  const int total = (b1 - b0) * rpb;

  // the lane's queue of row r: keys (measure bits << 32 | candidate), sorted;
  // one 64-bit comparison orders (measure, index) pairs
  uint64_t qk[4][kKQ];
  uint64_t qlo[4];  // smallest key this lane's queue of row r has dropped
  float nq[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = q0 + 4 * g + r;
    qlo[r] = kNoKey;
    nq[r] = 0.f;
    if (q < n) nq[r] = SDT == PECANN_U8 ? (float)(int)sr.norms[q] : __uint_as_float(sr.norms[q]);
#pragma unroll
    for (int s = 0; s < kKQ; ++s) qk[r][s] = kNoKey;
  }

  v4f accf[4];
  v4i acci[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) { accf[t] = v4f{0.f, 0.f, 0.f, 0.f}; acci[t] = v4i{0, 0, 0, 0}; }
  Round<SDT> nxt;
  nxt.load(sr, n, tid, g, qa, b0 * kCT, 0, true);
  for (int rd = 0; rd < total; ++rd) {
    const int blk = b0 + rd / rpb, rr = rd % rpb, buf = rd & 1;
    // stage this round (its loads were issued during the previous round)
#pragma unroll
    for (int u = 0; u < kSPB; ++u) bs[buf][tid >> 2][4 * u + (tid & 3)] = nxt.b[u];
    if (rr == 0 && tid < kCT) bn[blk & 1][tid] = nxt.nrm;
    uint4 av[kSPB];
#pragma unroll
    for (int u = 0; u < kSPB; ++u) av[u] = nxt.a[u];
    // one barrier per round: the tile written now was last read in round
    // rd - 2, and every wavefront has passed this barrier's predecessor since
    __syncthreads();
    if (rd + 1 < total) {
      const int nb = b0 + (rd + 1) / rpb, nr = (rd + 1) % rpb;
      nxt.load(sr, n, tid, g, qa, nb * kCT, nr * kSPB, nr == 0);
    }
#pragma unroll
    for (int u = 0; u < kSPB; ++u) {
      if (rr * kSPB + u >= steps) break;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint4 b = bs[buf][16 * t + c16][4 * u + g];
        if (SDT == PECANN_U8) {
          const v4i ai = {(int)av[u].x, (int)av[u].y, (int)av[u].z, (int)av[u].w};
          const v4i bi = {(int)b.x, (int)b.y, (int)b.z, (int)b.w};
          acci[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai, bi, acci[t], 0, 0, 0);
        } else {
          accf[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av[u].x), __uint_as_float(b.x), accf[t], 0, 0, 0);
          accf[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av[u].y), __uint_as_float(b.y), accf[t], 0, 0, 0);
          accf[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av[u].z), __uint_as_float(b.z), accf[t], 0, 0, 0);
          accf[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av[u].w), __uint_as_float(b.w), accf[t], 0, 0, 0);
        }
      }
    }
    if (rr != rpb - 1) continue;
    // the block's last round: its measures into the lane's queues
    const int cb = blk * kCT;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = cb + 16 * t + c16;
      const uint32_t nbits = bn[blk & 1][16 * t + c16];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = q0 + 4 * g + r;
        if (col >= n || q >= n || col == q) continue;
        float m;
        if (SDT == PECANN_U8) {
          const int d2 = (int)nq[r] + (int)nbits - 2 * acci[t][r];
          m = (float)(d2 < 0 ? 0 : d2);
        } else if (metric == PECANN_L2) {
          m = fmaxf(0.f, nq[r] + __uint_as_float(nbits) - 2.0f * accf[t][r]);
        } else {
          m = fmaxf(0.f, 1.0f - accf[t][r]);
        }
        // measures are >= 0; clearing the sign bit keeps a -0 from ordering last
        m = __uint_as_float(__float_as_uint(m) & 0x7fffffffu);
        const uint64_t ck = make_key(m, col);
        if (!(ck < qk[r][kKQ - 1])) {
          qlo[r] = min(qlo[r], ck);  // rejected
        } else {
          qlo[r] = min(qlo[r], qk[r][kKQ - 1]);  // the entry it evicts (~0: an empty slot)
#pragma unroll
          for (int s = kKQ - 1; s > 0; --s) {
            const bool shift = ck < qk[r][s - 1];
            const bool here = !shift && ck < qk[r][s];
            qk[r][s] = shift ? qk[r][s - 1] : (here ? ck : qk[r][s]);
          }
          if (ck < qk[r][0]) qk[r][0] = ck;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) { accf[t] = v4f{0.f, 0.f, 0.f, 0.f}; acci[t] = v4i{0, 0, 0, 0}; }
  }

  // queues out (this part's slice of the query's candidates); thr = smallest
  // key any of the 16 lanes of a row dropped (a lane that kept all of a
  // query's best candidates dropped none of them), one per part
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = q0 + 4 * g + r;
    uint64_t last = qlo[r];
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) last = min(last, shfl_xor_u64(last, m));
    if (q < n) {
      int32_t *o = cand + (int64_t)q * kCand + (part * 16 + c16) * kKQ;
#pragma unroll
      for (int s = 0; s < kKQ; ++s) o[s] = key_id(qk[r][s]);  // an empty slot gives -1
      if (c16 == 0) thr[(int64_t)q * kParts + part] = last;
    }
  }
}

__global__ __launch_bounds__(1024) void norm_max_kernel(const uint32_t *norms, int32_t n, float *out) {
  __shared__ float part[16];
  float m = 0.f;
  for (int i = threadIdx.x; i < n; i += 1024) m = fmaxf(m, __uint_as_float(norms[i]));
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s));
  if (lane_id() == 0) part[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x < 64) {
    float v = threadIdx.x < 16 ? part[threadIdx.x] : 0.f;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v = fmaxf(v, __shfl_xor(v, s));
    if (threadIdx.x == 0) *out = v;
  }
}

}  // namespace

// One wavefront per query: exact re-score of the scan's candidates, check, output.
template <int DT, int S>
__global__ __launch_bounds__(64) void exact_rerank_kernel(ExactMfmaParams p, float ce, int u8rows) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int k = p.k;
  const int kp = (k + 15) & ~15;
  SortedList top;
  top.a = (uint64_t *)smem;
  top.b = top.a + kp;
  top.tmp = top.b + kp;
  uint64_t *kb = top.tmp + 64;  // keys of the current 64 candidates
  top.fa = (uint8_t *)(kb + 64);
  top.fb = top.fa + kp;
  top.cap = k;
  ExactEngine<DT, S> eng;
  const int l = lane_id();
  for (;;) {
    const int q = next_item(p.head);
    if (q >= p.n) break;
    eng.load_query(p.rows, q);
    top.reset();
    wave_lds_sync();
    const int32_t *c = p.cand + (int64_t)q * kCand;
    static_assert(kCand % kWave == 0, "candidates are re-scored 64 at a time");
    for (int base = 0; base < kCand; base += kWave) {
      PECANN_CHECK(c[base + l] >= -1 && c[base + l] < p.n, CK_ITEM);  // (-1: none)
      score_keys(eng, p.rows, kWave, [&](int i) { return c[base + i]; }, kb);
      wave_lds_sync();
      const uint64_t key = kb[l];
      wave_lds_sync();
      top.merge(key);
    }
    bool ok = top.m == k;
    if (ok) {
      // rounding bound of the matrix-core measure against the exact one
      float nqv;
      if (u8rows) nqv = 0.f;
      else nqv = p.rows.xr ? p.rows.sqn_r[q] : __uint_as_float(p.rows.sqn[q]);
      const float e = u8rows ? ce : ce * (nqv + *p.nmax);
      uint64_t tk = p.thr[(int64_t)q * kParts];
      for (int t = 1; t < kParts; ++t) tk = min(tk, p.thr[(int64_t)q * kParts + t]);
      if (tk == kNoKey) ok = true;  // no queue dropped anything
      else if (u8rows) ok = top.a[k - 1] < tk;
      else ok = key_measure(top.a[k - 1]) < key_measure(tk) - e;
    }
    if (ok) {
      // rows, outputs and ids of this call are the instance's: global index =
      // base + local index
      const int64_t o = (int64_t)q * p.kstride;
      for (int t = l; t < p.kstride; t += kWave) {
        const uint64_t kt = t < k ? top.a[t] : kNoKey;
        p.knn_idx[o + t] = t < k ? key_id(kt) + p.base : -1;
        p.knn_dist[o + t] = t < k ? measure_to_dist(key_measure(kt), p.rows.metric)
                                  : __int_as_float(0x7f800000);
      }
      if (l == 0) {
        const uint64_t kk = top.a[k - 1];
        p.rho[q] = 1.0f / measure_to_dist(key_measure(kk), p.rows.metric);
        p.rank_key[q] = (kk & 0xffffffff00000000ull) | (uint32_t)(q + p.base);
      }
    } else if (l == 0) {
      p.fb_list[atomicAdd(p.fb_count, 1)] = q + p.base;
    }
    wave_lds_sync();
  }
}

template <int DT, int S>
static hipError_t launch_rerank_t(const ExactMfmaParams &p, float ce, int u8rows, int grid,
                                  hipStream_t st) {
  if constexpr (S > max_shape(DT)) {
    return hipErrorInvalidValue;
  } else {
    const size_t kp = (size_t)((p.k + 15) & ~15);
    hipLaunchKernelGGL((exact_rerank_kernel<DT, S>), dim3(grid), dim3(64), 8 * (2 * kp + 128) + 2 * kp,
                       st, p, ce, u8rows);
    return hipGetLastError();
  }
}

static hipError_t launch_rerank(int32_t dt, int S, const ExactMfmaParams &p, float ce, int u8rows,
                                int grid, hipStream_t st) {
  PECANN_DISPATCH_SHAPE(launch_rerank_t, dt, S, p, ce, u8rows, grid, st)
}

hipError_t launch_exact_mfma(int32_t dt, int S, const ExactMfmaParams &p, hipStream_t st) {
  const Rows &r = p.rows;
  ScanRows sr;
  const bool u8 = dt == PECANN_U8;
  if (dt == PECANN_F32 || u8) {
    sr.rows = r.xs;
    sr.stride = r.xs_stride;
    sr.nch = r.nch;
    sr.norms = r.sqn;
  } else {
    sr.rows = (const uint8_t *)r.xr;
    sr.stride = r.xr_stride * 4;
    sr.nch = r.nch_r;
    sr.norms = (const uint32_t *)r.sqn_r;
  }
  const unsigned blocks = (unsigned)((p.n + kQT - 1) / kQT);
  if (u8) {
    hipLaunchKernelGGL(exact_scan_kernel<PECANN_U8>, dim3(blocks, kParts), dim3(256), 0, st, sr, p.n,
                       r.metric, p.cand, p.thr);
  } else {
    hipLaunchKernelGGL(norm_max_kernel, dim3(1), dim3(1024), 0, st, sr.norms, p.n, p.nmax);
    hipLaunchKernelGGL(exact_scan_kernel<PECANN_F32>, dim3(blocks, kParts), dim3(256), 0, st, sr, p.n,
                       r.metric, p.cand, p.thr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Rounding bound.  Matrix-core measure |a|^2 + |b|^2 - 2 a.b against the
  // direct-difference float32 measure: each of the three float32 sums carries
  // at most gamma_d of its magnitudes, the direct sum gamma_d of D^2 <= 2
  // (|a|^2 + |b|^2), plus the final additions: E <= 4 (d + 4) u (|a|^2 + |b|^2),
  // u = 2^-24, and |b|^2 <= the largest row norm.  Cosine rows are unit:
  // E <= 4 (d + 4) u * 2.  uint8 rows: both measures are the same exact
  // integer sum of squared differences, rounded once to float32 the same way,
  // so E = 0.
  const float u = 5.9604645e-8f;
  const float dd = (float)r.d;
  float ce;
  if (u8) ce = 0.0f;
  else if (r.metric == PECANN_L2) ce = 4.0f * (dd + 4.0f) * u;
  else ce = 8.0f * (dd + 4.0f) * u;
  const int grid = (int)std::min<int64_t>((int64_t)p.n, 256 * 32);
  return launch_rerank(dt, S, p, ce, u8 ? 1 : 0, grid, st);
}

PECANN_CHECK_READER(exact)

}  // namespace pecann
