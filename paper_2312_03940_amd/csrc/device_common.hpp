// Device-side building blocks shared by the gfx950 kernels: 64-bit (distance,
// index) keys, wavefront primitives, row formats and the gather-distance engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pecann.h"
#include "kernels.hpp"

namespace pecann {

constexpr int kWave = 64;
constexpr uint64_t kNoKey = ~0ull;

// Checked builds (compiled with -DPECANN_CHECKED): kernels test invariants of
// their inputs and state and record a broken one as a bit of a device word of
// their translation unit; after each entry point the host synchronises, reads
// and clears the words and fails the call with PECANN_ECHECK.  Other builds
// compile the checks away.
enum CheckBit : uint32_t {
  CK_ITEM = 1u << 0,       // a work item or query outside the point set
  CK_NEIGHBOUR = 1u << 1,  // an adjacency entry or degree outside its range
  CK_BEAM = 1u << 2,       // a beam longer than its capacity or out of order
  CK_INSTANCE = 1u << 3,   // a point outside the instance found for it
  CK_PRUNE = 1u << 4,      // a prune's candidate count or output beyond its bound
  CK_REVERSE = 1u << 5,    // a reverse edge written outside its batch's segments
  CK_CHUNK = 1u << 6,      // a scan chunk outside its instance
  CK_LABEL = 1u << 7,      // a cluster label or dependent outside the point set
};
#ifdef PECANN_CHECKED
static __device__ uint32_t g_check_word;
#define PECANN_CHECK(cond, bit)                                               \
  do {                                                                        \
    if (!(cond)) atomicOr(&::pecann::g_check_word, (uint32_t)(bit));           \
  } while (0)
#define PECANN_CHECK_READER(name)                                             \
  uint32_t check_take_##name() {                                              \
    uint32_t v = 0, z = 0;                                                    \
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_check_word), 4, 0, hipMemcpyDeviceToHost) != hipSuccess) \
      return 0x80000000u;                                                     \
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_check_word), &z, 4, 0, hipMemcpyHostToDevice) != hipSuccess) \
      return 0x80000000u;                                                     \
    return v;                                                                 \
  }
#else
#define PECANN_CHECK(cond, bit) \
  do {                          \
  } while (0)
#define PECANN_CHECK_READER(name)
#endif

// ---------------------------------------------------------------------------
// Keys.  A candidate is (distance measure, index) packed as
// float_bits(measure) << 32 | index.  The measure is never negative (squared
// L2, or a clamped cosine distance), so unsigned order of the packed key is the
// (distance, index) order used everywhere.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t make_key(float m, int32_t id) {
  return ((uint64_t)__float_as_uint(m) << 32) | (uint32_t)id;
}
__device__ __forceinline__ float key_measure(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ int32_t key_id(uint64_t k) { return (int32_t)(uint32_t)k; }

// Reported distance from the measure: L2 keys hold D^2, cosine keys hold D.
__device__ __forceinline__ float measure_to_dist(float m, int metric) {
  return metric == PECANN_L2 ? sqrtf(m) : m;
}

// ---------------------------------------------------------------------------
// Wavefront helpers (one wavefront = 64 lanes on CDNA).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// number of set bits of mask strictly below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl_xor((int)lo, m);
  hi = (uint32_t)__shfl_xor((int)hi, m);
  return ((uint64_t)hi << 32) | lo;
}
// value of v in lane `src` (src wave-uniform)
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl((int)lo, src);
  hi = (uint32_t)__shfl((int)hi, src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = shfl_xor_u64(v, m);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Sum over aligned groups of G lanes; every lane of a group gets the total.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Bitonic sort of one 64-bit key per lane across the wavefront (ascending by
// lane index).
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j >= 1; j >>= 1) {
      uint64_t o = shfl_xor_u64(v, j);
      bool up = ((l & k) == 0);
      bool lower = ((l & j) == 0);
      // lower lane keeps min when ascending
      bool take_min = (lower == up);
      uint64_t mn = o < v ? o : v, mx = o < v ? v : o;
      v = take_min ? mn : mx;
    }
  }
  return v;
}

// Block-level barrier for one-wavefront blocks: orders the wave's LDS traffic.
__device__ __forceinline__ void wave_lds_sync() { __syncthreads(); }

// Lane 0 takes the next item of a device work queue; all lanes get it.
__device__ __forceinline__ int next_item(int32_t *head) {
  int v = 0;
  if (lane_id() == 0) v = atomicAdd(head, 1);
  return __shfl(v, 0);
}

// Instance of point i: the t with off[t] <= i < off[t+1] (0 for a single
// instance or no table).
__device__ __forceinline__ int find_instance(const InstTable &it, int64_t i) {
  if (it.count <= 1) return 0;
  int lo = 0, hi = it.count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (it.off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Row formats.  Rows are read in 16-byte chunks; EPC = elements per chunk.
// ---------------------------------------------------------------------------
template <int DT> struct RowFmt;
template <> struct RowFmt<PECANN_F32> { static constexpr int EPC = 4; static constexpr int BYTES = 4; };
template <> struct RowFmt<PECANN_U8> { static constexpr int EPC = 16; static constexpr int BYTES = 1; };
template <> struct RowFmt<PECANN_BF16> { static constexpr int EPC = 8; static constexpr int BYTES = 2; };
template <> struct RowFmt<PECANN_FP8E4M3> { static constexpr int EPC = 16; static constexpr int BYTES = 1; };

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

template <int DT>
__device__ __forceinline__ void unpack_chunk(const uint4 &c, float *o);

template <>
__device__ __forceinline__ void unpack_chunk<PECANN_F32>(const uint4 &c, float *o) {
  o[0] = __uint_as_float(c.x); o[1] = __uint_as_float(c.y);
  o[2] = __uint_as_float(c.z); o[3] = __uint_as_float(c.w);
}
template <>
__device__ __forceinline__ void unpack_chunk<PECANN_U8>(const uint4 &c, float *o) {
  const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[4 * i + 0] = (float)(w[i] & 0xffu);
    o[4 * i + 1] = (float)((w[i] >> 8) & 0xffu);
    o[4 * i + 2] = (float)((w[i] >> 16) & 0xffu);
    o[4 * i + 3] = (float)(w[i] >> 24);
  }
}
template <>
__device__ __forceinline__ void unpack_chunk<PECANN_BF16>(const uint4 &c, float *o) {
  const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) { o[2 * i] = bf16_lo(w[i]); o[2 * i + 1] = bf16_hi(w[i]); }
}
template <>
__device__ __forceinline__ void unpack_chunk<PECANN_FP8E4M3>(const uint4 &c, float *o) {
  const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    auto a = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
    auto b = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
    o[4 * i + 0] = a[0]; o[4 * i + 1] = a[1];
    o[4 * i + 2] = b[0]; o[4 * i + 3] = b[1];
  }
}

// Where the rows live (device pointers into the prepared buffer): see RowsDesc.
using Rows = RowsDesc;

// ---------------------------------------------------------------------------
// Gather-distance engine.  The shape S (a power of two in [4, 1024], at least
// the row's number of 16-byte chunks) is split into G lanes per candidate and
// CPL = S / G chunks per lane: as many chunks per lane as a 32-float query
// slice allows (more only when S > 64 * that), lane g of a group holding chunks
// g, g + G, ...  A wavefront scores NPL = 64 / G candidates per pass and issues
// the row loads of U passes (at most LCAP chunks per lane) before reducing any;
// the U partial sums of a group are then reduced together by recursive halving
// (each lane ends with the total of one candidate), which costs about one lane
// exchange per candidate instead of log2(G).
//   L2:     measure = sum (q - x)^2          (squared distance)
//   cosine: measure = max(0, 1 - q.x)        (rows are pre-normalised)
// FP8 candidate values are x8 * scale_row; U8 rows are summed in int32, so
// their measures are exact integers (rounded once to float).  XR = true makes
// a float32 engine over the rerank rows instead of the search rows.
// ---------------------------------------------------------------------------
// Scale of an FP8 search row.  Cosine rows are unit vectors stored as x * 448
// (e4m3's largest normal) with one scale for all rows: a floating-point code
// keeps its relative precision under any scale that avoids overflow, and the
// scorers then read no per-candidate scale (a 4-byte gather that costs a
// 64-byte line per candidate).  L2 rows keep max|x| / 448 per row.
constexpr float kFp8UnitInv = 448.0f;
__device__ __forceinline__ float fp8_row_scale(const Rows &r, int32_t row) {
  return r.metric == PECANN_COSINE ? 1.0f / kFp8UnitInv : r.scale[row];
}

constexpr int max_shape(int dt) { return dt == PECANN_F32 ? 1024 : dt == PECANN_BF16 ? 512 : 256; }

// Launch-time dispatch over (row format, shape).  FN<DT, S> is a function
// template that returns hipErrorInvalidValue for S > max_shape(DT) (under
// `if constexpr`, so that no kernel is instantiated for those shapes).
#define PECANN_SHAPES(FN, DT, S, ...)                                            \
  switch (S) {                                                                   \
    case 4: return FN<DT, 4>(__VA_ARGS__);                                       \
    case 8: return FN<DT, 8>(__VA_ARGS__);                                       \
    case 16: return FN<DT, 16>(__VA_ARGS__);                                     \
    case 32: return FN<DT, 32>(__VA_ARGS__);                                     \
    case 64: return FN<DT, 64>(__VA_ARGS__);                                     \
    case 128: return FN<DT, 128>(__VA_ARGS__);                                   \
    case 256: return FN<DT, 256>(__VA_ARGS__);                                   \
    case 512: return FN<DT, 512>(__VA_ARGS__);                                   \
    case 1024: return FN<DT, 1024>(__VA_ARGS__);                                 \
    default: return hipErrorInvalidValue;                                        \
  }
#define PECANN_DISPATCH_SHAPE(FN, dt, S, ...)                                    \
  switch (dt) {                                                                  \
    case PECANN_F32: PECANN_SHAPES(FN, PECANN_F32, S, __VA_ARGS__)               \
    case PECANN_U8: PECANN_SHAPES(FN, PECANN_U8, S, __VA_ARGS__)                 \
    case PECANN_BF16: PECANN_SHAPES(FN, PECANN_BF16, S, __VA_ARGS__)             \
    case PECANN_FP8E4M3: PECANN_SHAPES(FN, PECANN_FP8E4M3, S, __VA_ARGS__)       \
    default: return hipErrorInvalidValue;                                        \
  }

// Sums of U values over aligned groups of G lanes (U <= G, both powers of
// two), scattered: lane l ends with the total of value (l % G) / (G / U) of its
// group.  INT: the values are int32 bit patterns, added as integers.
template <int G, int U, bool INT>
__device__ __forceinline__ float reduce_scatter(float (&v)[U]) {
  const int l = lane_id();
#pragma unroll
  for (int k = 1; k < U; k <<= 1) {
    const int m = G / (2 * k);
    const int h = U / (2 * k);  // values kept after this step
    const bool hi = (l & m) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      float lo_v = v[i], hi_v = v[h + i];
      // pin both values in registers first: a select between two array loads
      // would otherwise become a load from a selected address (private memory)
      asm("" : "+v"(lo_v), "+v"(hi_v));
      const float send = hi ? lo_v : hi_v;
      const float keep = hi ? hi_v : lo_v;
      const float got = __shfl_xor(send, m);
      v[i] = INT ? __int_as_float(__float_as_int(keep) + __float_as_int(got)) : keep + got;
    }
  }
  float r = v[0];
#pragma unroll
  for (int m = G / (2 * U); m >= 1; m >>= 1) {
    const float got = __shfl_xor(r, m);
    r = INT ? __int_as_float(__float_as_int(r) + __float_as_int(got)) : r + got;
  }
  return r;
}

template <int DT, int S, bool XR = false, int LC = 0>
struct Engine {
  static_assert(S >= 4 && S <= 1024 && (S & (S - 1)) == 0, "shape must be a power of two in [4, 1024]");
  static_assert(!XR || DT == PECANN_F32, "the rerank rows are float32");
  static constexpr int EPC = RowFmt<DT>::EPC;
  // query budget: 32 floats per lane (16 for the rerank rows, whose engine is
  // live next to the search engine's state)
  static constexpr int QCAP = XR ? 16 : 32;
  static constexpr int CPL_Q = (QCAP / EPC) < S ? QCAP / EPC : S;
  static constexpr int CPL = (S / kWave) > CPL_Q ? S / kWave : CPL_Q;
  static constexpr int G = S / CPL;
  static constexpr int NPL = kWave / G;
  // chunks per lane in flight: 16 for float32 search rows, 8 for the narrower
  // formats and the rerank rows (whose kernels need more registers elsewhere;
  // measured best on MI355X); LC > 0 overrides it
  static constexpr int LCAP = LC > 0 ? LC : ((DT == PECANN_F32 && !XR) ? 16 : 8);
  static constexpr int U = (LCAP / CPL) < 1 ? 1 : ((LCAP / CPL) < G ? LCAP / CPL : G);
  static constexpr bool INT = DT == PECANN_U8 && !XR;
  float q[CPL * EPC];

  __device__ __forceinline__ static int gl() { return lane_id() % G; }
  __device__ __forceinline__ static int chunks(const Rows &r) { return XR ? r.nch_r : r.nch; }
  __device__ __forceinline__ static const uint8_t *row_ptr(const Rows &r, int32_t row) {
    return XR ? (const uint8_t *)(r.xr + (int64_t)row * r.xr_stride) : r.xs + (int64_t)row * r.xs_stride;
  }
  // Index (in [0, U)) of the candidate whose total this lane holds after a
  // measure_batch, and whether it is the lane that reports it.
  __device__ __forceinline__ static int owned() { return gl() / (G / U); }
  __device__ __forceinline__ static bool reporter() { return gl() % (G / U) == 0; }

  // Query from the float32 rows when present, else from the search rows.
  __device__ __forceinline__ void load_query(const Rows &r, int32_t row) {
    const int g = gl();
    if (XR || r.xr) {
      const float *base = r.xr + (int64_t)row * r.xr_stride;
      const int lim = r.nch_r * 4;  // floats held by a rerank row
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int c = g + G * t;
#pragma unroll
        for (int e = 0; e < EPC; e += 4) {
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          const int el = c * EPC + e;  // first element of this float4
          if (el < lim) v = *(const float4 *)(base + el);
          q[t * EPC + e + 0] = v.x; q[t * EPC + e + 1] = v.y;
          q[t * EPC + e + 2] = v.z; q[t * EPC + e + 3] = v.w;
        }
      }
    } else {
      const uint8_t *base = r.xs + (int64_t)row * r.xs_stride;
      const float s = (DT == PECANN_FP8E4M3) ? fp8_row_scale(r, row) : 1.0f;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int c = g + G * t;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (c < r.nch) v = *(const uint4 *)(base + 16 * c);
        unpack_chunk<DT>(v, q + t * EPC);
        if (DT == PECANN_FP8E4M3) {
#pragma unroll
          for (int e = 0; e < EPC; ++e) q[t * EPC + e] *= s;
        }
      }
    }
  }

  // This lane's partial measure against the chunks v of one candidate (scale s);
  // int32 bits for U8 rows.
  __device__ __forceinline__ float partial(const uint4 (&v)[CPL], float s, int metric) const {
    if (INT) {
      int acc = 0;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        float x[EPC];
        unpack_chunk<DT>(v[t], x);
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
          const int df = (int)q[t * EPC + e] - (int)x[e];
          acc += df * df;
        }
      }
      return __int_as_float(acc);
    }
    float acc = 0.f;
    if (metric == PECANN_L2) {
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        float x[EPC];
        unpack_chunk<DT>(v[t], x);
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
          const float xv = (DT == PECANN_FP8E4M3) ? x[e] * s : x[e];
          const float df = q[t * EPC + e] - xv;
          acc = fmaf(df, df, acc);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        float x[EPC];
        unpack_chunk<DT>(v[t], x);
#pragma unroll
        for (int e = 0; e < EPC; ++e) acc = fmaf(q[t * EPC + e], x[e], acc);
      }
      if (DT == PECANN_FP8E4M3) acc *= s;
    }
    return acc;
  }

  // Measure from a group total.
  __device__ __forceinline__ static float finish(float tot, int metric) {
    if (INT) return (float)__float_as_int(tot);
    return metric == PECANN_L2 ? tot : fmaxf(0.f, 1.0f - tot);
  }

  // Measures of the U candidates row[0..U) of this lane's group; the lane gets
  // the measure of row[owned()] (unspecified when that row is < 0).
  __device__ __forceinline__ float measure_batch(const Rows &r, const int32_t (&row)[U]) const {
    const int g = gl();
    const int nch = chunks(r);
    uint4 v[U][CPL];
    float sc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint8_t *base = row_ptr(r, row[u] < 0 ? 0 : row[u]);
      sc[u] = (DT == PECANN_FP8E4M3 && !XR && row[u] >= 0) ? fp8_row_scale(r, row[u]) : 1.0f;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int c = g + G * t;
        v[u][t] = make_uint4(0, 0, 0, 0);
        if (row[u] >= 0 && c < nch) v[u][t] = *(const uint4 *)(base + 16 * c);
      }
    }
    float part[U];
#pragma unroll
    for (int u = 0; u < U; ++u) part[u] = partial(v[u], sc[u], r.metric);
    return finish(reduce_scatter<G, U, INT>(part), r.metric);
  }

  // Measure of one candidate per lane group, valid in every lane of the group.
  __device__ __forceinline__ float measure(const Rows &r, int32_t row) const {
    const int g = gl();
    const int nch = chunks(r);
    const uint8_t *base = row_ptr(r, row < 0 ? 0 : row);
    uint4 v[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int c = g + G * t;
      v[t] = make_uint4(0, 0, 0, 0);
      if (row >= 0 && c < nch) v[t] = *(const uint4 *)(base + 16 * c);
    }
    const float s = (DT == PECANN_FP8E4M3 && !XR && row >= 0) ? fp8_row_scale(r, row) : 1.0f;
    float part[1] = {partial(v, s, r.metric)};
    return finish(reduce_scatter<G, 1, INT>(part), r.metric);
  }
};

// Float32 engine over the rerank rows.
template <int S>
using Engine32 = Engine<PECANN_F32, S, true>;

// Shape of the rerank-row engine that goes with search-row shape S: a
// BF16 (FP8) chunk holds 8 (16) values, a float32 chunk 4.
template <int DT, int S>
struct RerankShape {
  static constexpr int v = (S * RowFmt<DT>::EPC / 4) < 4 ? 4 : (S * RowFmt<DT>::EPC / 4);
};

// Engine over exact rows: the search rows themselves when they are float32 or
// uint8, else the float32 rerank rows.
template <int DT, int S>
using ExactEngine = typename std::conditional<(DT == PECANN_F32 || DT == PECANN_U8), Engine<DT, S>,
                                              Engine32<RerankShape<DT, S>::v>>::type;

// Keys (measure, id) of the candidates id_of(i), i in [0, c), into out[0, c)
// (LDS); ids < 0 give kNoKey.  Visible to the wavefront after a wave_lds_sync.
template <class E, class IdFn>
__device__ __forceinline__ void score_keys(const E &eng, const Rows &r, int c, IdFn id_of,
                                           uint64_t *out) {
  constexpr int NPL = E::NPL, U = E::U, G = E::G;
  const int grp = lane_id() / G;
  const int mine = E::owned();
  const bool rep = E::reporter();
  for (int base = 0; base < c; base += NPL * U) {
    int32_t row[U];
    int32_t myrow = -1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ci = base + u * NPL + grp;
      row[u] = ci < c ? id_of(ci) : -1;
      if (u == mine) myrow = row[u];
    }
    const float m = eng.measure_batch(r, row);
    const int ci = base + mine * NPL + grp;
    if (rep && ci < c) out[ci] = myrow >= 0 ? make_key(m, myrow) : kNoKey;
  }
}

}  // namespace pecann
