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
// Gather-distance engine.  A wavefront is split into 64/G groups of G lanes;
// each group computes the distance from the register-resident query to one
// candidate row per pass, lane g of a group reading chunks g, g+G, g+2G, ...
// The query slice is held in float32 (at most 64 floats per lane).
//   L2:     measure = sum (q - x)^2          (squared distance)
//   cosine: measure = max(0, 1 - q.x)        (rows are pre-normalised)
// For FP8 rows the candidate values are x8 * scale_row.
// ---------------------------------------------------------------------------
template <int DT, int G>
struct Engine {
  static constexpr int EPC = RowFmt<DT>::EPC;
  static constexpr int CPL = 64 / EPC;  // chunks per lane (max)
  static constexpr int NPL = kWave / G; // candidates per pass
  float q[CPL * EPC];

  __device__ __forceinline__ int grp() const { return lane_id() / G; }
  __device__ __forceinline__ int gl() const { return lane_id() % G; }

  // Query from the float32 rows when present, else from the search rows.
  __device__ __forceinline__ void load_query(const Rows &r, int32_t row) {
    const int g = gl();
    if (r.xr) {
      const float *base = r.xr + (int64_t)row * r.xr_stride;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int c = g + G * t;
#pragma unroll
        for (int e = 0; e < EPC; e += 4) {
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          const int el = c * EPC + e;  // first element of this float4
          if (c < r.nch && el < r.nch_r * 4) v = *(const float4 *)(base + el);
          q[t * EPC + e + 0] = v.x; q[t * EPC + e + 1] = v.y;
          q[t * EPC + e + 2] = v.z; q[t * EPC + e + 3] = v.w;
        }
      }
    } else {
      const uint8_t *base = r.xs + (int64_t)row * r.xs_stride;
      const float s = (DT == PECANN_FP8E4M3) ? r.scale[row] : 1.0f;
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

  // Partial measure of this lane against search row `row` (row < 0: returns 0).
  __device__ __forceinline__ float partial(const Rows &r, int32_t row) const {
    const int g = gl();
    uint4 v[CPL];
    const uint8_t *base = r.xs + (int64_t)(row < 0 ? 0 : row) * r.xs_stride;
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int c = g + G * t;
      v[t] = make_uint4(0, 0, 0, 0);
      if (row >= 0 && c < r.nch) v[t] = *(const uint4 *)(base + 16 * c);
    }
    float acc = 0.f;
    if (r.metric == PECANN_L2) {
      const float s = (DT == PECANN_FP8E4M3 && row >= 0) ? r.scale[row] : 1.0f;
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
      float dot = 0.f;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        float x[EPC];
        unpack_chunk<DT>(v[t], x);
#pragma unroll
        for (int e = 0; e < EPC; ++e) dot = fmaf(q[t * EPC + e], x[e], dot);
      }
      if (DT == PECANN_FP8E4M3 && row >= 0) dot *= r.scale[row];
      acc = dot;
    }
    return acc;
  }

  // Full measure for the candidate of this lane's group; valid in every lane.
  __device__ __forceinline__ float measure(const Rows &r, int32_t row) const {
    float s = group_sum<G>(partial(r, row));
    if (r.metric != PECANN_L2) s = fmaxf(0.f, 1.0f - s);
    return s;
  }
};

// Float32 engine over the rerank rows (same lane layout: G lanes, 16-byte
// chunks, 64 floats per lane at most).
template <int G>
struct Engine32 {
  static constexpr int CPL = 16;
  static constexpr int NPL = kWave / G;
  float q[CPL * 4];
  __device__ __forceinline__ int gl() const { return lane_id() % G; }
  __device__ __forceinline__ void load_query(const Rows &r, int32_t row) {
    const float *base = r.xr + (int64_t)row * r.xr_stride;
    const int g = gl();
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int c = g + G * t;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (c < r.nch_r) v = *(const float4 *)(base + 4 * c);
      q[4 * t] = v.x; q[4 * t + 1] = v.y; q[4 * t + 2] = v.z; q[4 * t + 3] = v.w;
    }
  }
  __device__ __forceinline__ float measure(const Rows &r, int32_t row) const {
    const int g = gl();
    const float *base = r.xr + (int64_t)(row < 0 ? 0 : row) * r.xr_stride;
    float4 v[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int c = g + G * t;
      v[t] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row >= 0 && c < r.nch_r) v[t] = *(const float4 *)(base + 4 * c);
    }
    float acc = 0.f;
    if (r.metric == PECANN_L2) {
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        float a = q[4 * t] - v[t].x, b = q[4 * t + 1] - v[t].y;
        float c = q[4 * t + 2] - v[t].z, d = q[4 * t + 3] - v[t].w;
        acc = fmaf(a, a, acc); acc = fmaf(b, b, acc); acc = fmaf(c, c, acc); acc = fmaf(d, d, acc);
      }
      acc = group_sum<G>(acc);
    } else {
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        acc = fmaf(q[4 * t], v[t].x, acc); acc = fmaf(q[4 * t + 1], v[t].y, acc);
        acc = fmaf(q[4 * t + 2], v[t].z, acc); acc = fmaf(q[4 * t + 3], v[t].w, acc);
      }
      acc = fmaxf(0.f, 1.0f - group_sum<G>(acc));
    }
    return acc;
  }
};

// Engine over exact rows: the search rows themselves when they are float32 or
// uint8, else the float32 rerank rows.
template <int DT, int G>
using ExactEngine = typename std::conditional<(DT == PECANN_F32 || DT == PECANN_U8), Engine<DT, G>,
                                              Engine32<G>>::type;

}  // namespace pecann
