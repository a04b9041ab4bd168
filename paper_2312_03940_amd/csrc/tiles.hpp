// Dense 16 x 16 dot-product tiles between search rows on the matrix cores, and
// the measures (squared L2 or cosine distance) formed from them with the rows'
// stored norms and scales.  Used by RobustPrune and by the NN-descent joins.
#pragma once

#include "device_common.hpp"

namespace pecann {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// NT 16 x 16 tiles of dot products between search rows on the matrix cores,
// sharing their A rows.  Lane l contributes row (l % 16) of the A tile (arow)
// and of each B tile (brow[t]); at step s it loads 16-byte chunk (l / 16) + 4 s
// of each.  The result is the MFMA accumulator layout: register r of lane l
// holds A-row 4 (l / 16) + r against B-row l % 16.  U8 rows are shifted to
// signed (x - 128) so that the integer dot is exact (its bits are returned in
// the float lanes).  Missing rows (-1) contribute zeros.
__device__ __forceinline__ uint4 load_chunk(const uint8_t *base, int32_t row, int64_t stride, int q,
                                            bool in, bool u8) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (in && row >= 0) {
    v = *(const uint4 *)(base + (int64_t)row * stride + 16 * q);
    if (u8) { v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u; }
  }
  return v;
}

template <int DT>
__device__ __forceinline__ void mfma_chunk(uint4 a, uint4 b, v4f &accf, v4i &acci) {
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

// Steps whose loads go out before their products (one memory round trip per
// SG steps): the rule is four for float32 rows and two for the narrower
// formats, which keeps the prune kernels at three waves per SIMD (measured:
// 1M x 128 BF16 reverse prune 247 -> 197 ms per step, forward 87 -> 75;
// float32 rows were 1 % faster with four); the autotuner may choose per shape.
template <int DT>
constexpr int tile_steps_rule() { return DT == PECANN_F32 ? 4 : 2; }

template <int DT, int NT, int SG = tile_steps_rule<DT>()>
__device__ __forceinline__ void dot_tiles(const Rows &r, int32_t arow, const int32_t (&brow)[NT],
                                          v4f (&out)[NT]) {
  const int g = lane_id() >> 4;
  const int steps = (r.nch + 3) >> 2;
  constexpr bool u8 = DT == PECANN_U8;
  v4f accf[NT];
  v4i acci[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accf[t] = v4f{0.f, 0.f, 0.f, 0.f};
    acci[t] = v4i{0, 0, 0, 0};
  }
  for (int st0 = 0; st0 < steps; st0 += SG) {
    uint4 a[SG], b[SG][NT];
#pragma unroll
    for (int u = 0; u < SG; ++u) {
      const int q = g + 4 * (st0 + u);
      const bool in = st0 + u < steps && q < r.nch;
      a[u] = load_chunk(r.xs, arow, r.xs_stride, q, in, u8);
#pragma unroll
      for (int t = 0; t < NT; ++t) b[u][t] = load_chunk(r.xs, brow[t], r.xs_stride, q, in, u8);
    }
#pragma unroll
    for (int u = 0; u < SG; ++u) {
#pragma unroll
      for (int t = 0; t < NT; ++t) mfma_chunk<DT>(a[u], b[u][t], accf[t], acci[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (DT == PECANN_U8)
      out[t] = v4f{__int_as_float(acci[t][0]), __int_as_float(acci[t][1]), __int_as_float(acci[t][2]),
                   __int_as_float(acci[t][3])};
    else
      out[t] = accf[t];
  }
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
  // (sa * sb) first: the measure is then symmetric in its two rows, bit for bit
  const float dt = (DT == PECANN_FP8E4M3) ? dotv * (sa * sb) : dotv;
  if (metric == PECANN_L2) return fmaxf(0.f, __uint_as_float(na) + __uint_as_float(nb) - 2.0f * dt);
  return fmaxf(0.f, 1.0f - dt);
}

}  // namespace pecann
