// Distances from a query to gathered candidate rows on the matrix cores, for
// BF16 and FP8-e4m3 search rows.  A beam search scores the new out-neighbours
// of each expanded point against one query: a matrix-vector product, which on
// the vector units costs a decode and a multiply-add per element.  Here the 16
// candidates of a group are the 16 columns of a B tile, each lane loading
// contiguous 16-byte chunks of its column's row straight from memory, and the
// query is the A tile's first rows: the matrix cores take the row bytes as they
// are stored (no decode) and accumulate in float32.
//
// The matrix cores multiply BF16 by BF16 and FP8 by FP8, so the float32 query
// is held as two parts of the row format, q ~ hi + lo with lo the rounded
// remainder q - hi (FP8: of q / s_q, s_q = max|q| / 448, the rows' own
// scaling).  The two parts are A rows 0 and 1; their products land in
// accumulator registers 0 and 1 of lanes 0-15 (lane c: candidate c) and are
// added.  hi + lo carries about twice the row format's mantissa bits, so the
// query's own rounding stays well below the candidate rows' and the ordering
// the beam sees is that of the stored rows.  Rows 2-15 of A are zero.
//
//   L2:     measure = |q|^2 + |x|^2 - 2 q.x, with |q|^2 the float32 query's
//           squared norm and |x|^2 the stored row's (both kept by the prepare
//           step); clamped at 0.
//   cosine: measure = max(0, 1 - q.x) (rows are normalised).
//
// A step multiplies K = 128 FP8 values (16x16x128 f8f6f4, unit block scales)
// or K = 32 BF16 values (16x16x32 bf16); lane group g = lane / 16 of a step
// covers the bytes [step * W + g * W / 4, + W / 4) of both the query part and
// the candidate row (W = 128 bytes FP8, 64 bytes BF16), so the dot product
// pairs equal elements whatever order the instruction sums them in.  Row bytes
// past the row's chunks are zeros on both sides.
//
// MXFP6 rows (OCP MX FP6 e2m3: 32 consecutive values share a power-of-two
// scale) are the B operand in their own format: 16x16x128 f8f6f4 with A FP8
// (the query parts) and B FP6.  For a 6-bit B the instruction reads lane group
// g's 32 packed values (24 bytes, value i in bits [6i, 6i + 6)) as K = 32 g ..
// 32 g + 31, and the lane's scale byte covers exactly those; an 8-bit A lane
// holds K = 16 g .. 16 g + 15 in its first 16 bytes and K = 64 + 16 g .. in its
// last 16.  So the row's block of 32 values (dims 128 s + 32 g ..) sits in one
// lane group with its own scale, and the query parts are stored permuted
// within each step: dim 128 s + 64 h + 16 g + j at byte 128 s + 32 g + 16 h + j.
#pragma once

#include <type_traits>

#include "tiles.hpp"

namespace pecann {

typedef int v8i __attribute__((ext_vector_type(8)));

template <int DT, int S>
struct MfmaScorer {
  static_assert(DT == PECANN_BF16 || DT == PECANN_FP8E4M3 || DT == PECANN_MXFP6,
                "matrix-core scoring is for BF16/FP8/MXFP6 rows");
  static constexpr bool MX6 = DT == PECANN_MXFP6;
  static constexpr bool FP8 = DT == PECANN_FP8E4M3 || MX6;  // FP8 query parts
  static constexpr int NC = FP8 ? 2 : 1;         // 16-byte chunks per lane per step
  static constexpr int CPS = 4 * NC;             // chunks per step (four lane groups)
  static constexpr int STEPS = (S + CPS - 1) / CPS;
  static constexpr int QB = STEPS * CPS * 16;    // bytes of one query part
  static constexpr int LDS_BYTES = 2 * QB + 32;  // two parts and a 32-byte zero block
  // steps whose row loads go out before their products: up to 16 chunks per
  // lane, so a 1024-byte FP8 row set (or a 512-byte BF16 one) of 16
  // candidates costs one memory round trip
  static constexpr int SB = (16 / NC) < STEPS ? 16 / NC : STEPS;

  uint8_t *qp;  // LDS, 16-byte aligned: part 0 (hi), part 1 (lo), 32 zero bytes
  float qs;     // FP8 / MXFP6: the query's scale s_q; BF16: 1
  float qn;     // squared norm of the float32 query (L2)

  // Splits the float32 query row into its two parts (LDS) and keeps its scale
  // and norm.  Every lane calls; the parts are visible after a wave_lds_sync.
  __device__ __forceinline__ void prepare(const Rows &r, int32_t qid) {
    const int l = lane_id();
    const float *q = r.xr + (int64_t)qid * r.xr_stride;
    const int lim = r.nch_r * 4;  // floats held by a float32 row (zero padded)
    constexpr int BPE = FP8 ? 1 : 2;
    constexpr int QE = QB / BPE;  // elements of a part
    float s = 1.0f, inv = 1.0f;
    if (FP8) {
      float mx = 0.f;
      for (int e = 4 * l; e < QE; e += 4 * kWave) {
        if (e < lim) {
          const float4 v = *(const float4 *)(q + e);
          mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
      inv = mx > 0.f ? 448.0f / mx : 1.0f;
      s = 1.0f / inv;
    }
    for (int e = 4 * l; e < QE; e += 4 * kWave) {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < lim) v = *(const float4 *)(q + e);
      const float f[4] = {v.x, v.y, v.z, v.w};
      if (FP8) {
        float h[4], o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = fminf(448.0f, fmaxf(-448.0f, f[i] * inv));
        int wh = __builtin_amdgcn_cvt_pk_fp8_f32(h[0], h[1], 0, false);
        wh = __builtin_amdgcn_cvt_pk_fp8_f32(h[2], h[3], wh, true);
        const auto b0 = __builtin_amdgcn_cvt_pk_f32_fp8(wh, false);
        const auto b1 = __builtin_amdgcn_cvt_pk_f32_fp8(wh, true);
        o[0] = h[0] - b0[0]; o[1] = h[1] - b0[1]; o[2] = h[2] - b1[0]; o[3] = h[3] - b1[1];
        int wl = __builtin_amdgcn_cvt_pk_fp8_f32(o[0], o[1], 0, false);
        wl = __builtin_amdgcn_cvt_pk_fp8_f32(o[2], o[3], wl, true);
        const int at = MX6 ? qperm(e) : e;
        *(int *)(qp + at) = wh;
        *(int *)(qp + QB + at) = wl;
      } else {
        uint32_t hb[4], lb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hb[i] = bf16_rne(f[i]);
          lb[i] = bf16_rne(f[i] - __uint_as_float(hb[i] << 16));
        }
        *(uint2 *)(qp + 2 * e) = make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16));
        *(uint2 *)(qp + QB + 2 * e) = make_uint2(lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16));
      }
    }
    if (l < 8) *(int *)(qp + 2 * QB + 4 * l) = 0;
    qs = s;
    qn = r.metric == PECANN_L2 ? r.sqn_r[qid] : 0.f;
  }

  // byte of query dim e in the MXFP6 A layout (e a multiple of 4: four
  // consecutive dims stay consecutive)
  __device__ __forceinline__ static int qperm(int e) {
    const int s = e >> 7, el = e & 127;
    return 128 * s + 32 * ((el >> 4) & 3) + 16 * (el >> 6) + (el & 15);
  }

  __device__ __forceinline__ static uint32_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
  }

  typedef typename std::conditional<FP8, v8i, v4i>::type Frag;
  // one step's B operand of a lane: its chunk(s) of the row and, for MXFP6,
  // the scale word of the step shifted so that the lane's block scale is byte 0
  struct Op {
    Frag b;
    int sc;
  };

  __device__ __forceinline__ static Op load(const Rows &r, const uint8_t *rb, int st, int g) {
    Op o;
    if constexpr (MX6) {
      const uint8_t *cb = rb + 24 * (4 * st + g);
      const uint2 d0 = *(const uint2 *)cb, d1 = *(const uint2 *)(cb + 8), d2 = *(const uint2 *)(cb + 16);
      o.b = v8i{(int)d0.x, (int)d0.y, (int)d1.x, (int)d1.y, (int)d2.x, (int)d2.y, 0, 0};
      o.sc = (int)(*(const uint32_t *)(rb + r.xg_soff + 4 * st) >> (8 * g));
    } else {
      o.b = *(const Frag *)(rb + 16 * (st * CPS + g * NC));
      o.sc = 0;
    }
    return o;
  }

  // acc += A x B for step st: the query fragment is read from the LDS right
  // before its product (rows 2-15 read the zero block)
  __device__ __forceinline__ static void product(v4f &acc, const uint8_t *qa, int qstep, int st, int g,
                                                 const Op &op) {
    const Frag a = *(const Frag *)(qa + 16 * qstep * (st * CPS + g * NC));
    const Frag &b = op.b;
    if constexpr (MX6) {
      // formats 0/2: e4m3 A with unit scale, e2m3 B with the lane's block scale
      acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 0, 2, 0, 127, 0, op.sc);
    } else if constexpr (FP8) {
      // formats 0/0: e4m3 for both operands; block scales 127 (2^0)
      acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b),
                                                    acc, 0, 0, 0);
    }
  }

  template <int B>
  __device__ __forceinline__ static void blocks(const Rows &r, v4f &acc, const uint8_t *qa, int qstep, int g,
                                                const uint8_t *rb, int &s0, int steps) {
#pragma unroll 1
    for (; s0 + B <= steps; s0 += B) {
      Op b[B];
#pragma unroll
      for (int u = 0; u < B; ++u) b[u] = load(r, rb, s0 + u, g);
#pragma unroll
      for (int u = 0; u < B; ++u) product(acc, qa, qstep, s0 + u, g, b[u]);
    }
    if constexpr (B > 1) blocks<B / 2>(r, acc, qa, qstep, g, rb, s0, steps);
  }

  // Keys (measure, id) of the candidates id_of(i), i in [0, c), into out[0, c)
  // (LDS); ids < 0 give kNoKey.  Visible to the wavefront after a wave_lds_sync.
  template <class IdFn>
  __device__ __forceinline__ void score(const Rows &r, int c, IdFn id_of, uint64_t *out) const {
    const int l = lane_id();
    const int col = l & 15, g = l >> 4;
    const int steps = r.nch / CPS;  // rows are padded to whole steps; at most STEPS
    // this lane's A row: query part 0 or 1, or (rows 2-15) a zero block that
    // every such lane reads at the same offsets
    const uint8_t *qa = col < 2 ? qp + col * QB : qp + 2 * QB;
    const int qstep = col < 2 ? 1 : 0;
    for (int base = 0; base < c; base += 16) {
      const int ci = base + col;
      const int32_t row = ci < c ? id_of(ci) : -1;
      // a missing candidate reads row 0 (its column's result is dropped)
      const uint8_t *rb = MX6 ? r.xg + (int64_t)(row < 0 ? 0 : row) * r.xg_stride
                              : r.xs + (int64_t)(row < 0 ? 0 : row) * r.xs_stride;
      v4f acc = {0.f, 0.f, 0.f, 0.f};
      // blocks of SB steps (the loop is kept rolled): the row loads of a block
      // go out together, then its products; the rest in blocks of SB / 2,
      // SB / 4, ... steps, so a row of any length costs few round trips.  The
      // rows end on a whole step (zero padded): no load needs a bound
      int s0 = 0;
      blocks<SB>(r, acc, qa, qstep, g, rb, s0, steps);
      if (l < 16 && ci < c) {
        uint64_t key = kNoKey;
        if (row >= 0) {
          float dot = acc[0] + acc[1];
          if constexpr (MX6) dot *= qs;  // the block scales are applied by the instruction
          else if (FP8) dot *= qs * fp8_row_scale(r, row);
          const uint32_t xn = MX6 ? r.sqn_g[row] : r.sqn[row];
          const float m = r.metric == PECANN_L2 ? fmaxf(0.f, qn + __uint_as_float(xn) - 2.0f * dot)
                                                : fmaxf(0.f, 1.0f - dot);
          key = make_key(m, row);
        }
        out[ci] = key;
      }
    }
  }
};

}  // namespace pecann
