// Non-templated kernels of the hot path:
//   K0  prepare       -- search/rerank copies of the point set (BF16, FP8, U8, F32)
//   K9a-c rev_*       -- group a batch's reverse edges by target (count, allocate, scatter)
//   K5  dep_in_knn    -- DPBruteForce over each point's kNN list (Alg. 3, first loop)
//   K7' bf_dep_finalize, min_key, fills
//   K10 select_centers (radix select of the n_c largest rho*delta) + noise mask
//   K11 labels        -- roots of the dependent forest by pointer jumping
#include <hip/hip_runtime.h>

#include <algorithm>

#include "claim.hpp"
#include "device_common.hpp"

namespace pecann {

// ---------------------------------------------------------------------------
// K0: one wavefront per row.  Reads the caller's row (F32 or U8), divides by
// its norm for the cosine metric, writes the float32 rerank row (if any) and
// the search row: F32 copy, U8 copy, BF16 round-to-nearest-even, or FP8 e4m3
// of x / scale with scale = max|x| / 448 (OCP e4m3 largest normal) for L2 and
// 1 / 448 for the (unit) cosine rows.
// Padding up to the 16-byte row stride is written as zeros.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// MXFP6 element e2m3 (sign, 2 exponent bits with bias 1, 3 mantissa bits):
// value of a 6-bit code
__device__ __forceinline__ float e2m3_value(int c) {
  const int e = (c >> 3) & 3, m = c & 7;
  const float v = e == 0 ? 0.125f * (float)m : ldexpf(1.0f + 0.125f * (float)m, e - 1);
  return (c & 32) ? -v : v;
}

// MXFP6 copy of one row (wavefront-wide; v[t] holds dim 64 t + lane, zero past
// d): blocks of 32 dims share the power-of-two scale 2^E with E the smallest
// integer that puts the block's largest magnitude at or below 7.5 (e2m3's
// largest value); each value x / 2^E is rounded to the nearest e2m3 value,
// ties to even.  Block b = 4 s + g of step s: 24 bytes of codes at 24 b (code
// i in bits [6i, 6i + 6)), its scale E + 127 in byte b of the scale words.
// Returns the squared norm of the dequantised row.
template <int T>
__device__ __forceinline__ float write_mxfp6(const float (&v)[T], const RowsDesc &r, uint8_t *og) {
  const int l = lane_id(), h = l >> 5, j = l & 31;
  const int nblk = 4 * (r.xg_soff / 96);
  float ng = 0.f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (2 * t >= nblk) break;  // wave-uniform: nblk is even
    const int blk = 2 * t + h;  // dims 64 t + 32 h .. + 31, one per lane of the half
    const float x = v[t];
    float amax = fabsf(x);
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) amax = fmaxf(amax, __shfl_xor(amax, m));
    int E = -127;
    if (amax > 0.f) {
      int k;
      const float fr = frexpf(amax, &k);  // amax = fr 2^k, fr in [0.5, 1)
      E = (k - 3) + (fr > 0.9375f ? 1 : 0);  // 7.5 2^(k-3) = 0.9375 2^k
      E = E < -127 ? -127 : E > 127 ? 127 : E;
    }
    const float y = ldexpf(x, -E);
    const float a = fabsf(y);
    int code;
    if (a < 1.0f) {
      code = (int)rintf(a * 8.0f);  // 8 is the code of 1.0
    } else {
      int k2;
      frexpf(a, &k2);
      const int kk = k2 - 1;  // floor(log2 a), 0..2
      code = 8 * kk + (int)rintf(ldexpf(a, 3 - kk));
    }
    if (y < 0.f) code |= 32;
    const float dq = ldexpf(e2m3_value(code), E);
    ng = fmaf(dq, dq, ng);
    // lane j < 6 forms word j of the block's 24 bytes from the (at most six)
    // codes that touch it, i0 = floor(32 j / 6) onwards
    const int i0 = (16 * (j < 6 ? j : 0)) / 3;
    uint32_t w = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int i = i0 + q < 31 ? i0 + q : 31;
      const uint32_t c = (uint32_t)__shfl(code, 32 * h + i);
      const int sh = 6 * (i0 + q) - 32 * j;
      if (i0 + q < 32 && sh > -6 && sh < 32) w |= sh >= 0 ? c << sh : c >> (-sh);
    }
    if (j < 6) *(uint32_t *)(og + 24 * blk + 4 * j) = w;
    if (j == 0) og[r.xg_soff + blk] = (uint8_t)(E + 127);
  }
  for (int b = r.xg_soff + nblk + l; b < r.xg_stride; b += kWave) og[b] = 0;
  return ng;
}

// T = values per lane (the row's padded length / 64, rounded up to a power of
// two); every loop over them is unrolled so the row stays in registers.
template <int T>
__global__ __launch_bounds__(256) void prepare_kernel(const void *x, int32_t x_dtype, int64_t x_stride,
                                                      int64_t n, int32_t d, int32_t metric,
                                                      int32_t sdt, RowsDesc r, uint8_t *xs,
                                                      float *xr, float *scale, uint32_t *sqn,
                                                      float *sqn_r, uint8_t *xg, uint32_t *sqn_g) {
  const int l = lane_id();
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= n) return;
  constexpr int kMaxPerLane = T;
  float v[kMaxPerLane];
  float ss = 0.f, mx = 0.f;
#pragma unroll
  for (int t = 0; t < kMaxPerLane; ++t) {
    const int e = l + 64 * t;
    float f = 0.f;
    if (e < d) {
      if (x_dtype == PECANN_U8) f = (float)((const uint8_t *)x)[row * x_stride + e];
      else f = ((const float *)x)[row * x_stride + e];
    }
    v[t] = f;
    ss = fmaf(f, f, ss);
  }
  if (metric == PECANN_COSINE) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m);
    const float inv = ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
#pragma unroll
    for (int t = 0; t < kMaxPerLane; ++t) v[t] *= inv;
  }
  if (xr) {
    float *o = xr + row * r.xr_stride;
    float nr = 0.f;
#pragma unroll
    for (int t = 0; t < kMaxPerLane; ++t) {
      const int e = l + 64 * t;
      if (e < r.xr_stride) {
        const float f = e < d ? v[t] : 0.f;
        o[e] = f;
        nr = fmaf(f, f, nr);
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) nr += __shfl_xor(nr, m);
    if (l == 0) sqn_r[row] = nr;
  }
  uint8_t *o = xs + row * r.xs_stride;
  float nf = 0.f;  // squared norm of the stored values
  int ni = 0;      // U8: sum of (x - 128)^2 over the padded row
  if (sdt == PECANN_F32) {
    float *of = (float *)o;
    const int64_t cap = r.xs_stride / 4;
#pragma unroll
    for (int t = 0; t < kMaxPerLane; ++t) {
      const int e = l + 64 * t;
      if (e < cap) {
        const float f = e < d ? v[t] : 0.f;
        of[e] = f;
        nf = fmaf(f, f, nf);
      }
    }
  } else if (sdt == PECANN_U8) {
#pragma unroll
    for (int t = 0; t < kMaxPerLane; ++t) {
      const int e = l + 64 * t;
      if (e < r.xs_stride) {
        const int b = e < d ? (int)v[t] : 0;
        o[e] = (uint8_t)b;
        ni += (b - 128) * (b - 128);
      }
    }
  } else if (sdt == PECANN_BF16) {
    uint16_t *ob = (uint16_t *)o;
    const int64_t cap = r.xs_stride / 2;
#pragma unroll
    for (int t = 0; t < kMaxPerLane; ++t) {
      const int e = l + 64 * t;
      if (e < cap) {
        const uint16_t h = e < d ? f32_to_bf16_rne(v[t]) : (uint16_t)0;
        ob[e] = h;
        const float f = __uint_as_float((uint32_t)h << 16);
        nf = fmaf(f, f, nf);
      }
    }
  } else {  // FP8 e4m3
#pragma unroll
    for (int t = 0; t < kMaxPerLane; ++t) mx = fmaxf(mx, fabsf(v[t]));
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
    const bool unit = metric == PECANN_COSINE;  // one scale for all unit rows
    const float inv = unit ? kFp8UnitInv : mx > 0.f ? 448.0f / mx : 1.0f;
    const float sc = unit ? 1.0f / kFp8UnitInv : 1.0f / inv;
    if (l == 0) scale[row] = sc;
#pragma unroll
    for (int t = 0; t < kMaxPerLane; ++t) {
      const int e = l + 64 * t;
      if (e < r.xs_stride) {
        const float f = e < d ? fminf(448.0f, fmaxf(-448.0f, v[t] * inv)) : 0.f;
        const int w = __builtin_amdgcn_cvt_pk_fp8_f32(f, 0.f, 0, false);
        o[e] = (uint8_t)(w & 0xff);
        const float back = __builtin_amdgcn_cvt_pk_f32_fp8(w, false)[0] * sc;
        nf = fmaf(back, back, nf);
      }
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    nf += __shfl_xor(nf, m);
    ni += __shfl_xor(ni, m);
  }
  if (l == 0) sqn[row] = sdt == PECANN_U8 ? (uint32_t)ni : __float_as_uint(nf);
  if (xg) {
    float ng = write_mxfp6<T>(v, r, xg + row * r.xg_stride);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ng += __shfl_xor(ng, m);
    if (l == 0) sqn_g[row] = __float_as_uint(ng);
  }
}

hipError_t launch_prepare(const void *x, int32_t x_dtype, int64_t x_stride, int64_t n, int32_t d,
                          int32_t metric, int32_t sdt, const RowsDesc &rows, uint8_t *xs,
                          float *xr, float *scale, uint32_t *sqn, float *sqn_r, uint8_t *xg,
                          uint32_t *sqn_g, hipStream_t s) {
  const int64_t blocks = (n + 3) / 4;
  // values per lane: the longest of the caller's row and the two stored rows
  const int64_t elems = std::max<int64_t>({(int64_t)d, rows.xr_stride, sdt == PECANN_F32 ? rows.xs_stride / 4
                                           : sdt == PECANN_BF16 ? rows.xs_stride / 2 : rows.xs_stride});
  const int64_t per = (elems + 63) / 64;
  const dim3 g((unsigned)blocks), b(256);
#define PECANN_PREP(T)                                                                             \
  hipLaunchKernelGGL(prepare_kernel<T>, g, b, 0, s, x, x_dtype, x_stride, n, d, metric, sdt, rows, xs, \
                     xr, scale, sqn, sqn_r, xg, sqn_g)
  if (per <= 2) PECANN_PREP(2);
  else if (per <= 4) PECANN_PREP(4);
  else if (per <= 8) PECANN_PREP(8);
  else if (per <= 16) PECANN_PREP(16);
  else if (per <= 32) PECANN_PREP(32);
  else if (per <= 64) PECANN_PREP(64);
  else return hipErrorInvalidValue;
#undef PECANN_PREP
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fills (graph-capture safe: kernels, not memset nodes).
// ---------------------------------------------------------------------------
__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_u64_kernel(uint64_t *p, uint64_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void identity_kernel(int32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}
static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_identity_perm(int32_t *p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(identity_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Read-bandwidth probe (a measurement aid, not a step of the method): every
// thread streams 16-byte loads over the buffer, four in flight, and folds them
// into an XOR that is stored only if it equals a value the caller picks, so
// the loads are kept and nothing but the reads reaches memory.
// ---------------------------------------------------------------------------
// Read of a buffer, eight 16-byte loads in flight per thread, grid-strided.
// A single pass (a buffer far beyond the caches) uses non-temporal loads, the
// best of the variants measured on MI355X for a 4 GiB buffer (6.5 TB/s, against
// 5.6 TB/s with four plain loads per thread); repeated passes over a small
// buffer keep plain loads, so that the data stays in the caches.
template <bool NT>
__global__ __launch_bounds__(256) void read_probe_kernel(const uint4 *p, int64_t n16, int32_t passes,
                                                         uint32_t key, uint32_t *sink) {
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  constexpr int U = 8;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const u4v *q = (const u4v *)p;
  uint32_t acc = 0;
  for (int32_t r = 0; r < passes; ++r) {
    // pass r: block b reads the slice block b + r read in pass 0, so that on
    // repeated passes no XCD re-reads data its own L2 took in the pass before
    // (blocks are dealt to the XCDs in turn): the repeats measure the
    // Infinity Cache, not the L2.  Every trip keeps U loads in flight, the
    // last one with the entries past the end masked off.
    const int64_t b = ((int64_t)blockIdx.x + r) % gridDim.x;
    for (int64_t i = b * blockDim.x + threadIdx.x; i < n16; i += U * stride) {
      u4v v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = i + u * stride;
        v[u] = j < n16 ? (NT ? __builtin_nontemporal_load(q + j) : q[j]) : u4v{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    acc = acc * 2654435761u + (uint32_t)r;
  }
  if (acc == key) atomicOr(sink, 1u);
}
hipError_t launch_read_probe(const void *buf, int64_t bytes, int32_t passes, uint32_t key,
                             uint32_t *sink, int grid, hipStream_t s) {
  if (passes == 1)
    hipLaunchKernelGGL(read_probe_kernel<true>, dim3(grid), dim3(256), 0, s, (const uint4 *)buf, bytes / 16,
                       passes, key, sink);
  else
    hipLaunchKernelGGL(read_probe_kernel<false>, dim3(grid), dim3(256), 0, s, (const uint4 *)buf, bytes / 16,
                       passes, key, sink);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K9a-c: reverse edges of a batch grouped by target.
//   count:   rcnt[q] += 1 per edge (p -> q); the first edge to reach q puts q in
//            the target list; each edge keeps its arrival ticket;
//   alloc:   each target reserves a segment of rcnt[q] slots;
//   scatter: source p goes to slot (segment of q) + ticket.
// Arrival order is not deterministic; the merge sorts each segment by index.
// ---------------------------------------------------------------------------
// Wave-wide inclusive prefix sum.

// Counting pass: each edge takes a ticket in its target's count; a target seen
// for the first time joins the target list (slots handed out per block).
__global__ __launch_bounds__(kAggThreads) void rev_count_kernel(
    const int32_t *adj, const int32_t *deg, const int32_t *items, int32_t nb, int32_t R,
    int32_t *rcnt, int32_t *ntargets, int32_t *tlist, int32_t *tidx, int32_t *ticket) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool act = i < (int64_t)nb * R;
  int32_t q = -1;
  int slot = -1;
  if (act) {
    const int t = (int)(i / R), e = (int)(i % R);
    const int32_t p = items[t];
    act = e < deg[p];
    if (act) {
      q = adj[(int64_t)p * R + e];
      slot = atomicAdd(&rcnt[q], 1);
      ticket[i] = slot;
    }
  }
  const uint64_t fm = ballot(act && slot == 0);
  const int cnt[1] = {(int)__popcll(fm)};
  int32_t *const ctr[1] = {ntargets};
  int base[1];
  block_claim<1>(cnt, ctr, base);
  if (act && slot == 0) {
    const int u = base[0] + lanes_below(fm);
    tlist[u] = q;
    tidx[q] = u;
  }
}
// Segment offsets of the targets, and two work lists in tord: targets with at
// most `light` new sources from the front (tord[0, *front)), the others from the
// back (tord[nt - *back, nt)).  The two lists are pruned by separate launches
// whose LDS is sized for their candidate counts.  Offsets and list slots are
// handed out per block (wave prefix sums and ballots, then block_claim).
__global__ __launch_bounds__(kAggThreads) void rev_alloc_kernel(
    const int32_t *tlist, const int32_t *ntargets, const int32_t *rcnt, int32_t *toff,
    int32_t *tcnt, int32_t *cursor, int32_t *tord, int32_t *front, int32_t *back, int32_t light,
    int32_t maxt) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int nt = *ntargets;
  const bool act = u < maxt && u < nt;
  const int c = act ? rcnt[tlist[u]] : 0;
  const int incl = wave_prefix_sum(c);
  const bool li = act && c <= light;
  const uint64_t lm = ballot(li), hm = ballot(act && !li);
  const int cnt[3] = {__shfl(incl, kWave - 1), (int)__popcll(lm), (int)__popcll(hm)};
  int32_t *const ctr[3] = {cursor, front, back};
  int base[3];
  block_claim<3>(cnt, ctr, base);
  if (act) {
    tcnt[u] = c;
    toff[u] = base[0] + incl - c;
  }
  if (li) tord[base[1] + lanes_below(lm)] = u;
  else if (act) tord[nt - 1 - (base[2] + lanes_below(hm))] = u;
}
// Sources grouped by target; with adjacency keys, the source's key for the
// target too: D(q, p) is taken as D(p, q), the measure p's prune formed.
__global__ void rev_scatter_kernel(const int32_t *adj, const int32_t *deg, const int32_t *items,
                                   int32_t nb, int32_t R, const int32_t *tidx,
                                   const int32_t *toff, const int32_t *ticket, int32_t *seg,
                                   const uint64_t *akey, uint64_t *segk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nb * R) return;
  const int t = (int)(i / R), e = (int)(i % R);
  const int32_t p = items[t];
  if (e >= deg[p]) return;
  const int64_t ae = (int64_t)p * R + e;
  const int32_t q = adj[ae];
  const int64_t pos = (int64_t)toff[tidx[q]] + ticket[i];
  PECANN_CHECK(pos >= 0 && pos < (int64_t)nb * R, CK_REVERSE);  // segments hold the batch's edges
  seg[pos] = p;
  if (akey) segk[pos] = (akey[ae] & 0xffffffff00000000ull) | (uint32_t)p;
}
hipError_t launch_rev_count(const int32_t *adj, const int32_t *deg, const int32_t *items,
                            int32_t nb, int32_t R, int32_t *rcnt, int32_t *ntargets,
                            int32_t *tlist, int32_t *tidx, int32_t *ticket, hipStream_t s) {
  const int64_t tot = (int64_t)nb * R;
  hipLaunchKernelGGL(rev_count_kernel, dim3((unsigned)((tot + kAggThreads - 1) / kAggThreads)),
                     dim3(kAggThreads), 0, s, adj, deg, items, nb, R, rcnt, ntargets, tlist, tidx,
                     ticket);
  return hipGetLastError();
}
hipError_t launch_rev_alloc(const int32_t *tlist, const int32_t *ntargets, const int32_t *rcnt,
                            int32_t *toff, int32_t *tcnt, int32_t *cursor, int32_t *tord,
                            int32_t *front, int32_t *back, int32_t light, int32_t maxt,
                            hipStream_t s) {
  hipLaunchKernelGGL(rev_alloc_kernel, dim3((unsigned)((maxt + kAggThreads - 1) / kAggThreads)),
                     dim3(kAggThreads), 0, s, tlist, ntargets, rcnt, toff, tcnt, cursor, tord, front,
                     back, light, maxt);
  return hipGetLastError();
}
hipError_t launch_rev_scatter(const int32_t *adj, const int32_t *deg, const int32_t *items,
                              int32_t nb, int32_t R, const int32_t *tidx,
                              const int32_t *toff, const int32_t *ticket, int32_t *seg,
                              const uint64_t *akey, uint64_t *segk, hipStream_t s) {
  const int64_t tot = (int64_t)nb * R;
  hipLaunchKernelGGL(rev_scatter_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, adj,
                     deg, items, nb, R, tidx, toff, ticket, seg, akey, segk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Smallest rank key (the densest point) of each instance, one workgroup each.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void min_key_kernel(const uint64_t *key, InstTable inst, uint64_t *out_all) {
  __shared__ uint64_t part[16];
  const int64_t lo = inst.off[blockIdx.x], hi = inst.off[blockIdx.x + 1];
  uint64_t *out = out_all + blockIdx.x;
  uint64_t m = kNoKey;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 1024) m = key[i] < m ? key[i] : m;
  m = wave_min_u64(m);
  if (lane_id() == 0) part[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x < 64) {
    uint64_t v = threadIdx.x < 16 ? part[threadIdx.x] : kNoKey;
    v = wave_min_u64(v);
    if (threadIdx.x == 0) *out = v;
  }
}
hipError_t launch_min_key(const uint64_t *key, const InstTable &inst, uint64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(min_key_kernel, dim3((unsigned)inst.count), dim3(1024), 0, s, key, inst, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K5: DPBruteForce over the kNN list.  The list is in (distance, index) order,
// so the first entry of strictly smaller rank key is the argmin.  The densest
// point gets no dependent; the others left without one join the unfinished list.
// ---------------------------------------------------------------------------
__global__ void dep_in_knn_kernel(int64_t n, InstTable inst, int32_t kstride, const uint64_t *key,
                                  const uint64_t *minkey, const int32_t *knn_idx,
                                  const float *knn_dist, int32_t *dep, float *delta,
                                  int32_t *ulist, int32_t *ucount, int32_t *ucnt_inst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ti = find_instance(inst, i);
  const int k = inst.k[ti];
  const uint64_t ki = key[i];
  if (ki == minkey[ti]) {
    dep[i] = -1;
    delta[i] = __int_as_float(0x7f800000);
    return;
  }
  for (int t = 0; t < k; ++t) {
    const int32_t j = knn_idx[i * kstride + t];
    if (j >= 0 && key[j] < ki) {
      dep[i] = j;
      delta[i] = knn_dist[i * kstride + t];
      return;
    }
  }
  dep[i] = -1;
  delta[i] = __int_as_float(0x7f800000);
  ulist[atomicAdd(ucount, 1)] = (int32_t)i;
  atomicAdd(ucnt_inst + ti, 1);
}
hipError_t launch_dep_in_knn(int64_t n, const InstTable &inst, int32_t kstride, const uint64_t *key,
                             const uint64_t *minkey, const int32_t *knn_idx, const float *knn_dist,
                             int32_t *dep, float *delta, int32_t *ulist, int32_t *ucount,
                             int32_t *ucnt_inst, hipStream_t s) {
  hipLaunchKernelGGL(dep_in_knn_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, inst,
                     kstride, key, minkey, knn_idx, knn_dist, dep, delta, ulist, ucount, ucnt_inst);
  return hipGetLastError();
}

__global__ void bf_dep_finalize_kernel(const int32_t *ulist, const int32_t *ucount,
                                       const unsigned long long *best, int32_t metric, int32_t *dep,
                                       float *delta, int32_t maxu) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= maxu || u >= *ucount) return;
  const uint64_t b = best[u];
  if (b == kNoKey) return;
  const int32_t i = ulist[u];
  dep[i] = key_id(b);
  delta[i] = measure_to_dist(key_measure(b), metric);
}
hipError_t launch_bf_dep_finalize(const int32_t *ulist, const int32_t *ucount,
                                  const unsigned long long *best, int32_t metric, int32_t *dep,
                                  float *delta, int32_t maxu, hipStream_t s) {
  hipLaunchKernelGGL(bf_dep_finalize_kernel, dim3((unsigned)((maxu + 255) / 256)), dim3(256), 0, s,
                     ulist, ucount, best, metric, dep, delta, maxu);
  return hipGetLastError();
}

__global__ void copy_count_kernel(const int32_t *src, int32_t *dst) {
  if (threadIdx.x == 0) *dst = *src;
}
hipError_t launch_copy_count(const int32_t *src, int32_t *dst, int32_t, hipStream_t s) {
  hipLaunchKernelGGL(copy_count_kernel, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

// Unsigned key with the order of the float (negative values included).
__device__ __forceinline__ uint32_t ordered_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ---------------------------------------------------------------------------
// Density functions from the kNN lists (Sec. 4.2 kth and normalized; the
// appendix's exp-sum, sum-exp and sum), in float32 from the reported
// distances.  Rank key: (~ordered_bits(rho) << 32) | index, so a smaller key
// is a strictly higher density with ties to the lower index.
// ---------------------------------------------------------------------------
__global__ void density_kernel(int64_t n, InstTable inst, int32_t kstride, int32_t fn,
                               const int32_t *knn_idx, const float *knn_dist, float *rho,
                               uint64_t *rank_key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = inst.k[find_instance(inst, i)];
  const float *ds = knn_dist + i * kstride;
  float v;
  if (fn == PECANN_DENSITY_KTH) {
    v = 1.0f / ds[k - 1];
  } else if (fn == PECANN_DENSITY_NORMALIZED) {
    float s = 0.f;
    for (int t = 0; t < k; ++t) s += 1.0f / knn_dist[(int64_t)knn_idx[i * kstride + t] * kstride + (k - 1)];
    v = (1.0f / ds[k - 1]) * (float)k / s;
  } else if (fn == PECANN_DENSITY_EXP_SUM) {
    float s = 0.f;
    for (int t = 0; t < k; ++t) s = fmaf(ds[t], ds[t], s);
    v = expf(-s / (float)k);
  } else if (fn == PECANN_DENSITY_SUM_EXP) {
    float s = 0.f;
    for (int t = 0; t < k; ++t) s += expf(-ds[t] * ds[t]);
    v = s / (float)k;
  } else {
    float s = 0.f;
    for (int t = 0; t < k; ++t) s += ds[t];
    v = -s;
  }
  rho[i] = v;
  // the kth keys stay those of the kNN search, which order by the k-th
  // neighbour's measure itself (1 / sqrt of it can tie where the measure does not)
  if (fn != PECANN_DENSITY_KTH) rank_key[i] = ((uint64_t)(~ordered_bits(v)) << 32) | (uint32_t)i;
}
hipError_t launch_density(int64_t n, const InstTable &inst, int32_t kstride, int32_t fn,
                          const int32_t *knn_idx, const float *knn_dist, float *rho,
                          uint64_t *rank_key, hipStream_t s) {
  hipLaunchKernelGGL(density_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, inst,
                     kstride, fn, knn_idx, knn_dist, rho, rank_key);
  return hipGetLastError();
}

// Local centers (appendix, Local Center): non-noise points whose rank key is
// smaller than that of every one of their k nearest neighbours.
__global__ void local_centers_kernel(int64_t n, InstTable inst, int32_t kstride,
                                     const int32_t *knn_idx, const uint64_t *rank_key,
                                     const float *rho, float rho_min, uint8_t *is_center) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = inst.k[find_instance(inst, i)];
  bool c = !(rho[i] < rho_min);
  const uint64_t ki = rank_key[i];
  for (int t = 0; t < k && c; ++t) {
    const int32_t j = knn_idx[i * kstride + t];
    c = j >= 0 && ki < rank_key[j];
  }
  is_center[i] = c ? 1 : 0;
}
hipError_t launch_local_centers(int64_t n, const InstTable &inst, int32_t kstride,
                                const int32_t *knn_idx, const uint64_t *rank_key, const float *rho,
                                float rho_min, uint8_t *is_center, hipStream_t s) {
  hipLaunchKernelGGL(local_centers_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, inst,
                     kstride, knn_idx, rank_key, rho, rho_min, is_center);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K10 + K11: noise, centers, labels.
// gkey[i] = 0 for noise; else (ordered_bits(gamma_i) << 32) | (0xffffffff - i),
// so the n_c largest keys are the n_c largest gamma with ties to the lower
// index (gamma may be negative for the `sum` density).
// ---------------------------------------------------------------------------
__global__ void gamma_kernel(int64_t n, const float *rho, const float *delta, int32_t center_mode,
                             float delta_min, float rho_min, uint64_t *gkey, uint8_t *is_center) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool noise = rho[i] < rho_min;
  if (center_mode == PECANN_CENTER_PRODUCT) {
    float g = rho[i] * delta[i];
    if (g != g) g = 0.f;  // inf * 0
    gkey[i] = noise ? 0ull : (((uint64_t)ordered_bits(g) << 32) | (uint32_t)(0xffffffffu - (uint32_t)i));
    is_center[i] = 0;
  } else if (center_mode == PECANN_CENTER_THRESHOLD) {
    gkey[i] = noise ? 1ull : 0ull;
    is_center[i] = (!noise && delta[i] >= delta_min) ? 1 : 0;
  } else {  // given centers; noise points are never centers
    gkey[i] = noise ? 1ull : 0ull;
    is_center[i] = (!noise && is_center[i]) ? 1 : 0;
  }
}

// Radix select (8 passes of 8 bits) of the n_c-th largest key of each
// instance (one workgroup each); marks centers.
__global__ __launch_bounds__(1024) void select_kernel(InstTable inst, const uint64_t *gkey,
                                                       uint8_t *is_center) {
  __shared__ int32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int32_t s_need;
  __shared__ int32_t s_nonnoise;
  const int64_t lo = inst.off[blockIdx.x], hi = inst.off[blockIdx.x + 1];
  const int32_t n_c = inst.nc[blockIdx.x];
  if (threadIdx.x == 0) { s_prefix = 0; s_need = n_c; s_nonnoise = 0; }
  __syncthreads();
  {
    int c = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 1024) c += gkey[i] != 0;
    c = wave_sum_i32(c);
    if (lane_id() == 0) atomicAdd(&s_nonnoise, c);
  }
  __syncthreads();
  uint64_t thr;
  if (s_nonnoise <= n_c) {
    thr = 1;  // every non-noise point is a center
  } else {
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int b = threadIdx.x; b < 256; b += 1024) hist[b] = 0;
      __syncthreads();
      const uint64_t prefix = s_prefix;
      const uint64_t hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
      for (int64_t i = lo + threadIdx.x; i < hi; i += 1024) {
        const uint64_t k = gkey[i];
        if ((k & hmask) == prefix) atomicAdd(&hist[(k >> shift) & 0xff], 1);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int need = s_need;
        int b = 255;
        for (; b > 0; --b) {
          if (hist[b] >= need) break;
          need -= hist[b];
        }
        s_need = need;
        s_prefix = prefix | ((uint64_t)b << shift);
      }
      __syncthreads();
    }
    thr = s_prefix;
  }
  for (int64_t i = lo + threadIdx.x; i < hi; i += 1024) {
    const uint64_t k = gkey[i];
    is_center[i] = (k != 0 && k >= thr) ? 1 : 0;
  }
}

// The same select for one large instance over the whole GPU: per 8-bit digit,
// every block counts the keys that match the prefix so far in an LDS
// histogram and adds it to the state's, then one thread picks the digit (the
// counts from the top until n_c is reached) and clears the histogram for the
// next digit.  The result -- the n_c-th largest key as threshold, or 1 when at
// most n_c points are not noise -- is the workgroup select's.
struct SelState {
  unsigned long long prefix;
  int32_t need, nonnoise, done;
  int32_t pad[59];
  int32_t hist[256];
};
static_assert(sizeof(SelState) == 4 * kSelWords, "select state size");

__global__ __launch_bounds__(256) void sel_init_kernel(SelState *st, const int32_t *nc) {
  st->hist[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    st->prefix = 0;
    st->need = nc[0];
    st->nonnoise = 0;
    st->done = 0;
  }
}

__global__ __launch_bounds__(256) void sel_hist_kernel(int64_t n, const uint64_t *gkey, SelState *st,
                                                        int32_t shift) {
  __shared__ int32_t h[256];
  __shared__ int32_t cnt;
  if (st->done) return;
  h[threadIdx.x] = 0;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const uint64_t prefix = st->prefix;
  const uint64_t hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint64_t k = gkey[i];
    c += k != 0;
    if ((k & hmask) == prefix) atomicAdd(&h[(k >> shift) & 0xff], 1);
  }
  if (shift == 56) {
    c = wave_sum_i32(c);
    if (lane_id() == 0) atomicAdd(&cnt, c);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
  if (shift == 56 && threadIdx.x == 0 && cnt) atomicAdd(&st->nonnoise, cnt);
}

__global__ void sel_pick_kernel(SelState *st, int32_t shift) {
  if (threadIdx.x != 0 || st->done) return;
  if (shift == 56 && st->nonnoise <= st->need) {  // every non-noise point is a center
    st->prefix = 1;
    st->done = 1;
    return;
  }
  int need = st->need;
  int b = 255;
  for (; b > 0; --b) {
    const int hb = st->hist[b];
    if (hb >= need) break;
    need -= hb;
  }
  st->need = need;
  st->prefix |= (unsigned long long)b << shift;
  for (int t = 0; t < 256; ++t) st->hist[t] = 0;
  if (shift == 0) st->done = 1;
}

__global__ __launch_bounds__(256) void sel_mark_kernel(int64_t n, const uint64_t *gkey, const SelState *st,
                                                        uint8_t *is_center) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t thr = st->prefix, k = gkey[i];
  is_center[i] = (k != 0 && k >= thr) ? 1 : 0;
}

__global__ void parent_kernel(int64_t n, const int32_t *dep, const uint8_t *is_center,
                              const uint64_t *gkey, const float *rho, float rho_min,
                              int32_t *labels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool noise = rho[i] < rho_min;
  const int32_t d = dep[i];
  const bool root = noise || is_center[i] || d < 0 || d >= n;  // out-of-range ids end a path
  labels[i] = root ? (int32_t)i : d;
}

// Pointer jumping: every value ever stored is an ancestor on the same path, so
// concurrent updates only speed convergence.  `flag` records a path that did not
// end within the step bound (a cycle: dependent pointers that do not go up).
__global__ void jump_kernel(int64_t n, int32_t *labels, int32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t cur = __hip_atomic_load(&labels[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  PECANN_CHECK(cur >= 0 && cur < n, CK_LABEL);
  for (int64_t step = 0; step <= n; ++step) {
    const int32_t nxt = __hip_atomic_load(&labels[cur], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (nxt == cur) {
      __hip_atomic_store(&labels[i], cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    cur = nxt;
    __hip_atomic_store(&labels[i], cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  atomicAdd(flag, 1);
}

hipError_t launch_cluster(int64_t n, const InstTable &inst, const float *rho, const int32_t *dep,
                          const float *delta, int32_t center_mode, float delta_min, float rho_min,
                          int32_t *labels, uint8_t *is_center, uint64_t *gkey, int32_t *flag,
                          uint32_t *sel, hipStream_t s) {
  const unsigned b = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(gamma_kernel, dim3(b), dim3(256), 0, s, n, rho, delta, center_mode, delta_min,
                     rho_min, gkey, is_center);
  if (center_mode == PECANN_CENTER_PRODUCT) {
    if (inst.count == 1 && n >= kWideSelect) {
      // one large instance: the select spread over the GPU (8 digit passes)
      SelState *st = (SelState *)sel;
      const unsigned hb = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
      hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(256), 0, s, st, inst.nc);
      for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(sel_hist_kernel, dim3(hb), dim3(256), 0, s, n, gkey, st, shift);
        hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(64), 0, s, st, shift);
      }
      hipLaunchKernelGGL(sel_mark_kernel, dim3(b), dim3(256), 0, s, n, gkey, st, is_center);
    } else {
      hipLaunchKernelGGL(select_kernel, dim3((unsigned)inst.count), dim3(1024), 0, s, inst, gkey,
                         is_center);
    }
  }
  hipLaunchKernelGGL(parent_kernel, dim3(b), dim3(256), 0, s, n, dep, is_center, gkey, rho, rho_min,
                     labels);
  hipLaunchKernelGGL(jump_kernel, dim3(b), dim3(256), 0, s, n, labels, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Instance tables and build-round work lists.
// ---------------------------------------------------------------------------
__global__ void put_i64_kernel(I64Chunk c, int32_t count, int64_t *dst) {
  const int j = threadIdx.x;
  if (j < count) dst[j] = c.v[j];
}
__global__ void put_i32_kernel(I32Chunk c, int32_t count, int32_t *dst) {
  const int j = threadIdx.x;
  if (j < count) dst[j] = c.v[j];
}
hipError_t launch_put_i64(const I64Chunk &c, int32_t count, int64_t *dst, hipStream_t s) {
  hipLaunchKernelGGL(put_i64_kernel, dim3(1), dim3(64), 0, s, c, count, dst);
  return hipGetLastError();
}
hipError_t launch_put_i32(const I32Chunk &c, int32_t count, int32_t *dst, hipStream_t s) {
  hipLaunchKernelGGL(put_i32_kernel, dim3(1), dim3(64), 0, s, c, count, dst);
  return hipGetLastError();
}

// blockIdx.y = range, blockIdx.x * 256 + threadIdx.x = position in it.
__global__ void gather_items_kernel(RangeChunk c, const int32_t *perm, int32_t *items,
                                    int32_t *item_sbase, int32_t *item_ns) {
  const int j = blockIdx.y;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= c.cnt[j]) return;
  const int o = c.obeg[j] + x;
  items[o] = perm[c.pbeg[j] + x];
  item_sbase[o] = c.sbase[j];
  item_ns[o] = c.ns[j];
}
hipError_t launch_gather_items(const RangeChunk &c, int32_t nranges, int32_t maxcnt,
                               const int32_t *perm, int32_t *items, int32_t *item_sbase,
                               int32_t *item_ns, hipStream_t s) {
  if (nranges <= 0 || maxcnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_items_kernel, dim3((unsigned)((maxcnt + 255) / 256), (unsigned)nranges),
                     dim3(256), 0, s, c, perm, items, item_sbase, item_ns);
  return hipGetLastError();
}

__global__ void small_instance_points_kernel(int64_t n, InstTable inst, int32_t below, int32_t *list,
                                             int32_t *count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = find_instance(inst, i);
  if (inst.off[t + 1] - inst.off[t] < below) list[atomicAdd(count, 1)] = (int32_t)i;
}
hipError_t launch_small_instance_points(int64_t n, const InstTable &inst, int32_t below,
                                        int32_t *list, int32_t *count, hipStream_t s) {
  hipLaunchKernelGGL(small_instance_points_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     n, inst, below, list, count);
  return hipGetLastError();
}

PECANN_CHECK_READER(misc)

}  // namespace pecann
