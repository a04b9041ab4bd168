// Wave prefix sums and block-wide claims on shared counters.  Device-scope
// atomics on one address serialise, so kernels that hand out list slots or
// segment offsets sum their counts per block and advance each shared counter
// once per block (1M-point Vamana build: the reverse-edge grouping with one
// atomic per wavefront took 207 + 113 us per round, per block 9.4 ms per step
// in all).
#pragma once
#include "device_common.hpp"

namespace pecann {

// Inclusive prefix sum over the wavefront's lanes.
__device__ __forceinline__ int wave_prefix_sum(int v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(v, off);
    if (l >= off) v += y;
  }
  return v;
}

constexpr int kAggThreads = 1024;  // largest block block_claim serves
constexpr int kAggWaves = kAggThreads / kWave;

// Block-wide exclusive offsets of NV per-wave counts (cnt[v], wave-uniform):
// base[v] = the block's range start in counter ctr[v] plus the counts of the
// block's earlier waves.  One atomic per counter and block.  Every thread of
// the block calls it (it synchronises the block), with blockDim.x <=
// kAggThreads; it may be called repeatedly.
template <int NV>
__device__ __forceinline__ void block_claim(const int (&cnt)[NV], int32_t *const (&ctr)[NV],
                                            int (&base)[NV]) {
  __shared__ int wsum[NV][kAggWaves];
  __shared__ int bbase[NV];
  const int w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  if (lane_id() == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) wsum[v][w] = cnt[v];
  __syncthreads();
  if (threadIdx.x < NV) {
    int tot = 0;
    for (int i = 0; i < nw; ++i) tot += wsum[threadIdx.x][i];
    bbase[threadIdx.x] = tot > 0 ? atomicAdd(ctr[threadIdx.x], tot) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    int b = bbase[v];
    for (int i = 0; i < w; ++i) b += wsum[v][i];
    base[v] = b;
  }
  __syncthreads();  // the next call may overwrite wsum and bbase
}

}  // namespace pecann
