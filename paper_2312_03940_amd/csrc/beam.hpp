// Wavefront-owned sorted candidate lists in LDS: the beam of the greedy search
// (Alg. 1), bounded top-k lists, and the visited hash.
#pragma once

#include "device_common.hpp"

namespace pecann {

// Number of entries of the sorted LDS array a[0..m) that are < key.
__device__ __forceinline__ int lower_bound_u64(const uint64_t *a, int m, uint64_t key) {
  int lo = 0, hi = m;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// A sorted list of at most `cap` distinct keys with one flag byte per entry,
// double-buffered in LDS.  Owned by one wavefront; every call is made by all 64
// lanes of it.
struct SortedList {
  uint64_t *a, *b;  // current / spare key buffers (cap entries each)
  uint8_t *fa, *fb; // flags moving with the keys (expanded marks)
  uint64_t *tmp;    // 64 keys of scratch
  int cap;
  int m;            // entries held
  int hint;         // every entry before index `hint` is flagged

  __device__ __forceinline__ void reset() { m = 0; hint = 0; }

  __device__ __forceinline__ void swap_bufs() {
    uint64_t *t = a; a = b; b = t;
    uint8_t *f = fa; fa = fb; fb = f;
  }

  // Merge one candidate key per lane (kNoKey = none) into the list, keeping the
  // `cap` smallest.  Keys already present are ignored; the keys of one call are
  // distinct.  Returns the number of keys that entered the list.
  __device__ int merge(uint64_t mykey) {
    if (m == cap && mykey != kNoKey && mykey >= a[cap - 1]) mykey = kNoKey;
    const uint64_t cm = ballot(mykey != kNoKey);
    if (cm == 0) return 0;
    return __popcll(cm) <= 16 ? merge_few(mykey) : merge_sorted(mykey);
  }

  // Few candidates: each finds its place in the list by binary search and its
  // rank among the others by direct comparison (no sort).
  __device__ int merge_few(uint64_t mykey) {
    const int l = lane_id();
    bool valid = mykey != kNoKey;
    int pos = 0;
    if (valid) {
      pos = lower_bound_u64(a, m, mykey);
      if (pos < m && a[pos] == mykey) valid = false;
    }
    const uint64_t vb = ballot(valid);
    const int nc = __popcll(vb);
    if (nc == 0) return 0;
    const int slot = lanes_below(vb);
    if (valid) tmp[slot] = mykey;
    wave_lds_sync();
    int r = 0;
    if (valid) {
      for (int t = 0; t < nc; ++t) r += tmp[t] < mykey;
      const int np = pos + r;
      if (np < cap) { b[np] = mykey; fb[np] = 0; }
    }
    for (int j = l; j < m; j += kWave) {
      const uint64_t k = a[j];
      int rj = 0;
      for (int t = 0; t < nc; ++t) rj += tmp[t] < k;
      const int np = j + rj;
      if (np < cap) { b[np] = k; fb[np] = fa[j]; }
    }
    // the smallest new key lands at its own lower bound
    const uint64_t lead = ballot(valid && r == 0);
    const int first_new = __shfl(pos, __builtin_ctzll(lead));
    wave_lds_sync();
    swap_bufs();
    m = min(cap, m + nc);
    hint = min(min(hint, first_new), m);
    return nc;
  }

  // Many candidates: bitonic sort across the wave, then merge by ranks.
  __device__ int merge_sorted(uint64_t mykey) {
    const int l = lane_id();
    uint64_t s = wave_sort_u64(mykey);
    bool valid = (s != kNoKey);
    uint64_t prev = shfl_u64(s, l > 0 ? l - 1 : 0);
    if (l > 0 && prev == s) valid = false;
    int pos = 0;
    if (valid) {
      pos = lower_bound_u64(a, m, s);
      if (pos < m && a[pos] == s) valid = false;
    }
    const uint64_t vb = ballot(valid);
    const int nc = __popcll(vb);
    if (nc == 0) return 0;
    const int r = lanes_below(vb);
    if (valid) tmp[r] = s;
    wave_lds_sync();
    if (valid) {
      const int np = pos + r;
      if (np < cap) { b[np] = s; fb[np] = 0; }
    }
    for (int j = l; j < m; j += kWave) {
      const uint64_t k = a[j];
      const int np = j + lower_bound_u64(tmp, nc, k);
      if (np < cap) { b[np] = k; fb[np] = fa[j]; }
    }
    const int first_new = __shfl(pos, __builtin_ctzll(vb));
    wave_lds_sync();
    swap_bufs();
    m = min(cap, m + nc);
    hint = min(min(hint, first_new), m);
    return nc;
  }

  // Index of the first entry whose flag is 0, or -1 (scans from `hint`).
  __device__ __forceinline__ int first_unflagged() {
    const int l = lane_id();
    for (int base = hint; base < m; base += kWave) {
      const int j = base + l;
      const uint64_t bm = ballot(j < m && fa[j] == 0);
      if (bm) {
        hint = base + __builtin_ctzll(bm);
        return hint;
      }
    }
    hint = m;
    return -1;
  }
};

// Open-addressing set of int32 ids in LDS (slots hold -1 when empty).  It may
// forget: when a probe sequence is exhausted the id is reported as new, which
// only costs a repeated distance evaluation -- the sorted list drops the
// duplicate key, because a point's key is a deterministic function of it.
struct IdHash {
  int32_t *slot;
  int bits;
  __device__ __forceinline__ void clear() {
    const int H = 1 << bits;
    for (int s = lane_id(); s < H; s += kWave) slot[s] = -1;
  }
  // true if id was not in the set (and is now, if there was room)
  __device__ __forceinline__ bool insert(int32_t id) {
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t s = ((uint32_t)id * 2654435761u) >> (32 - bits);
    for (int probe = 0; probe < 16; ++probe) {
      const int old = atomicCAS(&slot[s], -1, id);
      if (old == -1) return true;
      if (old == id) return false;
      s = (s + 1) & mask;
    }
    return true;
  }
};

// Sort cnt distinct keys src[0..cnt) into dst[0..cnt) by counting ranks.
__device__ __forceinline__ void lds_rank_sort(const uint64_t *src, uint64_t *dst, int cnt) {
  for (int j = lane_id(); j < cnt; j += kWave) {
    const uint64_t k = src[j];
    int r = 0;
    for (int t = 0; t < cnt; ++t) r += (src[t] < k);
    dst[r] = k;
  }
  wave_lds_sync();
}

}  // namespace pecann
