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
  uint64_t tail;    // key of the last entry (kNoKey while empty)

  __device__ __forceinline__ void reset() { m = 0; hint = 0; tail = kNoKey; }

  __device__ __forceinline__ void swap_bufs() {
    uint64_t *t = a; a = b; b = t;
    uint8_t *f = fa; fa = fb; fb = f;
  }

  // Merge one candidate key per lane (kNoKey = none) into the list, keeping the
  // `cap` smallest.  The merges are always inlined: an out-of-line copy would
  // reach the LDS through generic pointers from a scratch stack.  Keys already present are ignored; the keys of one call are
  // distinct.  Returns the number of keys that entered the list.
  __device__ __forceinline__ int merge(uint64_t mykey) {
    if (m == cap && mykey >= tail) mykey = kNoKey;
    const uint64_t cm = ballot(mykey != kNoKey);
    if (cm == 0) return 0;
    return __popcll(cm) <= 16 ? merge_few(mykey) : merge_sorted(mykey);
  }

  // Few candidates: each finds its place in the list by binary search and its
  // rank among the others by direct comparison (no sort); the list is updated
  // in place, moving only the entries behind the first insertion point (in
  // 64-entry chunks from the top, each read before any of it is written).
  __device__ __forceinline__ int merge_few(uint64_t mykey) {
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
    if (valid)
      for (int t = 0; t < nc; ++t) r += tmp[t] < mykey;
    // the smallest new key lands at its own lower bound; entries before it stay
    const uint64_t lead = ballot(valid && r == 0);
    const int first_new = __shfl(pos, __builtin_ctzll(lead));
    for (int top = m; top > first_new;) {
      const int c0 = max(first_new, top - kWave);
      const int j = c0 + l;
      uint64_t k = 0;
      uint8_t f = 0;
      int np = cap;
      if (j < top) {
        k = a[j];
        f = fa[j];
        int rj = 0;
        for (int t = 0; t < nc; ++t) rj += tmp[t] < k;
        np = j + rj;
      }
      wave_lds_sync();
      if (np < cap) { a[np] = k; fa[np] = f; }
      wave_lds_sync();
      top = c0;
    }
    if (valid && pos + r < cap) { a[pos + r] = mykey; fa[pos + r] = 0; }
    wave_lds_sync();
    m = min(cap, m + nc);
    hint = min(min(hint, first_new), m);
    tail = a[m - 1];
    return nc;
  }

  // Many candidates: bitonic sort across the wave, then merge by ranks.
  __device__ __forceinline__ int merge_sorted(uint64_t mykey) {
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
    tail = a[m - 1];
    return nc;
  }

  // Index of the first entry whose flag is 0, or -1 (scans from `hint`); its
  // key is read in the same pass.
  __device__ __forceinline__ int first_unflagged(uint64_t &key) {
    const int l = lane_id();
    for (int base = hint; base < m; base += kWave) {
      const int j = base + l;
      uint8_t fl = 1;
      uint64_t k = kNoKey;
      if (j < m) { fl = fa[j]; k = a[j]; }
      const uint64_t bm = ballot(fl == 0);
      if (bm) {
        const int t = __builtin_ctzll(bm);
        hint = base + t;
        key = readlane_u64(k, t);
        return hint;
      }
    }
    hint = m;
    return -1;
  }
};

// Open-addressing set of int32 ids in LDS (slots hold -1 when empty), in
// buckets of four slots (16 bytes, read at once).  A lookup reads a bucket,
// and claims an empty slot with a compare-and-swap only when the id is absent;
// it visits at most kProbes buckets.  The set may forget: when they are full the
// id is reported as new, which only costs a repeated distance evaluation --
// the sorted list drops the duplicate key, because a point's key is a
// deterministic function of it.  The ids inserted by one call are distinct.
//
// Compact form (16-bit slots, half the LDS): ids < 2^kb are mapped by
// h = id * c mod 2^kb (c odd: a bijection of [0, 2^kb)); the top bits of h
// pick the home bucket and a slot keeps only the rest, rem = h mod 2^rb, with
// the probe distance p in the next two bits.  (bucket - p, rem) gives h back,
// hence the id: nothing is confused with anything else, so the set answers
// exactly as the 32-bit one does (it may forget, never invent).  0xffff marks
// an empty slot (rem | p << rb < 2^15 with rb <= 13).  A bucket (four slots,
// 8 bytes) is read at once and claimed with a 64-bit compare-and-swap.
struct IdHash {
  int32_t *slot;  // 16-byte aligned
  int bits;       // log2 of the slot count (>= 3)
  int rb = -1;    // compact form: remainder bits (kb - bits + 2); -1: 32-bit slots
  uint32_t kmask = 0;  // compact form: 2^kb - 1
  // buckets visited at most.  Eight instead of four cut the 1.28M x 1024 FP8
  // build search's fetched bytes by only 1.5 % (80.2 -> 79.0 GB per launch,
  // against 70.0 GB of algorithmic reads; most of the rest are the 64-byte
  // lines around each 4-byte row scale) and made it 4 % slower
  static constexpr int kProbes = 4;
  __device__ __forceinline__ void clear() {
    const int H = 1 << bits;
    if (rb >= 0) {
      uint64_t *b64 = (uint64_t *)slot;
      for (int s = lane_id(); s < (H >> 2); s += kWave) b64[s] = ~0ull;
      return;
    }
    for (int s = lane_id(); s < H; s += kWave) slot[s] = -1;
  }
  __device__ __forceinline__ bool insert16(int32_t id) {
    const uint32_t mask = (1u << (bits - 2)) - 1u;
    const uint32_t h = ((uint32_t)id * 2654435761u) & kmask;
    uint32_t b = h >> rb;
    const uint32_t rem = h & ((1u << rb) - 1u);
    for (int probe = 0; probe < kProbes; ++probe) {
      unsigned long long *bk = (unsigned long long *)slot + b;
      const uint64_t tgt = rem | ((uint32_t)probe << rb);
      uint64_t v = *bk;
      for (;;) {
        int empty = -1;
        bool found = false;
#pragma unroll
        for (int e = 3; e >= 0; --e) {
          const uint64_t x = (v >> (16 * e)) & 0xffffull;
          found |= x == tgt;
          if (x == 0xffffull) empty = e;
        }
        if (found) return false;
        if (empty < 0) break;
        const uint64_t nv = (v & ~(0xffffull << (16 * empty))) | (tgt << (16 * empty));
        const uint64_t old = atomicCAS(bk, (unsigned long long)v, (unsigned long long)nv);
        if (old == v) return true;
        v = old;  // another lane took a slot of this bucket: look again
      }
      b = (b + 1) & mask;
    }
    return true;
  }
  // true if id was not in the set (and is now, if there was room)
  __device__ __forceinline__ bool insert(int32_t id) {
    if (rb >= 0) return insert16(id);
    const int bb = bits - 2;
    const uint32_t mask = (1u << bb) - 1u;
    uint32_t b = ((uint32_t)id * 2654435761u) >> (32 - bb);
    for (int probe = 0; probe < kProbes; ++probe) {
      int32_t *bucket = slot + 4 * b;
      const int4 v = *(const int4 *)bucket;
      if (v.x == id || v.y == id || v.z == id || v.w == id) return false;
      const int e4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (e4[e] != -1) continue;
        const int old = atomicCAS(&bucket[e], -1, id);
        if (old == -1) return true;
        if (old == id) return false;
      }
      b = (b + 1) & mask;
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
