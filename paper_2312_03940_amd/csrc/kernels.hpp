// Internal interface between the C-ABI layer (pecann_abi.hip) and the kernel
// translation units.  Every launcher enqueues on the given stream and returns
// the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pecann.h"

namespace pecann {

// Shape S of the gather-distance engine for a row format: the smallest power
// of two >= 4 and >= the row's number of 16-byte chunks (lanes x chunks per
// lane of one candidate).
int engine_shape(int32_t search_dtype, int32_t d);

struct RowsDesc {  // host copy of the row description (mirrors Rows)
  const uint8_t *xs;
  int64_t xs_stride;
  const float *scale;
  const float *xr;
  int64_t xr_stride;
  // per search row: squared norm of the values the matrix cores multiply --
  // float for F32/BF16/FP8 (dequantised), int32 bits of sum (x - 128)^2 over
  // the padded row for U8
  const uint32_t *sqn;
  const float *sqn_r;  // squared norms of the float32 rerank rows (BF16/FP8), else nullptr
  // MXFP6 search rows (PECANN_MXFP6 only, else nullptr): the rows the beam
  // searches score; every other kernel reads the FP8 copy in xs
  const uint8_t *xg;
  int64_t xg_stride;  // bytes
  int32_t xg_soff;    // byte offset of a row's scale words
  const uint32_t *sqn_g;  // squared norms of the dequantised MXFP6 rows (float bits)
  int32_t nch;
  int32_t nch_r;
  int32_t d;
  int32_t metric;
};

enum SearchMode { MODE_KNN = 0, MODE_DEP = 1, MODE_BUILD = 2 };

#ifdef PECANN_CHECKED
// invariant-check words of each translation unit (read and cleared)
uint32_t check_take_search();
uint32_t check_take_search_mfma();
uint32_t check_take_prune();
uint32_t check_take_misc();
uint32_t check_take_bruteforce();
uint32_t check_take_exact();
uint32_t check_take_nndescent();
#endif

// Independent instances over one point set (device tables): instance t owns
// points [off[t], off[t+1]); k[t] and nc[t] are its kNN size and center count.
struct InstTable {
  const int64_t *off;  // [count + 1]
  const int32_t *k;    // [count]
  const int32_t *nc;   // [count]
  int32_t count;
};

struct SearchParams {
  RowsDesc rows;
  const int32_t *adj;
  const int32_t *deg;
  int32_t R;
  int32_t n;
  const int32_t *items;       // point per work item (nullptr: item index is the point)
  const int32_t *item_count;  // device count of items (nullptr: nitems)
  int32_t nitems;
  int32_t *head;              // device work-queue head, 0 at launch
  const int32_t *starts;      // start points besides the query itself
  int32_t nstarts;
  const int32_t *item_sbase;  // per item: its start points are starts[item_sbase[it] ..]
  const int32_t *item_ns;     // per item: ... and there are item_ns[it] of them
                              // (both nullptr: starts[0 .. nstarts) for every item)
  InstTable inst;             // instance of each query (k per instance, round limits)
  int32_t L;                  // beam width
  int32_t hbits;              // log2 of visited-hash slots
  int32_t hid_bits;           // compact (16-bit) visited hash over ids < 2^hid_bits; 0: 32-bit slots
  int32_t mode;
  int32_t rerank;             // entries re-scored in float32 (0: none)
  int32_t mfma;               // BF16 / FP8 rows: score candidates on the matrix cores
  // MODE_KNN (k: the instance's, kstride: row stride of knn_idx / knn_dist)
  int32_t k;
  int32_t kstride;
  int32_t *knn_idx;
  float *knn_dist;
  float *rho;
  uint64_t *rank_key;
  int32_t *fb_list;           // queries with fewer than k results
  int32_t *fb_count;
  // MODE_DEP
  int32_t kdep;
  const uint64_t *key_in;
  int32_t *dep;
  float *delta;
  int32_t *u_out;
  int32_t *u_out_count;
  int32_t threshold;
  int32_t kdep_cap;           // per-instance limit min(kdep_cap, n_t - 1) on kdep
  const int32_t *ucnt_in;     // [instance] unfinished points entering this round
  int32_t *ucnt_out;          // [instance] unfinished points leaving it
  // MODE_BUILD
  uint64_t *vis;              // [item][vcap] keys of expanded points
  int32_t *vis_count;         // [item] expansions (may exceed vcap)
  int32_t vcap;
  // optional work counters (nullptr: off): [0] expansions, [1] neighbour ids
  // read, [2] rows gathered for distances, [3] float32 rows re-scored
  unsigned long long *counters;
};

size_t search_lds_bytes(int L, int hbits, int hid_bits);
// id bits of the compact visited hash for n points and 2^hbits slots, or 0
// when the ids need more than 13 bits beside the home bucket (32-bit slots)
int compact_hash_bits(int64_t n, int hbits);
hipError_t launch_search(int32_t dt, int S, const SearchParams &p, int grid, hipStream_t s);
// the matrix-core scoring variant (BF16 / FP8 rows); launch_search dispatches to it
hipError_t launch_search_mfma(int32_t dt, int S, const SearchParams &p, int grid, hipStream_t s);

// Exact (brute-force) kNN over the query's instance for a list of queries.
struct BfKnnParams {
  RowsDesc rows;
  int32_t n;
  int32_t k;                  // k of every query without an instance table
  int32_t kstride;            // row stride of knn_idx / knn_dist
  InstTable inst;
  int32_t skip_from;          // queries of instances with >= skip_from points are skipped
  const int32_t *items;       // nullptr: all points
  const int32_t *item_count;  // nullptr: nitems
  int32_t nitems;
  int32_t *head;
  int32_t *knn_idx;
  float *knn_dist;
  float *rho;
  uint64_t *rank_key;
  int32_t item_from;          // bf_knn takes items [item_from, count)
  // split path (launch_bf_knn_split): items [0, min(count, split_cap)), each
  // scanned as nchunk chunks of `chunk` candidates by separate wavefronts; a
  // chunk's kpart best keys go to part[item][chunk][0 .. kpart), then one
  // wavefront per item merges them
  uint64_t *part;
  int32_t split_cap;
  int32_t nchunk;
  int32_t chunk;
  int32_t kpart;
  int32_t *head2;             // work queue of the merge
};
size_t bf_knn_lds_bytes(int k);
hipError_t launch_bf_knn(int32_t dt, int S, const BfKnnParams &p, int grid, hipStream_t s);
hipError_t launch_bf_knn_split(int32_t dt, int S, const BfKnnParams &p, int grid_chunks, int grid_merge,
                               hipStream_t s);

// Exact dependent point for a list of unfinished points: chunked argmin over
// the points of strictly smaller rank key.
struct BfDepParams {
  RowsDesc rows;
  int32_t n;
  const int32_t *ulist;
  const int32_t *ucount;
  int32_t chunk;
  int32_t nchunks;
  int32_t *head;
  InstTable inst;             // candidates come from the query's instance
  const uint64_t *key;
  unsigned long long *best;  // [u] packed (measure, index), ~0 at launch
};
hipError_t launch_bf_dep(int32_t dt, int S, const BfDepParams &p, int grid, hipStream_t s);

// RobustPrune for a batch of new points (forward) and the reverse-edge merge.
struct PruneParams {
  RowsDesc rows;
  int32_t n;
  int32_t R;
  float alpha;
  int32_t *adj;
  int32_t *deg;
  // forward
  const int32_t *items;       // batch point of item t
  int32_t nb;
  const uint64_t *vis;
  const int32_t *vis_count;
  int32_t vcap;
  // reverse
  const int32_t *tlist;
  const int32_t *tord;        // work lists (indices into tlist): light from the front,
                              // heavy from the back
  const int32_t *nlight;      // length of the light list
  const int32_t *nheavy;      // length of the heavy list
  int32_t heavy;              // 0: prune the light list, 1: the heavy list
  const int32_t *ntargets;
  const int32_t *toff;
  const int32_t *tcnt;
  const int32_t *seg;
  int32_t *rcnt;
  int32_t capin;              // new in-edges a target's LDS holds at once (light list:
                              // the list's bound; heavy list: more are pruned in slices)
  int32_t *head;
  // keys (D(v, u), u) of the adjacency entries, kept beside adj (nullptr: none
  // kept; every prune then forms its distances from tiles), and of the batch's
  // reverse edges grouped by target ((D(p, q), p) for source p)
  uint64_t *akey;
  uint64_t *segk;
  // per point, how many leading adjacency entries its last prune selected
  // (nullptr: not kept)
  int32_t *cons;
  // NN-descent graph: Nout(i) = RobustPrune(i, list_i u rev_i) with the lists
  // (lk keys per point, kNoKey = empty) and reverse lists (lk ids, -1 = empty)
  const uint64_t *lists;
  const int32_t *rlists;
  int32_t lk;
  // optional work counters (nullptr: off): [0] row reads by forward prunes and
  // [1] by reverse prunes (32 per 16 x 16 tile), [2] targets pruned, [3] targets
  // appended
  unsigned long long *counters;
  int32_t sg;  // tile steps per memory round trip (0: the rule; else 2 or 4)
};
size_t prune_lds_bytes(int ccap, int R, int dt, int metric);
hipError_t launch_prune_forward(int32_t dt, const PruneParams &p, int grid, hipStream_t s);
hipError_t launch_prune_reverse(int32_t dt, const PruneParams &p, int grid, hipStream_t s);
hipError_t launch_prune_lists(int32_t dt, const PruneParams &p, int grid, hipStream_t s);

// NN-descent rounds (see nndescent.hip).  Lists: n x K keys (measure, index)
// ascending, kNoKey = empty, with one flag byte per entry (1 = new).
struct NndParams {
  RowsDesc rows;
  int32_t n;
  int32_t K;
  uint64_t *cur_keys;          // lists as the round began
  uint8_t *cur_flags;
  uint64_t *nxt_keys;          // lists after the round
  uint8_t *nxt_flags;
  int32_t *done;               // set once a round ends at or below the stop level
  unsigned long long *updates; // new entries counted at a round's end
  int32_t *rounds;             // rounds run
  long long thr;               // stop level: floor(delta * n * K)
  // reverse lists: per target the sources grouped (count, offset, ticket)
  int32_t *rcnt, *roff, *rcursor, *rticket;
  uint64_t *rseg;              // (measure, source) keys
  uint8_t *rsegf;              // source's flag
  int32_t *rnew, *rold;        // [n][K] closest new / old sources, -1 padded
  // local joins of one round (queue head kept across the round's passes) and
  // the proposals of one pass: join wave w writes slots [w * seg, (w + 1) * seg)
  int32_t *head;               // work-queue head
  int64_t maxprop;             // proposals of one join at most
  int64_t seg;                 // proposal slots per join wave (>= maxprop)
  int32_t *pfill;              // [join grid] slots each wave filled
  int32_t *ptgt;               // [slots] target
  uint64_t *pkey;              // [slots] (measure, proposed index)
  int32_t *pticket;            // [slots] slot within the target's group
  uint64_t *pseg;              // [slots] keys grouped by target
  int32_t *pcnt, *poff;        // [n] per target (pcnt 0 between chunks)
  int32_t *pcursor;
  int32_t *ptouch, *ptouch_n;  // targets with proposals
  int32_t *overflow;           // proposals that did not fit (never, by sizing)
  // optional work counters: [0] proposals, [1] 16 x 16 join tiles, [2] merges
  unsigned long long *counters;
};
size_t nnd_join_lds_bytes(int K);
hipError_t launch_nnd_init(int32_t dt, const NndParams &p, const int32_t *init, int grid, hipStream_t s);
hipError_t launch_nnd_round_begin(const NndParams &p, int cus, hipStream_t s);
hipError_t launch_nnd_reverse(const NndParams &p, int32_t split, int32_t ignore_done, int cus,
                              hipStream_t s);
hipError_t launch_nnd_join(int32_t dt, const NndParams &p, int grid, hipStream_t s);
hipError_t launch_nnd_proposals(const NndParams &p, int join_grid, int cus, hipStream_t s);
hipError_t launch_nnd_merge(const NndParams &p, int grid, hipStream_t s);
hipError_t launch_nnd_round_end(const NndParams &p, int cus, hipStream_t s);
hipError_t launch_nnd_acc_merge(const NndParams &p, uint64_t *acc, const uint64_t *src, int cus,
                                hipStream_t s);
hipError_t launch_nnd_out(const NndParams &p, const uint64_t *keys, int32_t *idx, float *dist, int cus,
                          hipStream_t s);
hipError_t launch_nnd_copy(const uint64_t *src, uint64_t *dst, int64_t n, int cus, hipStream_t s);

// Plain (non-templated) kernels.
// Center selection over one instance of at least kWideSelect points runs over the
// whole GPU with a state of kSelWords 32-bit words in the cluster workspace.
constexpr int64_t kWideSelect = 4096;
constexpr int kSelWords = 320;

hipError_t launch_prepare(const void *x, int32_t x_dtype, int64_t x_stride, int64_t n, int32_t d,
                          int32_t metric, int32_t sdt, const RowsDesc &rows, uint8_t *xs,
                          float *xr, float *scale, uint32_t *sqn, float *sqn_r, uint8_t *xg,
                          uint32_t *sqn_g, hipStream_t s);

// Exact kNN on the matrix cores: a scan that keeps, per query, the 16 best
// candidates of each lane's column stream by matrix-core distance, then an
// exact (direct-difference) re-score with a rounding-bound check.
// candidates the exact matrix-core scan keeps per query (16 lanes x 8)
constexpr int kExactCand = 128;
constexpr int kExactParts = 2;  // parts of the points the exact scan's workgroups take

struct ExactMfmaParams {
  RowsDesc rows;              // one instance's rows (row 0 = global index base)
  int32_t n;
  int32_t k;
  int32_t kstride;            // row stride of knn_idx / knn_dist
  int32_t base;               // global index of row 0
  int32_t *cand;               // [n][kExactCand] candidate ids of the scan
  uint64_t *thr;               // [n][kExactParts] smallest (measure, index) key a scan queue of each part dropped (~0: none)
  float *nmax;                 // [1] largest row norm (device)
  int32_t *head;
  int32_t *knn_idx;
  float *knn_dist;
  float *rho;
  uint64_t *rank_key;
  int32_t *fb_list;            // queries whose check failed
  int32_t *fb_count;
};
hipError_t launch_exact_mfma(int32_t dt, int S, const ExactMfmaParams &p, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
hipError_t launch_identity_perm(int32_t *p, int64_t n, hipStream_t s);
hipError_t launch_read_probe(const void *buf, int64_t bytes, int32_t passes, uint32_t key,
                             uint32_t *sink, int grid, hipStream_t s);
hipError_t launch_rev_count(const int32_t *adj, const int32_t *deg, const int32_t *items,
                            int32_t nb, int32_t R, int32_t *rcnt, int32_t *ntargets,
                            int32_t *tlist, int32_t *tidx, int32_t *ticket, hipStream_t s);
hipError_t launch_rev_alloc(const int32_t *tlist, const int32_t *ntargets, const int32_t *rcnt,
                            int32_t *toff, int32_t *tcnt, int32_t *cursor, int32_t *tord,
                            int32_t *front, int32_t *back, int32_t light, int32_t maxt,
                            hipStream_t s);
hipError_t launch_rev_scatter(const int32_t *adj, const int32_t *deg, const int32_t *items,
                              int32_t nb, int32_t R, const int32_t *tidx,
                              const int32_t *toff, const int32_t *ticket, int32_t *seg,
                              const uint64_t *akey, uint64_t *segk, hipStream_t s);
// Smallest rank key of each instance (one workgroup per instance).
hipError_t launch_min_key(const uint64_t *key, const InstTable &inst, uint64_t *out, hipStream_t s);
hipError_t launch_dep_in_knn(int64_t n, const InstTable &inst, int32_t kstride, const uint64_t *key,
                             const uint64_t *minkey, const int32_t *knn_idx, const float *knn_dist,
                             int32_t *dep, float *delta, int32_t *ulist, int32_t *ucount,
                             int32_t *ucnt_inst, hipStream_t s);
hipError_t launch_bf_dep_finalize(const int32_t *ulist, const int32_t *ucount,
                                  const unsigned long long *best, int32_t metric, int32_t *dep,
                                  float *delta, int32_t maxu, hipStream_t s);
hipError_t launch_copy_count(const int32_t *src, int32_t *dst, int32_t nmax, hipStream_t s);
hipError_t launch_cluster(int64_t n, const InstTable &inst, const float *rho, const int32_t *dep,
                          const float *delta, int32_t center_mode, float delta_min, float rho_min,
                          int32_t *labels, uint8_t *is_center, uint64_t *gkey, int32_t *flag,
                          uint32_t *sel,
                          hipStream_t s);

hipError_t launch_density(int64_t n, const InstTable &inst, int32_t kstride, int32_t fn,
                          const int32_t *knn_idx, const float *knn_dist, float *rho,
                          uint64_t *rank_key, hipStream_t s);
hipError_t launch_local_centers(int64_t n, const InstTable &inst, int32_t kstride,
                                const int32_t *knn_idx, const uint64_t *rank_key, const float *rho,
                                float rho_min, uint8_t *is_center, hipStream_t s);

// Host tables to device memory through kernel arguments (no host copy, no
// synchronisation): dst[first + j] = v[j] for j < count <= 64.
struct I64Chunk { int64_t v[64]; };
struct I32Chunk { int32_t v[64]; };
hipError_t launch_put_i64(const I64Chunk &c, int32_t count, int64_t *dst, hipStream_t s);
hipError_t launch_put_i32(const I32Chunk &c, int32_t count, int32_t *dst, hipStream_t s);

// One build round's work items from ranges of the insertion order: range j
// puts perm[pbeg[j] ..+ cnt[j]) at items[obeg[j] ..), every one with start
// points perm[sbase[j] ..+ ns[j]).
struct RangeChunk {
  int32_t pbeg[32], cnt[32], obeg[32], sbase[32], ns[32];
};
hipError_t launch_gather_items(const RangeChunk &c, int32_t nranges, int32_t maxcnt,
                               const int32_t *perm, int32_t *items, int32_t *item_sbase,
                               int32_t *item_ns, hipStream_t s);
// Appends to list every point whose instance has fewer than `below` points.
hipError_t launch_small_instance_points(int64_t n, const InstTable &inst, int32_t below,
                                        int32_t *list, int32_t *count, hipStream_t s);

}  // namespace pecann
