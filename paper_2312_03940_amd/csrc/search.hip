// K2 greedy beam search: the vector-unit scoring variant of every row format,
// and the dispatch between it and the matrix-core variant (search_mfma.hip).
#include <algorithm>

#include "search_impl.hpp"

namespace pecann {

size_t search_lds_bytes(int L, int hbits, int hid_bits) {
  const size_t Lp = (size_t)((L + 15) & ~15);
  return 8 * (2 * (size_t)L + 64) + 4 * 64 + 2 * Lp + (hid_bits ? 2 : 4) * ((size_t)1 << hbits);
}

int compact_hash_bits(int64_t n, int hbits) {
  int kb = 1;
  while (((int64_t)1 << kb) < n) ++kb;
  kb = std::max(kb, hbits - 2);
  return kb - (hbits - 2) <= 13 ? kb : 0;
}

template <int DT, int S>
static hipError_t launch_search_vec(const SearchParams &p, int grid, hipStream_t st) {
  return launch_search_t<DT, S, false>(p, grid, st);
}

hipError_t launch_search(int32_t dt, int S, const SearchParams &p, int grid, hipStream_t st) {
  if (dt == PECANN_MXFP6 || (p.mfma && (dt == PECANN_BF16 || dt == PECANN_FP8E4M3)))
    return launch_search_mfma(dt, S, p, grid, st);
  PECANN_DISPATCH_SHAPE(launch_search_vec, dt, S, p, grid, st)
}

PECANN_CHECK_READER(search)

}  // namespace pecann
