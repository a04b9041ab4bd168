// K2 greedy beam search with the candidates scored on the matrix cores
// (mfma_score.hpp): BF16, FP8 and MXFP6 search rows.
#include "search_impl.hpp"

namespace pecann {

template <int DT, int S>
static hipError_t launch_search_mf(const SearchParams &p, int grid, hipStream_t st) {
  return launch_search_t<DT, S, true>(p, grid, st);
}

hipError_t launch_search_mfma(int32_t dt, int S, const SearchParams &p, int grid, hipStream_t st) {
  switch (dt) {
    case PECANN_BF16: PECANN_SHAPES(launch_search_mf, PECANN_BF16, S, p, grid, st)
    case PECANN_FP8E4M3: PECANN_SHAPES(launch_search_mf, PECANN_FP8E4M3, S, p, grid, st)
    case PECANN_MXFP6: PECANN_SHAPES(launch_search_mf, PECANN_MXFP6, S, p, grid, st)
    default: return hipErrorInvalidValue;
  }
}

PECANN_CHECK_READER(search_mfma)

}  // namespace pecann
