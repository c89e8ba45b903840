// Tile-pass kernels for complex128 states: adjoint passes over phi and lambda
// (single circuit and batched).
#include "k_tile.h"

namespace qsv {

template hipError_t launch_tile_v<double, true>(hipStream_t, bool, const void*, void*, void*, const TileArgs&,
                                             const TOp*, const void*, const uint64_t*, double*, int, int, int, size_t);
template hipError_t launch_tile_batch_v<double, true>(hipStream_t, bool, const TileEntry*, const int32_t*,
                                                   const TileArgs*, const TOp*, const void*, const uint64_t*,
                                                   double*, int, int, int, size_t);

}  // namespace qsv
