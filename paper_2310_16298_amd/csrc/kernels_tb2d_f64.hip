// Instantiations of the FP64 time-blocked gather with its step count fixed at
// compile time, stars and boxes, on 32-row tiles and (grids of fewer tiles
// than CUs) 16-row tiles.
#include "kernels_tb2d.hpp"

namespace stencil {

Kernel tb2d_dma_f64(bool box, int R, int steps, int64_t items, bool small_tiles) {
  if (small_tiles)
    return box ? tb2d_dma_pick<double, true, kTbSmallRows>(R, steps, items)
               : tb2d_dma_pick<double, false, kTbSmallRows>(R, steps, items);
  return box ? tb2d_dma_pick<double, true>(R, steps, items) : tb2d_dma_pick<double, false>(R, steps, items);
}

}  // namespace stencil
