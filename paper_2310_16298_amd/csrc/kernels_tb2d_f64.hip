// Instantiations of the FP64 time-blocked gather with its step count fixed at
// compile time, stars and boxes.
#include "kernels_tb2d.hpp"

namespace stencil {

Kernel tb2d_dma_f64(bool box, int R, int steps, int64_t items) {
  return box ? tb2d_dma_pick<double, true>(R, steps, items) : tb2d_dma_pick<double, false>(R, steps, items);
}

}  // namespace stencil
