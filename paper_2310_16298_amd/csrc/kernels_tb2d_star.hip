// Instantiations of the FP32 time-blocked gather with its step count fixed at
// compile time: star stencils (the other shape and FP64 compile in parallel).
#include "kernels_tb2d.hpp"

namespace stencil {

Kernel tb2d_dma_star(int R, int steps, int64_t items) { return tb2d_dma_pick<float, false>(R, steps, items); }

}  // namespace stencil
