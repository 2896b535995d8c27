// Instantiations of the FP32 time-blocked gather with its step count fixed at
// compile time: box stencils (the other shape and FP64 compile in parallel).
#include "kernels_tb2d.hpp"

namespace stencil {

Kernel tb2d_dma_box(int R, int steps, int64_t items) { return tb2d_dma_pick<float, true>(R, steps, items); }

}  // namespace stencil
