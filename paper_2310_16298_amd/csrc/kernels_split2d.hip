// Instantiations of the 2D split-precision (BF16x3 / FP16x3) kernel.
#include "dma2d.hpp"
#include "kernels_split2d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <int KIND, int R>
static Kernel pick_split2d(KArgs& a, int32_t chunk) {
  if (dma2d_ok(a)) return kernel_of<split2d_dma_kernel<KIND, R>, split2d_dma_batch<KIND, R>>(strip_grid(a, kSplitTN, kDmaBM, 1024, dma_chunk(a, kSplitTN, R, 2, chunk)));
  return kernel_of<split2d_kernel<KIND, R>, split2d_batch<KIND, R>>(strip_grid(a, 64, 64, 2048, chunk));
}

template <int KIND>
static Picker pick(int R) {
  switch (R) {
    case 1: return pick_split2d<KIND, 1>;
    case 2: return pick_split2d<KIND, 2>;
    case 3: return pick_split2d<KIND, 3>;
    case 4: return pick_split2d<KIND, 4>;
  }
  return nullptr;
}

Picker find_split2d(int kind, int R, int /*variant*/) { return kind == 1 ? pick<1>(R) : pick<0>(R); }

}  // namespace stencil
