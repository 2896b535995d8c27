// Instantiations of the 2D gather-form baseline kernel.
#include "dma2d.hpp"
#include "kernels_2d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, bool BOX>
static Kernel pick_gather2d(KArgs& a, int32_t chunk) {
  constexpr int TN = Gather2DDma<T>::TN;
  // FP32 grids at most one 64-column tile wide: the 64 x 64 tiled kernel
  // (a 256-column window would leave three quarters of its lanes idle)
  if (dma2d_ok(a) && !(sizeof(T) == 4 && a.d1 <= kTile2D))
    return kernel_of<gather2d_dma_kernel<T, R, BOX>, gather2d_dma_batch<T, R, BOX>>(
        strip_grid(a, TN, kDmaBM, 1024, dma_chunk(a, TN, R, BOX, chunk)));
  return kernel_of<gather2d_kernel<T, R, BOX>, gather2d_batch<T, R, BOX>>(strip_grid(a, kTile2D, kTile2D, 2048, chunk));
}

template <typename T, bool BOX>
static Picker pick(int R) {
  switch (R) {
    case 1: return pick_gather2d<T, 1, BOX>;
    case 2: return pick_gather2d<T, 2, BOX>;
    case 3: return pick_gather2d<T, 3, BOX>;
    case 4: return pick_gather2d<T, 4, BOX>;
  }
  return nullptr;
}

Picker find_gather2d(int dtype, int R, bool box) {
  if (dtype == STENCIL_F64) return box ? pick<double, true>(R) : pick<double, false>(R);
  return box ? pick<float, true>(R) : pick<float, false>(R);
}

}  // namespace stencil
