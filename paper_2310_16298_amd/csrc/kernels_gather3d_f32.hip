// Instantiations of the 3D gather-form baseline kernel, float grids.
#include "kernels_3d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <int R, bool BOX>
static Kernel pick_gather3d(KArgs& a, int32_t chunk) {
  const Kernel whole = whole3d_kernel<float, R, BOX>(a, chunk);  // small grids
  if (whole.launch) return whole;
  if (dma3d_ok<float>(a)) return kernel3d<gather3d_kernel<float, R, BOX, true>, gather3d_batch<float, R, BOX, true>>(a, R, chunk);
  return kernel3d<gather3d_kernel<float, R, BOX, false>, gather3d_batch<float, R, BOX, false>>(a, R, chunk);
}

template <bool BOX>
static Picker pick(int R) {
  switch (R) {
    case 1: return pick_gather3d<1, BOX>;
    case 2: return pick_gather3d<2, BOX>;
    case 3: return pick_gather3d<3, BOX>;
    case 4: return pick_gather3d<4, BOX>;
  }
  return nullptr;
}

Picker find_gather3d_f32(int R, bool box) { return box ? pick<true>(R) : pick<false>(R); }

}  // namespace stencil
