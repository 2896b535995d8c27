// Instantiations of the 3D split-precision kernels.  Box: r = 1 (27 points).
#include "kernels_3d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <int KIND, int R, bool BOX>
static Kernel pick_split3d(KArgs& a, int32_t) {
  const int64_t items = chunk3d_items(a);
  if (dma3d_ok<float>(a)) return kernel_of<split3d_kernel<KIND, R, BOX, true>, split3d_batch<KIND, R, BOX, true>>(items);
  return kernel_of<split3d_kernel<KIND, R, BOX, false>, split3d_batch<KIND, R, BOX, false>>(items);
}

template <int KIND>
static Picker pick(int R, bool box) {
  if (box) return R == 1 ? pick_split3d<KIND, 1, true> : nullptr;
  switch (R) {
    case 1: return pick_split3d<KIND, 1, false>;
    case 2: return pick_split3d<KIND, 2, false>;
    case 3: return pick_split3d<KIND, 3, false>;
    case 4: return pick_split3d<KIND, 4, false>;
  }
  return nullptr;
}

Picker find_split3d(int kind, int R, bool box) { return kind == 1 ? pick<1>(R, box) : pick<0>(R, box); }

}  // namespace stencil
