// Instantiations of the 3D split-precision kernels.  Boxes r = 1..4; stars:
// parallel (k lines on MFMA) and hybrid (j and k lines) covers.
#include "kernels_3d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <int KIND, int R, bool BOX>
static Kernel pick_split3d(KArgs& a, int32_t chunk) {
  if (dma3d_ok<float>(a)) return kernel3d<split3d_kernel<KIND, R, BOX, true>, split3d_batch<KIND, R, BOX, true>>(a, R, chunk);
  return kernel3d<split3d_kernel<KIND, R, BOX, false>, split3d_batch<KIND, R, BOX, false>>(a, R, chunk);
}

// Stars in the hybrid cover: the lines along j and k on MFMA, the i arm on VALU
template <int KIND, int R>
static Kernel pick_split3d_hybrid(KArgs& a, int32_t chunk) {
  if (dma3d_ok<float>(a))
    return kernel3d<split3d_hybrid_kernel<KIND, R, true>, split3d_hybrid_batch<KIND, R, true>>(a, R, chunk);
  return kernel3d<split3d_hybrid_kernel<KIND, R, false>, split3d_hybrid_batch<KIND, R, false>>(a, R, chunk);
}

template <int KIND>
static Picker pick(int R, bool box, bool hybrid) {
  if (box) {
    switch (R) {
      case 1: return pick_split3d<KIND, 1, true>;
      case 2: return pick_split3d<KIND, 2, true>;
      case 3: return pick_split3d<KIND, 3, true>;
      case 4: return pick_split3d<KIND, 4, true>;
    }
    return nullptr;
  }
  if (hybrid) {
    switch (R) {
      case 1: return pick_split3d_hybrid<KIND, 1>;
      case 2: return pick_split3d_hybrid<KIND, 2>;
      case 3: return pick_split3d_hybrid<KIND, 3>;
      case 4: return pick_split3d_hybrid<KIND, 4>;
    }
    return nullptr;
  }
  switch (R) {
    case 1: return pick_split3d<KIND, 1, false>;
    case 2: return pick_split3d<KIND, 2, false>;
    case 3: return pick_split3d<KIND, 3, false>;
    case 4: return pick_split3d<KIND, 4, false>;
  }
  return nullptr;
}

Picker find_split3d(int kind, int R, bool box, bool hybrid) {
  return kind == 1 ? pick<1>(R, box, hybrid) : pick<0>(R, box, hybrid);
}

}  // namespace stencil
