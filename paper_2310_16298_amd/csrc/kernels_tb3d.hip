// Instantiations of the time-blocked 3D gather kernel (r = 1, two steps).
#include <type_traits>

#include "kernels_tb3d.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, bool BOX>
static Kernel pick_tb3d(KArgs& a, int32_t chunk) {
  const int dtype = std::is_same<T, double>::value ? STENCIL_F64 : STENCIL_F32;
  // a launch of one step (the remainder of a run): the one-step gather
  if (a.steps <= 1) return find_gather3d(dtype, 1, BOX)(a, chunk);
  if (!tb3d_ok(a) || a.steps != 2) return Kernel{};
  int64_t ti, tj, tk;
  tb3d_tiles<T, 1, 2>(a.d0, a.d1, a.d2, &ti, &tj, &tk);
  return kernel_of<tb3d_dma_kernel<T, 1, BOX, 2>, tb3d_dma_batch<T, 1, BOX, 2>>(ti * tj * tk);
}

Picker find_tb3d(int dtype, int R, bool box) {
  if (R != 1) return nullptr;
  if (dtype == STENCIL_F64) return box ? pick_tb3d<double, true> : pick_tb3d<double, false>;
  return box ? pick_tb3d<float, true> : pick_tb3d<float, false>;
}

}  // namespace stencil
