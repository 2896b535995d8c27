// Instantiations of the 3D gather-form baseline kernel.
#include "kernels_3d.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, bool BOX>
static hipError_t launch_gather3d(const KArgs& a, dim3 grid, hipStream_t s) {
  gather3d_kernel<T, R, BOX><<<grid, dim3(kThreads), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, bool BOX>
static LaunchFn pick(int R) {
  switch (R) {
    case 1: return launch_gather3d<T, 1, BOX>;
    case 2: return launch_gather3d<T, 2, BOX>;
    case 3: return launch_gather3d<T, 3, BOX>;
    case 4: return launch_gather3d<T, 4, BOX>;
  }
  return nullptr;
}

LaunchFn find_gather3d(int dtype, int R, bool box) {
  if (dtype == STENCIL_F64) return box ? pick<double, true>(R) : pick<double, false>(R);
  return box ? pick<float, true>(R) : pick<float, false>(R);
}

}  // namespace stencil
