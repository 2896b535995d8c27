// Instantiations of the 3D gather-form baseline kernel, double grids.
#include "kernels_3d.hpp"
#include "plan.hpp"

namespace stencil {

template <int R, bool BOX>
static hipError_t launch_gather3d(const KArgs& a, dim3 grid, hipStream_t s) {
  if (dma3d_ok<double>(a))
    gather3d_kernel<double, R, BOX, true><<<grid, dim3(kThreads), 0, s>>>(a);
  else
    gather3d_kernel<double, R, BOX, false><<<grid, dim3(kThreads), 0, s>>>(a);
  return hipGetLastError();
}

template <bool BOX>
static LaunchFn pick(int R) {
  switch (R) {
    case 1: return launch_gather3d<1, BOX>;
    case 2: return launch_gather3d<2, BOX>;
    case 3: return launch_gather3d<3, BOX>;
    case 4: return launch_gather3d<4, BOX>;
  }
  return nullptr;
}

LaunchFn find_gather3d_f64(int R, bool box) { return box ? pick<true>(R) : pick<false>(R); }

}  // namespace stencil
