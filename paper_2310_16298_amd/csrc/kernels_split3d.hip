// Instantiations of the 3D split-precision kernels.  Box: r = 1 (27 points).
#include "kernels_3d.hpp"
#include "plan.hpp"

namespace stencil {

template <int KIND, int R, bool BOX>
static hipError_t launch_split3d(const KArgs& a, dim3 grid, hipStream_t s) {
  if (dma3d_ok<float>(a))
    split3d_kernel<KIND, R, BOX, true><<<grid, dim3(kThreads), 0, s>>>(a);
  else
    split3d_kernel<KIND, R, BOX, false><<<grid, dim3(kThreads), 0, s>>>(a);
  return hipGetLastError();
}

template <int KIND>
static LaunchFn pick(int R, bool box) {
  if (box) return R == 1 ? launch_split3d<KIND, 1, true> : nullptr;
  switch (R) {
    case 1: return launch_split3d<KIND, 1, false>;
    case 2: return launch_split3d<KIND, 2, false>;
    case 3: return launch_split3d<KIND, 3, false>;
    case 4: return launch_split3d<KIND, 4, false>;
  }
  return nullptr;
}

LaunchFn find_split3d(int kind, int R, bool box) { return kind == 1 ? pick<1>(R, box) : pick<0>(R, box); }

}  // namespace stencil
