// Instantiations of the 2D split-precision (BF16x3 / FP16x3) kernel.
#include "dma2d.hpp"
#include "kernels_split2d.hpp"
#include "plan.hpp"

namespace stencil {

template <int KIND, int R>
static hipError_t launch_split2d(const KArgs& a0, dim3, hipStream_t s) {
  KArgs a = a0;
  if (dma2d_ok(a)) {
    const dim3 grid = strip_grid(a, kSplitTN, kDmaBM);
    split2d_dma_kernel<KIND, R><<<grid, dim3(256), 0, s>>>(a);
  } else {
    const dim3 grid = strip_grid(a, 64, 64, 2048);
    split2d_kernel<KIND, R><<<grid, dim3(256), 0, s>>>(a);
  }
  return hipGetLastError();
}

template <int KIND>
static LaunchFn pick(int R) {
  switch (R) {
    case 1: return launch_split2d<KIND, 1>;
    case 2: return launch_split2d<KIND, 2>;
    case 3: return launch_split2d<KIND, 3>;
    case 4: return launch_split2d<KIND, 4>;
  }
  return nullptr;
}

LaunchFn find_split2d(int kind, int R, int /*variant*/) { return kind == 1 ? pick<1>(R) : pick<0>(R); }

}  // namespace stencil
