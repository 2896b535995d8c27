// Instantiations of the 2D gather-form baseline kernel.
#include "dma2d.hpp"
#include "kernels_2d.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, bool BOX>
static hipError_t launch_gather2d(const KArgs& a0, dim3, hipStream_t s) {
  KArgs a = a0;
  if constexpr (sizeof(T) == 4) {
    if (dma2d_ok(a)) {
      const dim3 grid = strip_grid(a, kDmaTN, kDmaBM);
      gather2d_dma_kernel<R, BOX><<<grid, dim3(kThreads), 0, s>>>(a);
      return hipGetLastError();
    }
  }
  const dim3 grid = strip_grid(a, kTile2D, kTile2D, 2048);
  gather2d_kernel<T, R, BOX><<<grid, dim3(kThreads), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, bool BOX>
static LaunchFn pick(int R) {
  switch (R) {
    case 1: return launch_gather2d<T, 1, BOX>;
    case 2: return launch_gather2d<T, 2, BOX>;
    case 3: return launch_gather2d<T, 3, BOX>;
    case 4: return launch_gather2d<T, 4, BOX>;
  }
  return nullptr;
}

LaunchFn find_gather2d(int dtype, int R, bool box) {
  if (dtype == STENCIL_F64) return box ? pick<double, true>(R) : pick<double, false>(R);
  return box ? pick<float, true>(R) : pick<float, false>(R);
}

}  // namespace stencil
