// Instantiations of the 3D outer-product kernels (FP32 / FP64 MFMA).
// Box: r <= 2 (the band fragments of all (2r+1)^2 lines stay in VGPRs).
#include "kernels_3d.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, bool BOX>
static hipError_t launch_mfma3d(const KArgs& a, dim3 grid, hipStream_t s) {
  if (dma3d_ok<T>(a))
    mfma3d_kernel<T, R, BOX, true><<<grid, dim3(kThreads), 0, s>>>(a);
  else
    mfma3d_kernel<T, R, BOX, false><<<grid, dim3(kThreads), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T>
static LaunchFn pick(int R, bool box) {
  if (box) {
    switch (R) {
      case 1: return launch_mfma3d<T, 1, true>;
      case 2: return launch_mfma3d<T, 2, true>;
    }
    return nullptr;
  }
  switch (R) {
    case 1: return launch_mfma3d<T, 1, false>;
    case 2: return launch_mfma3d<T, 2, false>;
    case 3: return launch_mfma3d<T, 3, false>;
    case 4: return launch_mfma3d<T, 4, false>;
  }
  return nullptr;
}

LaunchFn find_mfma3d(int dtype, int R, bool box) {
  return dtype == STENCIL_F64 ? pick<double>(R, box) : pick<float>(R, box);
}

}  // namespace stencil
