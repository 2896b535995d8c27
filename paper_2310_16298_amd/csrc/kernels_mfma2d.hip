// Instantiations of the 2D outer-product kernel (FP32 / FP64 MFMA).
#include "kernels_2d.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, int VAR>
static hipError_t launch_mfma2d(const KArgs& a, dim3 grid, hipStream_t s) {
  mfma2d_kernel<T, R, VAR><<<grid, dim3(kThreads), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int VAR>
static LaunchFn pick(int R) {
  switch (R) {
    case 1: return launch_mfma2d<T, 1, VAR>;
    case 2: return launch_mfma2d<T, 2, VAR>;
    case 3: return launch_mfma2d<T, 3, VAR>;
    case 4: return launch_mfma2d<T, 4, VAR>;
  }
  return nullptr;
}

template <typename T>
static LaunchFn pick_var(int R, int var) {
  switch (var) {
    case VAR_BOX: return pick<T, VAR_BOX>(R);
    case VAR_STAR_PARALLEL: return pick<T, VAR_STAR_PARALLEL>(R);
    case VAR_STAR_ORTHO: return pick<T, VAR_STAR_ORTHO>(R);
  }
  return nullptr;
}

LaunchFn find_mfma2d(int dtype, int R, int variant) {
  return dtype == STENCIL_F64 ? pick_var<double>(R, variant) : pick_var<float>(R, variant);
}

}  // namespace stencil
