// Instantiations of the 2D outer-product kernel (FP32 / FP64 MFMA).
#include "dma2d.hpp"
#include "kernels_2d.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, int VAR>
static hipError_t launch_mfma2d(const KArgs& a0, dim3, hipStream_t s) {
  KArgs a = a0;
  const dim3 grid = strip_grid(a, kTile2D, kTile2D, 2048);
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

template <int R, bool BOX>
static hipError_t launch_b4(const KArgs& a0, dim3, hipStream_t s) {
  KArgs a = a0;
  if (dma2d_ok(a)) {
    const dim3 grid = strip_grid(a, kDmaTN, kDmaBM);
    mfma2d_b4_dma_kernel<R, BOX><<<grid, dim3(kThreads), 0, s>>>(a);
  } else {
    const dim3 grid = strip_grid(a, kTile2D, kTile2D, 2048);
    mfma2d_b4_kernel<R, BOX><<<grid, dim3(kThreads), 0, s>>>(a);
  }
  return hipGetLastError();
}

template <bool BOX>
static LaunchFn pick_b4(int R) {
  switch (R) {
    case 1: return launch_b4<1, BOX>;
    case 2: return launch_b4<2, BOX>;
    case 3: return launch_b4<3, BOX>;
    case 4: return launch_b4<4, BOX>;
  }
  return nullptr;
}

LaunchFn find_mfma2d_b4(int R, bool box) { return box ? pick_b4<true>(R) : pick_b4<false>(R); }

LaunchFn find_mfma2d(int dtype, int R, int variant) {
  return dtype == STENCIL_F64 ? pick_var<double>(R, variant) : pick_var<float>(R, variant);
}

}  // namespace stencil
