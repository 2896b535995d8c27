// Instantiations of the 3D outer-product kernels (FP32 / FP64 MFMA).
// Box: r <= 2 (the band fragments of all (2r+1)^2 lines stay in VGPRs).
#include "kernels_3d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, bool BOX>
static Kernel pick_mfma3d(KArgs& a, int32_t chunk) {
  if (dma3d_ok<T>(a)) return kernel3d<mfma3d_kernel<T, R, BOX, true>, mfma3d_batch<T, R, BOX, true>>(a, R, chunk);
  return kernel3d<mfma3d_kernel<T, R, BOX, false>, mfma3d_batch<T, R, BOX, false>>(a, R, chunk);
}

template <typename T>
static Picker pick(int R, bool box) {
  if (box) {
    switch (R) {
      case 1: return pick_mfma3d<T, 1, true>;
      case 2: return pick_mfma3d<T, 2, true>;
    }
    return nullptr;
  }
  switch (R) {
    case 1: return pick_mfma3d<T, 1, false>;
    case 2: return pick_mfma3d<T, 2, false>;
    case 3: return pick_mfma3d<T, 3, false>;
    case 4: return pick_mfma3d<T, 4, false>;
  }
  return nullptr;
}

// n = 4 blocks (FP32): stars r = 1..4 and the 27-point box
template <int R, bool BOX>
static Kernel pick_mfma3d_b4(KArgs& a, int32_t chunk) {
  if (dma3d_ok<float>(a)) return kernel3d<mfma3d_b4_kernel<R, BOX, true>, mfma3d_b4_batch<R, BOX, true>>(a, R, chunk);
  return kernel3d<mfma3d_b4_kernel<R, BOX, false>, mfma3d_b4_batch<R, BOX, false>>(a, R, chunk);
}

template <int R>
static Kernel pick_mfma3d_b4box(KArgs& a, int32_t chunk) {
  if (dma3d_ok<float>(a)) return kernel3d<mfma3d_b4box_kernel<R, true>, mfma3d_b4box_batch<R, true>>(a, R, chunk);
  return kernel3d<mfma3d_b4box_kernel<R, false>, mfma3d_b4box_batch<R, false>>(a, R, chunk);
}

Picker find_mfma3d_b4(int R, bool box) {
  if (box) {
    switch (R) {
      case 1: return pick_mfma3d_b4<1, true>;
      case 2: return pick_mfma3d_b4box<2>;
      case 3: return pick_mfma3d_b4box<3>;
      case 4: return pick_mfma3d_b4box<4>;
    }
    return nullptr;
  }
  switch (R) {
    case 1: return pick_mfma3d_b4<1, false>;
    case 2: return pick_mfma3d_b4<2, false>;
    case 3: return pick_mfma3d_b4<3, false>;
    case 4: return pick_mfma3d_b4<4, false>;
  }
  return nullptr;
}

Picker find_mfma3d(int dtype, int R, bool box) {
  return dtype == STENCIL_F64 ? pick<double>(R, box) : pick<float>(R, box);
}

}  // namespace stencil
