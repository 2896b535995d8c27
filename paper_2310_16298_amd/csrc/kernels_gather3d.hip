// Dispatch for the 3D gather-form baseline kernels; the instantiations live
// in kernels_gather3d_f32.hip and kernels_gather3d_f64.hip (compiled apart).
#include "plan.hpp"

namespace stencil {

Picker find_gather3d_f32(int R, bool box);
Picker find_gather3d_f64(int R, bool box);

Picker find_gather3d(int dtype, int R, bool box) {
  return dtype == STENCIL_F64 ? find_gather3d_f64(R, box) : find_gather3d_f32(R, box);
}

}  // namespace stencil
