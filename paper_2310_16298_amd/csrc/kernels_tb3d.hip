// Instantiations of the time-blocked 3D gather kernels (two steps per launch):
// the streaming form for stars of order 1 (FP32 up to 4) and the 27-point box
// on planes of at least 32 (j, k) tiles, the whole-window form for order 1
// otherwise.
#include <type_traits>

#include "kernels_tb3d.hpp"
#include "plan.hpp"

namespace stencil {

// MANY: the grid is one of many in a batched launch.  The whole-window form
// recomputes a halo of every window to give a small grid alone enough
// workgroups; among many grids, whose items fill the chip anyway, that work
// only costs (MI355X, FP64 batches of 8^3 to 64^3 grids, order 1: 1.3-3.2x
// behind the one-step gather), so such grids get no two-step kernel there.
template <typename T, int R, bool BOX, bool MANY = false>
static Kernel pick_tb3d(KArgs& a, int32_t chunk) {
  const int dtype = std::is_same<T, double>::value ? STENCIL_F64 : STENCIL_F32;
  // a launch of one step (the remainder of a run): the one-step gather
  if (a.steps <= 1) return find_gather3d(dtype, R, BOX)(a, chunk);
  if (!tb3d_ok(a) || a.steps != 2) return Kernel{};
  // the streaming form wants planes of at least 32 (j, k) tiles: fewer
  // leave its chunks too shallow for their 4r warm-up planes (measured on
  // MI355X: 128^3 and 64^3 lose to the whole-window form at order 1)
  // The 5- and 6-wave workgroups of the FP32 stars of order 1-2 run at most
  // two per CU: with a third resident on some CUs (576 items of 72 tiles at
  // 384^3) those CUs set the launch time (MI355X: 573 GStencil/s at 384^3
  // against 1056 at 512^3, where 512 items fill every CU with two).
  typedef Tb3Stream<T, R, BOX> S;
  if (R >= 2 || tb3d_plane_tiles(a) >= 32)
    return kernel3d<tb3d_stream_kernel<T, R, BOX>, tb3d_stream_batch<T, R, BOX>, S::NT>(a, R, chunk,
                                                                                        S::SPREAD ? 2 : 0);
  if constexpr (R == 1 && !MANY) {
    int64_t ti, tj, tk;
    tb3d_tiles<T, R, 2>(a.d0, a.d1, a.d2, &ti, &tj, &tk);
    return kernel_of<tb3d_dma_kernel<T, R, BOX, 2>, tb3d_dma_batch<T, R, BOX, 2>>(ti * tj * tk);
  }
  return Kernel{};
}

bool tb3d_built(int dtype, int R, bool box) {
  return R == 1 || (dtype == STENCIL_F32 && R <= 4 && !box);
}

template <bool MANY>
static Picker find(int dtype, int R, bool box) {
  if (!tb3d_built(dtype, R, box)) return nullptr;
  if (dtype == STENCIL_F64) return box ? pick_tb3d<double, 1, true, MANY> : pick_tb3d<double, 1, false, MANY>;
  if (R == 2) return pick_tb3d<float, 2, false, MANY>;
  if (R == 3) return pick_tb3d<float, 3, false, MANY>;
  if (R == 4) return pick_tb3d<float, 4, false, MANY>;
  return box ? pick_tb3d<float, 1, true, MANY> : pick_tb3d<float, 1, false, MANY>;
}

Picker find_tb3d(int dtype, int R, bool box) { return find<false>(dtype, R, box); }
Picker find_tb3d_batch(int dtype, int R, bool box) { return find<true>(dtype, R, box); }

}  // namespace stencil
