// Instantiations of the time-blocked 2D gather kernels.
#include <type_traits>

#include "kernels_tb2d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

// MANY: the grid is one of many in a batched launch, whose items fill the
// chip without the small-grid tiles below
template <typename T, int R, bool BOX, bool MANY = false>
static Kernel pick_tb2d(KArgs& a, int32_t chunk) {
  // a launch of one step (the remainder of a run): the one-step gather
  if (a.steps <= 1) return find_gather2d(std::is_same<T, double>::value ? STENCIL_F64 : STENCIL_F32, R, BOX)(a, chunk);
  if (tb2d_fast<T>(a) && a.zeros != nullptr) {
    int TM = tb2d_dma_rows<T>();
    a.tiles1 = (int32_t)((a.d1 + 63) / 64);
    // FP64 grids of fewer tiles than CUs (launch-bound: 512^2 has 128) take
    // 16-row tiles, twice the workgroups at the cost of more halo rows
    // (MI355X, 512^2 FP64 five-point star, 8 steps per launch: see below);
    // not in a batch, where their halo rows cost without the occupancy gain
    const bool small =
        !MANY && !std::is_same<T, float>::value && (int64_t)((a.d0 + TM - 1) / TM) * a.tiles1 < 256;
    if (small) TM = kTbSmallRows;
    a.tiles0 = (int32_t)((a.d0 + TM - 1) / TM);
    const int64_t items = (int64_t)a.tiles0 * a.tiles1;
    Kernel k;
    if constexpr (std::is_same<T, float>::value) k = BOX ? tb2d_dma_box(R, a.steps, items) : tb2d_dma_star(R, a.steps, items);
    else k = tb2d_dma_f64(BOX, R, a.steps, items, small);
    if (k.launch) return k;
  }
  const int64_t items = tb2d_items<T>(a);
  if (tb2d_fast<T>(a)) return kernel_of<tb2d_kernel<T, R, BOX, true>, tb2d_batch<T, R, BOX, true>>(items);
  return kernel_of<tb2d_kernel<T, R, BOX, false>, tb2d_batch<T, R, BOX, false>>(items);
}

template <typename T, bool BOX, bool MANY>
static Picker pick(int R) {
  switch (R) {
    case 1: return pick_tb2d<T, 1, BOX, MANY>;
    case 2: return pick_tb2d<T, 2, BOX, MANY>;
    case 3: return pick_tb2d<T, 3, BOX, MANY>;
    case 4: return pick_tb2d<T, 4, BOX, MANY>;
  }
  return nullptr;
}

template <bool MANY>
static Picker find(int dtype, int R, bool box) {
  if (dtype == STENCIL_F64) return box ? pick<double, true, MANY>(R) : pick<double, false, MANY>(R);
  return box ? pick<float, true, MANY>(R) : pick<float, false, MANY>(R);
}

Picker find_tb2d(int dtype, int R, bool box) { return find<false>(dtype, R, box); }
Picker find_tb2d_batch(int dtype, int R, bool box) { return find<true>(dtype, R, box); }

int tb2d_max_steps(int dtype, int R) {
  const int hmax = dtype == STENCIL_F64 ? TbShape<double>::HMAX : TbShape<float>::HMAX;
  int t = 1;
  while (tb_halo(R, t + 1) <= hmax) ++t;
  return t;
}

}  // namespace stencil
