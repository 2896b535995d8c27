// Instantiations of the 2D box outer products on n = 4 blocks with register
// tiles of 8 / 16 / 32 rows per wave and workgroup tiles of 256 / 128 columns
// (the default 16 rows x 256 columns is in kernels_mfma2d.hip).
#include "dma2d.hpp"
#include "kernels_2d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <int R, int UI, int WR>
static Kernel pick_tiles(KArgs& a, int32_t chunk) {
  constexpr int TN = 256 / WR, BM = 4 * UI * WR;
  if (dma2d_ok(a))
    return kernel_of<mfma2d_b4_dma_kernel<R, true, UI, WR>, mfma2d_b4_dma_batch<R, true, UI, WR>>(
        strip_grid(a, TN, BM, 1024, dma_chunk(a, TN, R, 1, chunk)));
  return kernel_of<mfma2d_b4_kernel<R, true>, mfma2d_b4_batch<R, true>>(strip_grid(a, kTile2D, kTile2D, 2048, chunk));
}

template <int UI, int WR>
static Picker pick_r(int R) {
  switch (R) {
    case 1: return pick_tiles<1, UI, WR>;
    case 2: return pick_tiles<2, UI, WR>;
    case 3: return pick_tiles<3, UI, WR>;
    case 4: return pick_tiles<4, UI, WR>;
  }
  return nullptr;
}

Picker find_mfma2d_b4_tiles(int R, int ui, int wr) {
  if (wr == 1) {
    if (ui == 2) return pick_r<2, 1>(R);
    if (ui == 8) return pick_r<8, 1>(R);
  } else if (wr == 2) {
    if (ui == 2) return pick_r<2, 2>(R);
    if (ui == 4) return pick_r<4, 2>(R);
    if (ui == 8) return pick_r<8, 2>(R);
  }
  return nullptr;
}

}  // namespace stencil
