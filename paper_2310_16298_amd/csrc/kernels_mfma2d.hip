// Instantiations of the 2D outer-product kernels (FP32 / FP64 MFMA).
#include "dma2d.hpp"
#include "kernels_2d.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace stencil {

template <typename T, int R, int VAR>
static Kernel pick_mfma2d(KArgs& a, int32_t chunk) {
  return kernel_of<mfma2d_kernel<T, R, VAR>, mfma2d_batch<T, R, VAR>>(strip_grid(a, kTile2D, kTile2D, 2048, chunk));
}

template <typename T, int VAR>
static Picker pick(int R) {
  switch (R) {
    case 1: return pick_mfma2d<T, 1, VAR>;
    case 2: return pick_mfma2d<T, 2, VAR>;
    case 3: return pick_mfma2d<T, 3, VAR>;
    case 4: return pick_mfma2d<T, 4, VAR>;
  }
  return nullptr;
}

template <typename T>
static Picker pick_var(int R, int var) {
  switch (var) {
    case VAR_BOX: return pick<T, VAR_BOX>(R);
    case VAR_STAR_PARALLEL: return pick<T, VAR_STAR_PARALLEL>(R);
    case VAR_STAR_ORTHO: return pick<T, VAR_STAR_ORTHO>(R);
    case VAR_COVER: return pick<T, VAR_COVER>(R);
  }
  return nullptr;
}

template <int R, bool BOX>
static Kernel pick_b4(KArgs& a, int32_t chunk) {
  if (dma2d_ok(a)) return kernel_of<mfma2d_b4_dma_kernel<R, BOX>, mfma2d_b4_dma_batch<R, BOX>>(strip_grid(a, kDmaTN, kDmaBM, 1024, dma_chunk(a, kDmaTN, R, BOX, chunk)));
  return kernel_of<mfma2d_b4_kernel<R, BOX>, mfma2d_b4_batch<R, BOX>>(strip_grid(a, kTile2D, kTile2D, 2048, chunk));
}

template <bool BOX>
static Picker pick_b4r(int R) {
  switch (R) {
    case 1: return pick_b4<1, BOX>;
    case 2: return pick_b4<2, BOX>;
    case 3: return pick_b4<3, BOX>;
    case 4: return pick_b4<4, BOX>;
  }
  return nullptr;
}

Picker find_mfma2d_b4(int R, bool box, int ui, int wr) {
  if (box && (ui != 4 || wr != 1)) return find_mfma2d_b4_tiles(R, ui, wr);
  return box ? pick_b4r<true>(R) : pick_b4r<false>(R);
}

// Line cover on n = 4 blocks; grids the direct-to-LDS kernels cannot take use
// the 16x16 cover kernel, whose fragments follow the n = 4 ones in the buffer.
template <int R>
static Kernel pick_b4c(KArgs& a, int32_t chunk) {
  if (dma2d_ok(a))
    return kernel_of<mfma2d_b4c_dma_kernel<R>, mfma2d_b4c_dma_batch<R>>(
        strip_grid(a, kDmaTN, kDmaBM, 1024, dma_chunk(a, kDmaTN, R, true, chunk)));
  a.frag = static_cast<const char*>(a.frag) + cover_b4_frag_bytes(R);
  return kernel_of<mfma2d_kernel<float, R, VAR_COVER>, mfma2d_batch<float, R, VAR_COVER>>(
      strip_grid(a, kTile2D, kTile2D, 2048, chunk));
}

Picker find_mfma2d_b4c(int R) {
  switch (R) {
    case 1: return pick_b4c<1>;
    case 2: return pick_b4c<2>;
    case 3: return pick_b4c<3>;
    case 4: return pick_b4c<4>;
  }
  return nullptr;
}

Picker find_mfma2d(int dtype, int R, int variant) {
  return dtype == STENCIL_F64 ? pick_var<double>(R, variant) : pick_var<float>(R, variant);
}

}  // namespace stencil
