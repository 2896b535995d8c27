// Picker of the two-step n = 4 box outer products (FP32, 2D): a launch of
// two steps takes the time-blocked kernel, a launch of one (the remainder of
// an odd run) the one-step kernel it equals bit for bit.
#include "kernels_tbm2d.hpp"
#include "plan.hpp"

namespace stencil {

template <int R>
static Kernel pick_tbm2d(KArgs& a, int32_t chunk) {
  if (a.steps <= 1) return find_mfma2d_b4(R, true, 4, 1)(a, chunk);
  if (a.steps != 2 || !dma2d_ok(a)) return Kernel{};
  int32_t ch = chunk;
  if (ch <= 0) {
    // long chunks (one level-1 block of warm-up each), as many as fill every
    // CU with resident workgroups once
    const Residency res = resident_workgroups(reinterpret_cast<const void*>(tbm2d_kernel<R>));
    const int64_t strips = (a.d1 + kTbmStride - 1) / kTbmStride;
    const int64_t slots = res.per_cu > 0 && res.cus > 0 ? (int64_t)res.per_cu * res.cus : 512;
    int64_t nch = slots / strips;
    if (nch < 1) nch = 1;
    const int64_t c = (a.d0 + nch - 1) / nch;
    ch = (int32_t)(c < (int64_t(1) << 30) ? c : (int64_t(1) << 30));
  }
  return kernel_of<tbm2d_kernel<R>, tbm2d_batch<R>>(strip_grid(a, kTbmStride, TbmShape<R>::BM, 1, ch));
}

Picker find_tbm2d(int R) {
  switch (R) {
    case 1: return pick_tbm2d<1>;
    case 2: return pick_tbm2d<2>;
    case 3: return pick_tbm2d<3>;
    case 4: return pick_tbm2d<4>;
  }
  return nullptr;
}

}  // namespace stencil
