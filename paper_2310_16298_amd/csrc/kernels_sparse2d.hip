// Gather-form kernel over the nonzero weights of a GENERAL 2D stencil.
//
// Section 3.5 covers the nonzero weights of C^g with lines and leaves weights
// that no row or column line reaches cheaply (diagonals, scattered points) to
// the vector units.  This kernel is that vector form: its cost follows the
// number of nonzero taps n, not the (2r+1)^2 of the full box.
//
// The plan lists the taps in the fragment buffer (layout in plan.hpp): the
// count, one code per tap (row a << 8 | column b, 0 <= a, b <= 2r) and the
// weights in the arithmetic dtype.  Lane t % 64 of every wave keeps tap t in
// registers; each step of the tap loop takes one tap with readlane, so the
// loop waits on nothing but its own LDS reads.
//
// Direct-to-LDS windows as in the other 2D DMA kernels (256 threads, 16-row
// blocks, TN-column strips).  Wave w owns rows 4 w .. 4 w + 3 of each block
// and lane l the columns l + 64 q, so every LDS read is 64 consecutive
// elements of one window row: no bank conflicts at any tap offset.
#include "dma2d.hpp"
#include "kernels_2d.hpp"
#include "launch.hpp"
#include "plan.hpp"
#include "sparse_common.hpp"

namespace stencil {

template <typename T, int R>
__device__ __forceinline__ void sparse2d_dma_item(const KArgs& a, int item) {
  constexpr int BM = kDmaBM, TN = Gather2DDma<T>::TN, CPT = TN / 64, PR = BM / 4;
  static_assert(kSparseTapMax <= 128 && (2 * R + 1) * (2 * R + 1) <= kSparseTapMax, "taps fit two registers");
  typedef DmaWindow<T, R, BM, TN, 256> D;
  __shared__ __attribute__((aligned(16))) T bufs[2 * D::BUF];

  const int64_t N = a.d1;
  T* __restrict__ out = (T*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const Strip2D sp = decode_strip(a, item, TN);

  const int32_t* __restrict__ tab = (const int32_t*)a.frag;
  const T* __restrict__ wts = (const T*)((const char*)a.frag + kSparseWeightOffset);
  const int nt = __builtin_amdgcn_readfirstlane(tab[0]);
  int code[2];
  T cf[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = 64 * h + lane;
    code[h] = t < nt ? tab[1 + t] : 0;
    cf[h] = t < nt ? wts[t] : T(0);
  }
  const int n0 = nt < 64 ? nt : 64;

  dma_block_loop<D, BM>(bufs, a, sp, [&](const T* cur, int64_t ib) {
    T acc[PR][CPT];
#pragma unroll
    for (int p = 0; p < PR; ++p)
#pragma unroll
      for (int q = 0; q < CPT; ++q) acc[p][q] = T(0);
    // output row 4 w + p, column l + 64 q takes window row 4 w + p + a and
    // LDS column WCOL0 + l + 64 q + b for tap (a, b)
    const T* base = cur + PR * w * D::PITCH + D::WCOL0 + lane;
    auto tap = [&](int c, T f) {
      const T* p0 = base + (c >> 8) * D::PITCH + (c & 255);
#pragma unroll
      for (int p = 0; p < PR; ++p)
#pragma unroll
        for (int q = 0; q < CPT; ++q) acc[p][q] += f * p0[p * D::PITCH + 64 * q];
    };
#pragma unroll 2
    for (int t = 0; t < n0; ++t) tap(__builtin_amdgcn_readlane(code[0], t), lane_value(cf[0], t));
    for (int t = 64; t < nt; ++t) tap(__builtin_amdgcn_readlane(code[1], t - 64), lane_value(cf[1], t - 64));
#pragma unroll
    for (int p = 0; p < PR; ++p) {
      const int64_t gi = ib + PR * w + p;
      if (gi >= sp.i1) continue;
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int64_t gj = sp.j0 + lane + 64 * q;
        if (gj < N) out[gi * N + gj] = acc[p][q];
      }
    }
  });
}

template <typename T, int R>
__global__ __launch_bounds__(256) void sparse2d_dma_kernel(KArgs a) {
  sparse2d_dma_item<T, R>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R>
__global__ __launch_bounds__(256) void sparse2d_dma_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { sparse2d_dma_item<T, R>(x, id); });
}

// Grids without direct-to-LDS windows (column count not a multiple of 4,
// unaligned buffers) and FP32 grids one 64-column tile wide take the tiled
// gather kernel over every tap of the box (the dense C^g, zeros included).
template <typename T, int R>
static Kernel pick_sparse2d(KArgs& a, int32_t chunk) {
  constexpr int TN = Gather2DDma<T>::TN;
  if (dma2d_ok(a) && !(sizeof(T) == 4 && a.d1 <= kTile2D))
    return kernel_of<sparse2d_dma_kernel<T, R>, sparse2d_dma_batch<T, R>>(
        strip_grid(a, TN, kDmaBM, 1024, dma_chunk(a, TN, R, 0, chunk)));
  return kernel_of<gather2d_kernel<T, R, true>, gather2d_batch<T, R, true>>(strip_grid(a, kTile2D, kTile2D, 2048, chunk));
}

template <typename T>
static Picker pick_sparse(int R) {
  switch (R) {
    case 1: return pick_sparse2d<T, 1>;
    case 2: return pick_sparse2d<T, 2>;
    case 3: return pick_sparse2d<T, 3>;
    case 4: return pick_sparse2d<T, 4>;
  }
  return nullptr;
}

Picker find_sparse2d(int dtype, int R) {
  return dtype == STENCIL_F64 ? pick_sparse<double>(R) : pick_sparse<float>(R);
}

}  // namespace stencil
