// Gather-form kernel over the nonzero weights of a GENERAL 3D stencil (the 3D
// counterpart of kernels_sparse2d.hip: weights that no line carries go to
// the vector units, Section 3.5).
//
// Plane order as in the other 3D kernels (Algorithm 1): a workgroup owns a
// 32 x 64 (j, k) tile and a chunk of output planes, walks the input planes
// once and scatters each into the ring of 2r+1 output planes it reaches.  The
// plan lists the nonzero taps grouped by coefficient plane a (layout in
// plan.hpp); the loop over a is unrolled, so every tap of plane a adds into
// the compile-time ring slot 2r - a, and the taps of one plane are walked
// with readlane from registers (lane t % 64 holds tap t; at most 128 taps).
// Wave w owns j rows 8 w .. 8 w + 7 and lane l the k column l, so each LDS
// read of a tap is 64 consecutive elements of one window row.
#include "kernels_3d.hpp"
#include "launch.hpp"
#include "plan.hpp"
#include "sparse_common.hpp"

namespace stencil {

template <typename T, int R, bool DMA>
__device__ __forceinline__ void sparse3d_item(const KArgs& a, int item) {
  constexpr int W = 2 * R + 1, PR = kTJ / 4;
  static_assert(kThreads == 256 && kTK == 64 && kSparse3DTapMax == 128, "one k column per lane, two tap registers");
  typedef PlaneWalk<T, R, kTJ + 2 * R, DMA, true> PW;
  static_assert(PW::COL0 + R == 4, "tile body at LDS column 4");
  __shared__ __attribute__((aligned(16))) T bufs[PW::NBUF * PW::BUF];

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  T* __restrict__ out = (T*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

  const int32_t* __restrict__ tab = (const int32_t*)a.frag;
  const T* __restrict__ wts = (const T*)((const char*)a.frag + kSparse3DWeightOffset);
  const int nt = __builtin_amdgcn_readfirstlane(tab[0]);
  int start[W + 1];
#pragma unroll
  for (int p = 0; p <= W; ++p) start[p] = __builtin_amdgcn_readfirstlane(tab[1 + p]);
  int code[2];
  T cf[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = 64 * h + lane;
    code[h] = t < nt ? tab[kSparse3DCodeIndex + t] : 0;
    cf[h] = t < nt ? wts[t] : T(0);
  }

  T ring[W][PR];
#pragma unroll
  for (int z = 0; z < W; ++z)
#pragma unroll
    for (int p = 0; p < PR; ++p) ring[z][p] = T(0);

  PW::walk(
      bufs, a, ch,
      [&](const T* win, bool valid) {
        if (!valid) return;  // a zero-halo plane adds nothing
        // output (j row PR w + p, k column l), tap (b, c) of plane a: window
        // row PR w + p + b, LDS column 4 - r + l + c
        const T* base = win + PR * w * PW::PITCH + (4 - R) + lane;
        // ACC: each plane's taps sum into acc, added to its ring slot once, so
        // the tap loop carries no slot index (the compiler otherwise merges
        // the plane loops and picks the slot per tap); FP64 at r >= 3 keeps
        // the direct form, whose smaller register set measured faster there
        constexpr bool ACC = sizeof(T) == 4 || R <= 2;
#pragma unroll
        for (int ap = 0; ap < W; ++ap) {
          const int t0 = start[ap], t1 = start[ap + 1];
          if constexpr (!ACC) {
            for (int t = t0; t < t1; ++t) {
              const int c = __builtin_amdgcn_readlane(t < 64 ? code[0] : code[1], t & 63);
              const T f = lane_value(t < 64 ? cf[0] : cf[1], t & 63);
              const T* p0 = base + (c >> 8) * PW::PITCH + (c & 255);
#pragma unroll
              for (int p = 0; p < PR; ++p) ring[2 * R - ap][p] += f * p0[p * PW::PITCH];
            }
            continue;
          }
          if (t0 == t1) continue;
          T acc[PR];
#pragma unroll
          for (int p = 0; p < PR; ++p) acc[p] = T(0);
          // two taps per step: all 2 PR reads issue before the first FMA
          int t = t0;
          for (; t + 1 < t1; t += 2) {
            const int c0 = __builtin_amdgcn_readlane(t < 64 ? code[0] : code[1], t & 63);
            const int c1 = __builtin_amdgcn_readlane(t + 1 < 64 ? code[0] : code[1], (t + 1) & 63);
            const T f0 = lane_value(t < 64 ? cf[0] : cf[1], t & 63);
            const T f1 = lane_value(t + 1 < 64 ? cf[0] : cf[1], (t + 1) & 63);
            const T* p0 = base + (c0 >> 8) * PW::PITCH + (c0 & 255);
            const T* p1 = base + (c1 >> 8) * PW::PITCH + (c1 & 255);
            T v0[PR], v1[PR];
#pragma unroll
            for (int p = 0; p < PR; ++p) v0[p] = p0[p * PW::PITCH];
#pragma unroll
            for (int p = 0; p < PR; ++p) v1[p] = p1[p * PW::PITCH];
#pragma unroll
            for (int p = 0; p < PR; ++p) acc[p] += f0 * v0[p];
#pragma unroll
            for (int p = 0; p < PR; ++p) acc[p] += f1 * v1[p];
          }
          if (t < t1) {
            const int c = __builtin_amdgcn_readlane(t < 64 ? code[0] : code[1], t & 63);
            const T f = lane_value(t < 64 ? cf[0] : cf[1], t & 63);
            const T* p0 = base + (c >> 8) * PW::PITCH + (c & 255);
#pragma unroll
            for (int p = 0; p < PR; ++p) acc[p] += f * p0[p * PW::PITCH];
          }
#pragma unroll
          for (int p = 0; p < PR; ++p) ring[2 * R - ap][p] += acc[p];
        }
      },
      [&](int64_t o, bool live) {
        const int64_t gk = ch.k0 + lane;
        if (live && gk < Nk) {
#pragma unroll
          for (int p = 0; p < PR; ++p) {
            const int64_t gj = ch.j0 + PR * w + p;
            if (gj < Nj) out[o * plane + gj * Nk + gk] = ring[0][p];
          }
        }
#pragma unroll
        for (int z = 0; z < 2 * R; ++z)
#pragma unroll
          for (int p = 0; p < PR; ++p) ring[z][p] = ring[z + 1][p];
#pragma unroll
        for (int p = 0; p < PR; ++p) ring[2 * R][p] = T(0);
      });
}

template <typename T, int R, bool DMA>
__global__ __launch_bounds__(kThreads) void sparse3d_kernel(KArgs a) {
  sparse3d_item<T, R, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool DMA>
__global__ __launch_bounds__(kThreads) void sparse3d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { sparse3d_item<T, R, DMA>(x, id); });
}

template <typename T, int R>
static Kernel pick_sparse3d(KArgs& a, int32_t) {
  const int64_t items = chunk3d_items(a);
  if (dma3d_ok<T>(a)) return kernel_of<sparse3d_kernel<T, R, true>, sparse3d_batch<T, R, true>>(items);
  return kernel_of<sparse3d_kernel<T, R, false>, sparse3d_batch<T, R, false>>(items);
}

template <typename T>
static Picker pick_sparse(int R) {
  switch (R) {
    case 1: return pick_sparse3d<T, 1>;
    case 2: return pick_sparse3d<T, 2>;
    case 3: return pick_sparse3d<T, 3>;
    case 4: return pick_sparse3d<T, 4>;
  }
  return nullptr;
}

Picker find_sparse3d(int dtype, int R) {
  return dtype == STENCIL_F64 ? pick_sparse<double>(R) : pick_sparse<float>(R);
}

}  // namespace stencil
