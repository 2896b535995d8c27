// Asynchronous window loads for the FP32 2D kernels (gfx950 direct-to-LDS).
//
// A workgroup walks a strip of TN columns in blocks of BM rows.  The input
// window of a block -- rows [ib - r, ib + BM + r), columns [j0 - 4, j0 + TN + 4)
// -- is copied from global memory straight into LDS with
// global_load_lds_dwordx4 (16 bytes per lane, 1 KiB per wave instruction, no
// registers), into one of two buffers, while the previous block is computed
// from the other buffer.  Wide strips keep every row segment a workgroup
// reads long and contiguous (TN = 256: 1 KiB), which HBM serves far better
// than short scattered segments.
//
// Every wave issues exactly NPW load instructions per window with all lanes
// active (lanes past the window end read a 16-byte zero line into slack at the
// end of the buffer), so "s_waitcnt vmcnt(NPW)" right after issuing window b+1
// guarantees that this wave's loads of window b (and its older stores) have
// completed; a barrier then makes all waves' loads visible.
//
// Requirements (checked on the host before choosing these kernels): the
// column extent is a multiple of 4 and the grid pointer is 16-byte aligned, so
// every 16-byte line lies entirely inside or outside the grid.  Lines outside
// the grid come from the zero line (zero halo) or wrap (periodic).
#pragma once

#include "device_common.hpp"
#include "kernels_split2d.hpp"
#include "stream2d.hpp"

namespace stencil {

typedef __attribute__((address_space(3))) void lds_void_t;

template <int R, int BM, int TN, int NT>
struct DmaWindow {
  static constexpr int RAD = R;
  static constexpr int PITCH = TN + 8;          // floats per LDS row: columns j0-4 .. j0+TN+3
  static constexpr int LPR = PITCH / 4;         // 16-byte lines per row
  static constexpr int WCOL0 = 4 - R;           // LDS column of window column 0 (global j0 - r)
  static constexpr int ROWS = BM + 2 * R;
  static constexpr int LINES = ROWS * LPR;
  static constexpr int NWAVES = NT / 64;
  static constexpr int NI = (LINES + 63) / 64;              // wave instructions per window
  static constexpr int NPW = (NI + NWAVES - 1) / NWAVES;    // per wave
  static constexpr int BUF = NPW * NWAVES * 64 * 4;          // floats per buffer, incl. slack
  static_assert(R <= 4, "window covers at most 4 halo columns");
  static_assert(NPW < 64, "vmcnt range");

  // Issue the loads of window rows grow0 .. grow0 + ROWS - 1 into `buf`.
  static __device__ __forceinline__ void issue(float* buf, const float* __restrict__ src,
                                               const float* __restrict__ zeros, int64_t M, int64_t N,
                                               int64_t grow0, int64_t j0, bool periodic) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int inst = k * NWAVES + w;
      const int line = inst * 64 + lane;
      const float* s = zeros;
      if (line < LINES) {
        const int row = line / LPR, lc = line - (line / LPR) * LPR;
        const int64_t g = map_index(grow0 + row, M, periodic);
        const int64_t c = map_index(j0 - 4 + 4 * lc, N, periodic);
        if (g >= 0 && c >= 0) s = src + g * N + c;
      }
      __builtin_amdgcn_global_load_lds(s, (lds_void_t*)(buf + inst * 256), 16, 0, 0);
    }
  }

  // Wait until this wave's loads issued before its latest NPW load
  // instructions have landed (wait_all: every load).
  static __device__ __forceinline__ void wait_previous() {
    // s_waitcnt vmcnt(NPW): vmcnt[3:0] in bits 3:0, vmcnt[5:4] in bits 15:14;
    // expcnt (bits 6:4) and lgkmcnt (bits 11:8) left at their maxima.
    __builtin_amdgcn_s_waitcnt((NPW & 0xf) | ((NPW >> 4) << 14) | (0x7 << 4) | (0xf << 8));
  }
  static __device__ __forceinline__ void wait_all() { __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xf << 8)); }
};

// Host-side condition for the direct-to-LDS kernels.
inline bool dma2d_ok(const KArgs& a) {
  return a.d1 % 4 == 0 && (reinterpret_cast<uintptr_t>(a.in) & 15) == 0 && a.zeros != nullptr;
}

// Block loop shared by the DMA kernels: body(cur, ib) computes and stores the
// block of rows [ib, min(ib + BM, i1)) from the window in `cur`.
template <class D, int BM, class Body>
__device__ __forceinline__ void dma_block_loop(float* bufs, const KArgs& a, const Strip2D& sp, Body body) {
  const float* __restrict__ in = (const float*)a.in;
  const float* __restrict__ zeros = (const float*)a.zeros;
  const bool periodic = a.periodic != 0;
  const int nb = (int)((sp.i1 - sp.i0 + BM - 1) / BM);
  D::issue(bufs, in, zeros, a.d0, a.d1, sp.i0 - D::RAD, sp.j0, periodic);
  for (int bi = 0; bi < nb; ++bi) {
    const int64_t ib = sp.i0 + (int64_t)bi * BM;
    if (bi + 1 < nb) {
      D::issue(bufs + ((bi + 1) & 1) * D::BUF, in, zeros, a.d0, a.d1, ib + BM - D::RAD, sp.j0, periodic);
      D::wait_previous();
    } else {
      D::wait_all();
    }
    __syncthreads();
    body(bufs + (bi & 1) * D::BUF, ib);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// n = 4 block outer products (see mfma2d_b4_kernel) on DMA-fed windows:
// 256-column strips, 16-row blocks; wave w owns columns 64 w .. 64 w + 63.
// ---------------------------------------------------------------------------
constexpr int kDmaTN = 256, kDmaBM = 16;

template <int R, bool BOX>
__global__ __launch_bounds__(256) void mfma2d_b4_dma_kernel(KArgs a) {
  constexpr int BM = kDmaBM, TN = kDmaTN, NB = 4 + 2 * R, NL = BOX ? 2 * R + 1 : 1;
  typedef DmaWindow<R, BM, TN, 256> D;
  __shared__ __attribute__((aligned(16))) float bufs[2 * D::BUF];

  const int64_t N = a.d1;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const Strip2D sp = decode_strip(a, TN);

  const float* __restrict__ frag = (const float*)a.frag;
  float af[NL * NB];
#pragma unroll
  for (int c = 0; c < NL * NB; ++c) af[c] = frag[c * 64 + lane];
  float cw[2 * R + 1];
  if constexpr (!BOX) {
    const float* __restrict__ c = (const float*)a.coef;
#pragma unroll
    for (int b = 0; b <= 2 * R; ++b) cw[b] = c[R * (2 * R + 1) + b];
  }
  const int64_t gj = sp.j0 + 64 * w + lane;

  dma_block_loop<D, BM>(bufs, a, sp, [&](const float* cur, int64_t ib) {
    const float* rowp = cur + D::WCOL0 + 64 * w + lane;
    floatx4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = floatx4{0, 0, 0, 0};
#pragma unroll
    for (int li = 0; li < NL; ++li) {
      const int b = BOX ? li : R;
#pragma unroll
      for (int x = 0; x < 16 + 2 * R; ++x) {
        const float bv = rowp[x * D::PITCH + b];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int d = x - 4 * s;
          if (d < 0 || d >= NB) continue;
          acc[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(af[li * NB + d], bv, acc[s], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // keep each line's LDS reads next to its MFMAs
    }
    if constexpr (!BOX) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float* rp = rowp + (4 * s + v + R) * D::PITCH;
          float sum = 0.0f;
#pragma unroll
          for (int b = 0; b <= 2 * R; ++b) {
            if (b == R) continue;
            sum += cw[b] * rp[b];
          }
          acc[s][v] += sum;
        }
    }
    if (gj < N) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gi = ib + 4 * s + v;
          if (gi < sp.i1) out[gi * N + gj] = acc[s][v];
        }
    }
  });
}

// ---------------------------------------------------------------------------
// Gather-form baseline on DMA-fed windows: thread t owns column t of the
// 256-column strip and the 16 rows of each block (register window down the
// column, wave-uniform coefficients).
// ---------------------------------------------------------------------------
template <int R, bool BOX>
__global__ __launch_bounds__(256) void gather2d_dma_kernel(KArgs a) {
  constexpr int BM = kDmaBM, TN = kDmaTN, W = 2 * R + 1;
  typedef DmaWindow<R, BM, TN, 256> D;
  __shared__ __attribute__((aligned(16))) float bufs[2 * D::BUF];

  const int64_t N = a.d1;
  float* __restrict__ out = (float*)a.out;
  const float* __restrict__ c = (const float*)a.coef;
  const int t = threadIdx.x;
  const Strip2D sp = decode_strip(a, TN);
  const int64_t gj = sp.j0 + t;

  dma_block_loop<D, BM>(bufs, a, sp, [&](const float* cur, int64_t ib) {
    const float* base = cur + D::WCOL0 + t;
    float acc[BM];
#pragma unroll
    for (int p = 0; p < BM; ++p) acc[p] = 0.0f;
#pragma unroll
    for (int x = 0; x < BM + 2 * R; ++x) {
      float h[W];
#pragma unroll
      for (int b = 0; b < W; ++b) h[b] = base[x * D::PITCH + b];
#pragma unroll
      for (int p = 0; p < BM; ++p) {
        const int aa = x - p;
        if (aa < 0 || aa > 2 * R) continue;
#pragma unroll
        for (int b = 0; b < W; ++b) {
          if (!BOX && aa != R && b != R) continue;
          acc[p] += c[aa * W + b] * h[b];
        }
      }
    }
    if (gj < N) {
#pragma unroll
      for (int p = 0; p < BM; ++p) {
        const int64_t gi = ib + p;
        if (gi < sp.i1) out[gi * N + gj] = acc[p];
      }
    }
  });
}

// ---------------------------------------------------------------------------
// Split-precision outer products (see split2d_kernel) on DMA-fed FP32
// windows: 128-column strips, 16-row blocks, wave w owns columns
// 32 w .. 32 w + 31 (two 16 x 16 output blocks).  After a window lands, one
// pass splits it into the hi/lo 16-bit LDS planes read by the 16x16x32 MFMAs.
// ---------------------------------------------------------------------------
constexpr int kSplitTN = 128;

template <int KIND, int R>
__global__ __launch_bounds__(256) void split2d_dma_kernel(KArgs a) {
  constexpr int NL = 2 * R + 1, BM = kDmaBM, TN = kSplitTN;
  constexpr int WROWS = BM + 2 * R, WEND = TN + 2 * R;
  constexpr int P = 152;  // 16-bit pitch: multiple of 8, odd number of 16-byte units, >= 96 + 16 + 32
  static_assert(WEND <= P && 32 * 3 + 16 + 32 <= P, "pitch too small");
  typedef DmaWindow<R, BM, TN, 256> D;
  __shared__ __attribute__((aligned(16))) float bufs[2 * D::BUF];
  __shared__ __attribute__((aligned(16))) uint16_t lhi[WROWS * P];
  __shared__ __attribute__((aligned(16))) uint16_t llo[WROWS * P];

  const int64_t N = a.d1;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, q = lane & 15;
  const Strip2D sp = decode_strip(a, TN);

  const u16x8* __restrict__ frag = (const u16x8*)a.frag;
  u16x8 bh[NL], bl[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    bh[l] = frag[(l * 2 + 0) * 64 + lane];
    bl[l] = frag[(l * 2 + 1) * 64 + lane];
  }
  zero_region<uint16_t, 256>(lhi, WROWS, P - WEND, P, 0, WEND);
  zero_region<uint16_t, 256>(llo, WROWS, P - WEND, P, 0, WEND);
  const float lo_mul = 1.0f / a.lo_scale;
  const float ls = a.lo_scale, os = a.out_scale;

  dma_block_loop<D, BM>(bufs, a, sp, [&](const float* cur, int64_t ib) {
    // split the window into hi/lo planes, two columns per thread and step
    constexpr int HALF = WEND / 2;
    for (int idx = threadIdx.x; idx < WROWS * HALF; idx += 256) {
      const int row = idx / HALF, y = 2 * (idx - (idx / HALF) * HALF);
      const float* src = cur + row * D::PITCH + D::WCOL0 + y;
      uint16_t h0, l0, h1, l1;
      Split16<KIND>::split(src[0], lo_mul, h0, l0);
      Split16<KIND>::split(src[1], lo_mul, h1, l1);
      *reinterpret_cast<uint32_t*>(lhi + row * P + y) = (uint32_t)h0 | ((uint32_t)h1 << 16);
      *reinterpret_cast<uint32_t*>(llo + row * P + y) = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    __syncthreads();
    floatx4 acc[2], acx[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      acc[t] = floatx4{0, 0, 0, 0};
      acx[t] = floatx4{0, 0, 0, 0};
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const uint16_t* ph = lhi + (l + q) * P + 32 * w + 8 * g;
      const uint16_t* pl = llo + (l + q) * P + 32 * w + 8 * g;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const u16x8 ah = *reinterpret_cast<const u16x8*>(ph + 16 * t);
        const u16x8 al = *reinterpret_cast<const u16x8*>(pl + 16 * t);
        acc[t] = Split16<KIND>::mma(ah, bh[l], acc[t]);
        acx[t] = Split16<KIND>::mma(ah, bl[l], acx[t]);
        acx[t] = Split16<KIND>::mma(al, bh[l], acx[t]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = ib + 4 * g + v;
      if (gi >= sp.i1) continue;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int64_t gj = sp.j0 + 32 * w + 16 * t + q;
        if (gj < N) out[gi * N + gj] = (acc[t][v] + ls * acx[t][v]) * os;
      }
    }
  });
}

}  // namespace stencil
