// 2D outer-product form with 16-bit split operands (BF16 or FP16 hi/lo) on
// v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulation and FP32 grids.
//
// Every operand x is split as x = hi + lo (+ a residual of order 2^-16 |x| for
// BF16, 2^-22 |x| for FP16), hi = RN16(x), lo = RN16(x - hi); the product of
// two split values is formed from three MFMAs, hi*hi + hi*lo + lo*hi, dropping
// lo*lo.  For FP16 the lo parts are stored multiplied by 2^11 (keeping them in
// the normal range) and the coefficients by a power of two chosen by the plan;
// both scales are exact and undone in the epilogue.  Integer data below 2^16
// (BF16) or 65504 (FP16) are represented exactly, so integer stencils whose
// partial sums stay below 2^24 are reproduced bit for bit.
//
// Lines run along j (C^g row a, the row coefficient line of Eq. (14)), in the
// form D[p][q] += sum_y H[p + a][y] * S_a[y][q], S_a[y][q] = C^g[a][y - q]:
// the MFMA A operand is eight consecutive 16-bit input values of one LDS row
// (one 16-byte read), the B operand is the band S_a, kept in registers.  With
// K = 32 >= 16 + 2r each line is one instruction per part.  Star stencils use
// the same cover with their zero weights (Section 3.3).
#pragma once

#include "device_common.hpp"
#include "stream2d.hpp"

namespace stencil {

template <int KIND> struct Split16;  // 0 = bf16, 1 = f16
template <> struct Split16<0> {
  static __device__ __forceinline__ void split(float x, float /*lo_mul*/, uint16_t& hi, uint16_t& lo) {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  }
  static __device__ __forceinline__ floatx4 mma(u16x8 a, u16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
};
template <> struct Split16<1> {
  static __device__ __forceinline__ void split(float x, float lo_mul, uint16_t& hi, uint16_t& lo) {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)((x - (float)h) * lo_mul);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  }
  static __device__ __forceinline__ floatx4 mma(u16x8 a, u16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, a),
                                                  __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
  }
};

// Stage a ROWS x (BODY + 2R) FP32 window, split into hi/lo 16-bit planes.
// Window element (row, y) goes to hi[row * P + y], lo[row * P + y].
template <int KIND, int R, int ROWS, int BODY, int P, int NT>
__device__ __forceinline__ void stage_split(uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                            const float* __restrict__ src, int64_t M, int64_t N,
                                            int64_t r0, int64_t c0, bool periodic, float lo_mul) {
  constexpr int NV = BODY / 4;
  constexpr int WCOLS = BODY + 2 * R;
  const int tid = threadIdx.x;
  const bool fast = (c0 + BODY <= N) && (N % 4 == 0) && ((reinterpret_cast<uintptr_t>(src) & 15) == 0);
  if (fast) {
    for (int idx = tid; idx < ROWS * NV; idx += NT) {
      const int row = idx / NV;
      const int v = idx - row * NV;
      const int64_t g = map_index(r0 + row, M, periodic);
      float4 val = g >= 0 ? *reinterpret_cast<const float4*>(src + g * N + c0 + 4 * v) : float4{0, 0, 0, 0};
      const int base = row * P + R + 4 * v;
      const float xs[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) Split16<KIND>::split(xs[e], lo_mul, hi[base + e], lo[base + e]);
    }
    for (int idx = tid; idx < ROWS * 2 * R; idx += NT) {
      const int row = idx / (2 * R);
      const int h = idx - row * (2 * R);
      const int64_t gc = (h < R) ? (c0 - R + h) : (c0 + BODY + (h - R));
      const int y = (h < R) ? h : (BODY + h);
      const int64_t g = map_index(r0 + row, M, periodic);
      const int64_t c = map_index(gc, N, periodic);
      const float x = (g >= 0 && c >= 0) ? src[g * N + c] : 0.0f;
      Split16<KIND>::split(x, lo_mul, hi[row * P + y], lo[row * P + y]);
    }
  } else {
    for (int idx = tid; idx < ROWS * WCOLS; idx += NT) {
      const int row = idx / WCOLS;
      const int y = idx - row * WCOLS;
      const int64_t g = map_index(r0 + row, M, periodic);
      const int64_t c = map_index(c0 - R + y, N, periodic);
      const float x = (g >= 0 && c >= 0) ? src[g * N + c] : 0.0f;
      Split16<KIND>::split(x, lo_mul, hi[row * P + y], lo[row * P + y]);
    }
  }
}

template <int R>
struct Split2DShape {
  static constexpr int TM = 64, TN = 64;
  static constexpr int WROWS = TM + 2 * R;
  static constexpr int WEND = TN + 2 * R;       // window columns
  static constexpr int LCOLS = (TN - 16) + 32;  // columns read by the padded K = 32
  static constexpr int P = 88;                  // pitch in 16-bit elements (multiple of 8)
  static_assert(LCOLS <= P && WEND <= P, "pitch too small");
};

// Writer splitting FP32 window values into the hi/lo 16-bit LDS planes.
template <int KIND, int P>
struct SplitWriter {
  uint16_t* hi;
  uint16_t* lo;
  float lo_mul;
  __device__ __forceinline__ void put(int row, int y, float x) {
    Split16<KIND>::split(x, lo_mul, hi[row * P + y], lo[row * P + y]);
  }
  __device__ __forceinline__ void put_vec(int row, int y, const float4& v) {
    const float xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) put(row, y + e, xs[e]);
  }
};

template <int KIND, int R>
__device__ __forceinline__ void split2d_item(const KArgs& a, int item) {
  typedef Split2DShape<R> S;
  constexpr int NL = 2 * R + 1, BM = S::TM;
  __shared__ __attribute__((aligned(16))) uint16_t lhi[S::WROWS * S::P];
  __shared__ __attribute__((aligned(16))) uint16_t llo[S::WROWS * S::P];

  const int64_t M = a.d0, N = a.d1;
  const bool periodic = a.periodic != 0;
  const float* __restrict__ in = (const float*)a.in;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, q = lane & 15;
  const Strip2D sp = decode_strip(a, item, S::TN);
  const bool fast = strip_fast(in, N, sp.j0, S::TN);

  // Band fragments S_a (hi, lo) for this lane: 16 bytes each.
  const u16x8* __restrict__ frag = (const u16x8*)a.frag;
  u16x8 bh[NL], bl[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    bh[l] = frag[(l * 2 + 0) * 64 + lane];
    bl[l] = frag[(l * 2 + 1) * 64 + lane];
  }

  zero_region<uint16_t, 256>(lhi, S::WROWS, S::P - S::WEND, S::P, 0, S::WEND);
  zero_region<uint16_t, 256>(llo, S::WROWS, S::P - S::WEND, S::P, 0, S::WEND);
  const float lo_mul = 1.0f / a.lo_scale;
  stage_split<KIND, R, S::WROWS, S::TN, S::P, 256>(lhi, llo, in, M, N, sp.i0 - R, sp.j0, periodic, lo_mul);
  __syncthreads();

  SplitWriter<KIND, S::P> wr{lhi, llo, lo_mul};
  RowPrefetch<float, R, BM, S::TN, 256> pf;
  RowMover<uint16_t, R, S::WEND, 256> mvh, mvl;
  const float ls = a.lo_scale, os = a.out_scale;
  for (int64_t ib = sp.i0; ib < sp.i1; ib += BM) {
    const bool more = ib + BM < sp.i1;
    if (more) pf.fetch(in, M, N, ib + BM + R, sp.j0, periodic, fast);
    floatx4 acc[4], acx[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = floatx4{0, 0, 0, 0};
      acx[t] = floatx4{0, 0, 0, 0};
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const uint16_t* ph = lhi + (16 * w + l + q) * S::P + 8 * g;
      const uint16_t* pl = llo + (16 * w + l + q) * S::P + 8 * g;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const u16x8 ah = *reinterpret_cast<const u16x8*>(ph + 16 * t);
        const u16x8 al = *reinterpret_cast<const u16x8*>(pl + 16 * t);
        acc[t] = Split16<KIND>::mma(ah, bh[l], acc[t]);
        acx[t] = Split16<KIND>::mma(ah, bl[l], acx[t]);
        acx[t] = Split16<KIND>::mma(al, bh[l], acx[t]);
      }
    }
    const int64_t gj = sp.j0 + q;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = ib + 16 * w + 4 * g + v;
      if (gi >= sp.i1) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (gj + 16 * t < N) out[gi * N + gj + 16 * t] = (acc[t][v] + ls * acx[t][v]) * os;
      }
    }
    if (more) {
      mvh.load([&](int rr, int cc) { return lhi[(BM + rr) * S::P + cc]; });
      mvl.load([&](int rr, int cc) { return llo[(BM + rr) * S::P + cc]; });
    }
    __syncthreads();
    if (more) {
      mvh.store([&](int rr, int cc, uint16_t v) { lhi[rr * S::P + cc] = v; });
      mvl.store([&](int rr, int cc, uint16_t v) { llo[rr * S::P + cc] = v; });
      pf.commit(2 * R, wr);
    }
    __syncthreads();
  }
}

template <int KIND, int R>
__global__ __launch_bounds__(256) void split2d_kernel(KArgs a) {
  split2d_item<KIND, R>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int KIND, int R>
__global__ __launch_bounds__(256) void split2d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { split2d_item<KIND, R>(x, id); });
}

}  // namespace stencil
