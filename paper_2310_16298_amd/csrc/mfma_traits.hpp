// Matrix-core (MFMA) operations used by the outer-product kernels, with the
// gfx950 lane layouts of their operands (each checked against host matrix
// products on an MI355X).
//
// v_mfma_*_16x16x4 (f32, f64): D[16x16] += A[16x4] * B[4x16].  One MFMA is
// four rank-1 updates a_k (x) b_k accumulated into the same 16x16 block,
// i.e. four of the outer products of Eq. (12) at once.
//   A: lane l holds A[l % 16][l / 16]
//   B: lane l holds B[l / 16][l % 16]
// v_mfma_f32_16x16x32_{bf16,f16}: 32 rank-1 updates per instruction.
//   A: lane l, element e holds A[l % 16][8 (l / 16) + e]
//   B: lane l, element e holds B[8 (l / 16) + e][l % 16]
// D: lane l, register v holds D[row(l, v)][col(l)] with col(l) = l % 16 and
//   row(l, v) = 4 (l / 16) + v  for the FP32-accumulating instructions,
//   row(l, v) = 4 v + l / 16    for v_mfma_f64_16x16x4.
#pragma once

#include "device_common.hpp"

namespace stencil {

template <typename T> struct Mfma16;

template <> struct Mfma16<float> {
  typedef floatx4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ int col(int lane) { return lane & 15; }
};

template <> struct Mfma16<double> {
  typedef doublex4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
  static __device__ __forceinline__ int col(int lane) { return lane & 15; }
};

}  // namespace stencil
