// Asynchronous plane windows for the 3D kernels (gfx950 direct-to-LDS).
//
// The 3D kernels walk the input planes of a chunk in the order of Algorithm 1.
// With this loader the (j, k) window of plane i+1 -- rows [j0 - r, j0 + ROWS - r),
// columns [k0 - 4, k0 + TK + 4) -- is copied straight into one of two LDS
// buffers with global_load_lds_dwordx4 while plane i is scattered into the
// accumulator ring.  Every wave issues the same number of load instructions
// per plane with all lanes active (lanes past the window, and every lane of a
// zero-halo plane outside the grid, read a 16-byte zero line), so an
// immediate "s_waitcnt vmcnt(n)" after issuing plane i+1 waits exactly for
// plane i.  Requirements (checked on the host): the k extent is a multiple of
// the 16-byte vector and both grid pointers are 16-byte aligned.
#pragma once

#include "device_common.hpp"

namespace stencil {

typedef __attribute__((address_space(3))) void lds_void3_t;

template <typename T, int R, int ROWS, int TK, int NT, int M = 4>
struct DmaPlane {
  static constexpr int VEC = 16 / (int)sizeof(T);
  static constexpr int PITCH = TK + 2 * M;       // elements per LDS row: columns k0-M .. k0+TK+M-1
  static constexpr int LPR = PITCH / VEC;        // 16-byte lines per row
  static constexpr int COL0 = M - R;             // LDS column of window column 0 (global k0 - r)
  static constexpr int LINES = ROWS * LPR;
  static constexpr int NWAVES = NT / 64;
  static constexpr int NPW = ((LINES + 63) / 64 + NWAVES - 1) / NWAVES;
  static constexpr int BUF = NPW * NWAVES * 64 * VEC;   // elements per buffer, incl. slack
  static_assert(R <= M, "window covers at most M halo columns");
  static_assert(M % VEC == 0, "16-byte lines start on a line boundary");
  static_assert(NPW < 64, "vmcnt range");

  // Per-lane source offsets (elements from the plane's start) of the lines
  // this lane loads, -1 for a zero line.  They are the same for every plane
  // of a work item, so they are computed once: window rows (global j)
  // grow0 .. grow0 + ROWS - 1, columns k0 - M .., under the boundary rule.
  struct Lines {
    int64_t off[NPW];
  };

  static __device__ __forceinline__ void prepare(Lines& L, int64_t Nj, int64_t Nk, int64_t grow0, int64_t k0,
                                                 bool periodic) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int line = (k * NWAVES + w) * 64 + lane;
      L.off[k] = -1;
      if (line < LINES) {
        const int row = line / LPR, lc = line - (line / LPR) * LPR;
        const int64_t g = map_index(grow0 + row, Nj, periodic);
        const int64_t c = map_index(k0 - M + VEC * lc, Nk, periodic);
        if (g >= 0 && c >= 0) L.off[k] = g * Nk + c;
      }
    }
  }

  // Issue the loads of one plane (nullptr: a zero-halo plane outside the grid).
  static __device__ __forceinline__ void issue(T* dst, const T* __restrict__ plane, const T* __restrict__ zeros,
                                               const Lines& L) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const T* s = (plane != nullptr && L.off[k] >= 0) ? plane + L.off[k] : zeros;
      __builtin_amdgcn_global_load_lds(s, (lds_void3_t*)(dst + (k * NWAVES + w) * 64 * VEC), 16, 0, 0);
    }
  }

  // s_waitcnt vmcnt(n) (vmcnt[3:0] bits 3:0, vmcnt[5:4] bits 15:14; expcnt and
  // lgkmcnt left at their maxima).
  template <int n>
  static __device__ __forceinline__ void wait_vm() {
    __builtin_amdgcn_s_waitcnt((n & 0xf) | ((n >> 4) << 14) | (0x7 << 4) | (0xf << 8));
  }
};

template <typename T>
inline bool dma3d_ok(const KArgs& a) {
  constexpr int VEC = 16 / (int)sizeof(T);
  return a.d2 % VEC == 0 && (reinterpret_cast<uintptr_t>(a.in) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(a.out) & 15) == 0 && a.zeros != nullptr;
}

}  // namespace stencil
