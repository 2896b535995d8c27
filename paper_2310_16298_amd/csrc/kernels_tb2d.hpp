// Time-blocked 2D gather kernel: T Jacobi steps per launch (the temporal
// reuse the paper leaves to future work, Section 6).
//
// A workgroup owns a TM x TN output tile.  It stages the tile's window with a
// halo of HW = round_up(r T, 4) on every side into LDS once, then applies T
// steps between two LDS buffers and stores the tile: HBM traffic per
// point-step falls about T-fold.  Step s (1-based) computes the shrinking
// region of window points at least r s from the window edge, which depends
// only on the region of step s-1; the tile lies HW >= r T inside the edge.  Zero halo: window points outside the
// grid are 0 at load and reset to 0 after every step; periodic: the window
// is the periodic extension of the grid, so no reset is needed.
//
// LDS layout: window element (x, y) at buf[x * P + 4 + y] (16-byte aligned
// body); each thread computes 2 x 4 blocks from 12-wide row vectors, as the
// other gather kernels do.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace stencil {

template <typename T> struct TbShape;
template <> struct TbShape<float> {
  static constexpr int TM = 64, TN = 64, HMAX = 12;  // LDS: 2 x 92 x 96 x 4 B = 70,656 B (2 workgroups / CU)
};
template <> struct TbShape<double> {
  static constexpr int TM = 32, TN = 64, HMAX = 8;   // LDS: 2 x 52 x 88 x 8 B = 73,216 B (2 workgroups / CU)
};

__host__ __device__ constexpr int tb_halo(int R, int steps) { return round_up(R * steps, 4); }

// Tiles of a time-blocked launch: tiles0 = tile rows, tiles1 = tile columns.
template <typename T>
inline int64_t tb2d_items(KArgs& a) {
  typedef TbShape<T> S;
  a.tiles0 = (int32_t)((a.d0 + S::TM - 1) / S::TM);
  a.tiles1 = (int32_t)((a.d1 + S::TN - 1) / S::TN);
  return (int64_t)a.tiles0 * a.tiles1;
}

template <typename T>
inline bool tb2d_fast(const KArgs& a) {
  return a.d1 % 4 == 0 && (reinterpret_cast<uintptr_t>(a.in) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(a.out) & 15) == 0;
}

template <typename T, int R, bool BOX, bool FAST>
__device__ __forceinline__ void tb2d_item(const KArgs& a, int item) {
  typedef TbShape<T> S;
  typedef typename Vec16<T>::type V;
  constexpr int W = 2 * R + 1, VEC = 16 / (int)sizeof(T);
  constexpr int WMAX = S::TM + 2 * S::HMAX + 4;  // + 4 rows: the last 2-row block may run past the window
  constexpr int P = S::TN + 2 * S::HMAX + 8;      // columns 4 + y; 12-wide reads reach 4 past the window
  __shared__ __attribute__((aligned(16))) T buf[2][WMAX * P];

  const int steps = a.steps;
  const int HW = tb_halo(R, steps);
  const int WM = S::TM + 2 * HW, WN = S::TN + 2 * HW, NSEG = WN / 4;
  const int ti = item / a.tiles1, tj = item - (item / a.tiles1) * a.tiles1;
  const int64_t M = a.d0, N = a.d1;
  const int64_t i0 = (int64_t)ti * S::TM - HW, j0 = (int64_t)tj * S::TN - HW;
  const bool periodic = a.periodic != 0;
  const T* __restrict__ in = (const T*)a.in;
  T* __restrict__ out = (T*)a.out;
  const ConstPtr<T> c = (ConstPtr<T>)a.coef;

  // stage the window: 4-element segments
  for (int idx = threadIdx.x; idx < WM * NSEG; idx += 256) {
    const int x = idx / NSEG, sg = idx - (idx / NSEG) * NSEG;
    const int64_t gi = map_index(i0 + x, M, periodic);
    const int64_t gj = j0 + 4 * sg;
    T v[4];
    if (FAST && gi >= 0 && gj >= 0 && gj + 3 < N) {
      const V* src = reinterpret_cast<const V*>(in + gi * N + gj);
#pragma unroll
      for (int k = 0; k < 4 / VEC; ++k) {
        const V t = src[k];
        const T* pt = reinterpret_cast<const T*>(&t);
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[k * VEC + e] = pt[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t cj = map_index(gj + e, N, periodic);
        v[e] = (gi >= 0 && cj >= 0) ? in[gi * N + cj] : T(0);
      }
    }
    V* dst = reinterpret_cast<V*>(&buf[0][x * P + 4 + 4 * sg]);
#pragma unroll
    for (int k = 0; k < 4 / VEC; ++k) {
      V t;
      T* pt = reinterpret_cast<T*>(&t);
#pragma unroll
      for (int e = 0; e < VEC; ++e) pt[e] = v[k * VEC + e];
      dst[k] = t;
    }
  }
  __syncthreads();

  for (int s = 0; s < steps; ++s) {
    const T* __restrict__ src = buf[s & 1];
    T* __restrict__ dstb = buf[(s + 1) & 1];
    // valid after this step: rows and columns [lo, W - lo), covered by 2 x 4
    // blocks (their extra row / columns read stale values and are never used)
    const int lo = R * (s + 1);
    const int sg0 = lo / 4, nseg = (WN - lo + 3) / 4 - sg0;
    const int nblk = ((WM - 2 * lo + 1) / 2) * nseg;
    for (int idx = threadIdx.x; idx < nblk; idx += 256) {
      const int bx = idx / nseg, sg = sg0 + idx - (idx / nseg) * nseg;
      const int x = lo + 2 * bx;  // window rows x, x + 1
      T acc[2][4];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[p][e] = T(0);
#pragma unroll
      for (int dx = 0; dx < 2 + 2 * R; ++dx) {
        // window row x - r + dx, LDS columns 4 sg .. 4 sg + 11 = window columns 4 sg - 4 .. 4 sg + 7
        const V* rp = reinterpret_cast<const V*>(src + (x - R + dx) * P + 4 * sg);
        T v[12];
#pragma unroll
        for (int k = 0; k < 12 / VEC; ++k) {
          const V t = rp[k];
          const T* pt = reinterpret_cast<const T*>(&t);
#pragma unroll
          for (int e = 0; e < VEC; ++e) v[k * VEC + e] = pt[e];
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int aa = dx - p;  // C^g row
          if (aa < 0 || aa > 2 * R) continue;
#pragma unroll
          for (int b = 0; b < W; ++b) {
            if (!BOX && aa != R && b != R) continue;
            const T w = c[aa * W + b];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[p][e] += w * v[4 - R + e + b];
          }
        }
      }
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (!periodic) {
          const int64_t gi = i0 + x + p;
          const bool row_in = gi >= 0 && gi < M;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t gj = j0 + 4 * sg + e;
            if (!row_in || gj < 0 || gj >= N) acc[p][e] = T(0);
          }
        }
        V* dv = reinterpret_cast<V*>(dstb + (x + p) * P + 4 + 4 * sg);
#pragma unroll
        for (int k = 0; k < 4 / VEC; ++k) {
          V t;
          T* pt = reinterpret_cast<T*>(&t);
#pragma unroll
          for (int e = 0; e < VEC; ++e) pt[e] = acc[p][k * VEC + e];
          dv[k] = t;
        }
      }
    }
    __syncthreads();
  }

  // store the tile: window rows HW .., columns HW ..
  const T* __restrict__ fin = buf[steps & 1];
  constexpr int TSEG = S::TN / 4;
  for (int idx = threadIdx.x; idx < S::TM * TSEG; idx += 256) {
    const int x = idx / TSEG, sg = idx - (idx / TSEG) * TSEG;
    const int64_t gi = (int64_t)ti * S::TM + x, gj = (int64_t)tj * S::TN + 4 * sg;
    if (gi >= M || gj >= N) continue;
    const T* srcp = fin + (HW + x) * P + 4 + HW + 4 * sg;
    T* dstp = out + gi * N + gj;
    if (FAST) {  // N % 4 == 0: the 4-element segment lies inside the row
      const V* sv = reinterpret_cast<const V*>(srcp);
#pragma unroll
      for (int k = 0; k < 4 / VEC; ++k) reinterpret_cast<V*>(dstp)[k] = sv[k];
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (gj + e < N) dstp[e] = srcp[e];
    }
  }
}

template <typename T, int R, bool BOX, bool FAST>
__global__ __launch_bounds__(256) void tb2d_kernel(KArgs a) {
  tb2d_item<T, R, BOX, FAST>(a, blockIdx.x);
}

template <typename T, int R, bool BOX, bool FAST>
__global__ __launch_bounds__(256) void tb2d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { tb2d_item<T, R, BOX, FAST>(x, id); });
}

// ---------------------------------------------------------------------------
// Form with the step count TS fixed at compile time, for grids that take
// direct-to-LDS windows (column extent a multiple of 4, 16-byte aligned
// buffers, a zero line).  The window is sized for TS: halo HW =
// round_up(r TS, 4), so a 64 x 64 FP32 tile at r TS <= 4 holds 72 x 80 floats
// (23 KiB) and six workgroups share a CU, against two for the general form,
// which sizes its two buffers for the largest halo (FP64: 32 x 64 tiles).
// The window is copied from global memory straight into LDS
// (global_load_lds_dwordx4, no registers; lines outside a zero-halo grid and
// the 4-column margins read the zero line) and the steps update it in place:
// each thread computes its 2 x 4 blocks of a step into registers, a barrier,
// then writes them back.  Every loop bound is a constant once TS is.
// ---------------------------------------------------------------------------
// TM_ = 0: the library's tile rows (64 FP32, 32 FP64); FP64 grids of fewer
// tiles than CUs take 16-row tiles (twice the workgroups).
template <typename T, int R, int TS, int TM_ = 0>
struct TbDmaShape {
  static constexpr int TM = TM_ > 0 ? TM_ : (sizeof(T) == 4 ? 64 : 32), TN = 64;
  // 16 rows is the smallest tile verified against the oracle (8-row FP64
  // tiles gave wrong results and are not built)
  static_assert(TM >= 16, "tile rows");
  static constexpr int VEC = 16 / (int)sizeof(T);  // elements per 16-byte line
  static constexpr int HW = round_up(R * TS, 4);
  static constexpr int WM = TM + 2 * HW, WN = TN + 2 * HW;
  static constexpr int P = WN + 8;                 // LDS row: window columns -4 .. WN + 3
  static constexpr int LPR = P / VEC;              // 16-byte lines per LDS row
  static constexpr int MARGIN = 4 / VEC;           // lines of the 4-column margins
  static constexpr int NI = (WM * LPR + 63) / 64;  // load instructions (1 KiB each)
  static constexpr int NPW = (NI + 3) / 4;         // per wave, at most
  // elements: the loaded lines (whole instructions) and one row past the
  // window, which the last 2-row block of a step reads
  static constexpr int BUF = NI * 64 * VEC > (WM + 1) * P ? NI * 64 * VEC : (WM + 1) * P;
  // 2 x 4 blocks of the first (largest) step, and per thread
  static constexpr int NBLK1 = ((WM - 2 * R + 1) / 2) * ((WN - R + 3) / 4 - R / 4);
  static constexpr int NBPT = (NBLK1 + 255) / 256;
  static_assert(HW <= TbShape<T>::HMAX, "halo within the general form's limit");
};

template <typename T> struct TbVec;
template <> struct TbVec<float> { typedef floatx4 type; };
template <> struct TbVec<double> { typedef double __attribute__((ext_vector_type(2))) type; };

template <typename T, int R, bool BOX, int TS, int TM_ = 0>
__device__ __forceinline__ void tb2d_dma_item(const KArgs& a, int item) {
  typedef TbDmaShape<T, R, TS, TM_> S;
  typedef typename TbVec<T>::type V;
  constexpr int W = 2 * R + 1, VEC = S::VEC;
  __shared__ __attribute__((aligned(16))) T buf[S::BUF];

  const int ti = item / a.tiles1, tj = item - (item / a.tiles1) * a.tiles1;
  const int64_t M = a.d0, N = a.d1;
  const int64_t i0 = (int64_t)ti * S::TM - S::HW, j0 = (int64_t)tj * S::TN - S::HW;  // window origin
  const bool periodic = a.periodic != 0;
  const T* __restrict__ in = (const T*)a.in;
  const T* __restrict__ zeros = (const T*)a.zeros;
  T* __restrict__ out = (T*)a.out;
  // the weights a step uses: scalar registers up to 49 FP32 / 25 FP64 of
  // them; more (the r = 4 FP32 box, FP64 boxes from r = 3) go to vector registers
  constexpr int NW = BOX ? W * W : 2 * W - 1;
  typedef typename std::conditional<NW <= (sizeof(T) == 4 ? 49 : 25), ConstPtr<T>, const T*>::type CoefPtr;
  const CoefPtr c = (CoefPtr)a.coef;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;

  // window rows 0 .. WM - 1, LDS column k = window column k - 4
#pragma unroll
  for (int k = 0; k < S::NPW; ++k) {
    const int inst = k * 4 + w;
    if (inst >= S::NI) break;  // wave-uniform
    const int line = inst * 64 + lane;
    const T* src = zeros;
    const int row = line / S::LPR, lc = line - (line / S::LPR) * S::LPR;
    if (row < S::WM && lc >= S::MARGIN && lc < S::LPR - S::MARGIN) {
      const int64_t g = map_index(i0 + row, M, periodic);
      const int64_t cc = map_index(j0 - 4 + VEC * lc, N, periodic);
      if (g >= 0 && cc >= 0) src = in + g * N + cc;
    }
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t*)(buf + inst * 64 * VEC), 16, 0, 0);
  }
  __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's lines are in LDS
  __syncthreads();

#pragma unroll
  for (int s = 0; s < TS; ++s) {
    // valid after step s + 1: window rows and columns [lo, W - lo)
    const int lo = R * (s + 1);
    const int sg0 = lo / 4, nseg = (S::WN - lo + 3) / 4 - sg0;
    const int nblk = ((S::WM - 2 * lo + 1) / 2) * nseg;
    T res[S::NBPT][2][4];
#pragma unroll
    for (int q = 0; q < S::NBPT; ++q) {
      const int idx = tid + 256 * q;
      if (idx >= nblk) break;
      const int bx = idx / nseg, sg = sg0 + idx - (idx / nseg) * nseg;
      const int x = lo + 2 * bx;  // window rows x, x + 1
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) res[q][p][e] = T(0);
#pragma unroll
      for (int dx = 0; dx < 2 + 2 * R; ++dx) {
        // window row x - r + dx, LDS columns 4 sg .. 4 sg + 11 (window
        // columns 4 sg - 4 .. 4 sg + 7), read as whole 16-byte vectors.  A row
        // uses columns 4 - r .. 7 + r of the 12 (a star row other than the two
        // output rows' own: 4 .. 7 only); vectors outside are skipped, and
        // the compiler would narrow a partly used one into 4- or 8-byte reads
        // that meet a fraction of the banks at this lane stride, so the empty
        // asm keeps it whole (at the cost of a wait for it)
        const V* rp = reinterpret_cast<const V*>(buf + (x - R + dx) * S::P + 4 * sg);
        const bool full = BOX || dx == R || dx == R + 1;
        T v[12];
#pragma unroll
        for (int k = 0; k < 12 / VEC; ++k) {
          const int lo_e = full ? 4 - R : 4, hi_e = full ? 7 + R : 7;  // columns used
          if (VEC * k + VEC - 1 < lo_e || VEC * k > hi_e) continue;
          V t4 = rp[k];
          if (VEC * k < lo_e || VEC * k + VEC - 1 > hi_e) asm volatile("" : "+v"(t4));
#pragma unroll
          for (int e = 0; e < VEC; ++e) v[VEC * k + e] = t4[e];
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int aa = dx - p;  // C^g row
          if (aa < 0 || aa > 2 * R) continue;
#pragma unroll
          for (int b = 0; b < W; ++b) {
            if (!BOX && aa != R && b != R) continue;
            const T wgt = c[aa * W + b];
#pragma unroll
            for (int e = 0; e < 4; ++e) res[q][p][e] += wgt * v[4 - R + e + b];
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < S::NBPT; ++q) {
      const int idx = tid + 256 * q;
      if (idx >= nblk) break;
      const int bx = idx / nseg, sg = sg0 + idx - (idx / nseg) * nseg;
      const int x = lo + 2 * bx;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (!periodic) {
          // zero halo: points outside the grid stay 0
          const int64_t gi = i0 + x + p;
          const bool row_in = gi >= 0 && gi < M;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t gj = j0 + 4 * sg + e;
            if (!row_in || gj < 0 || gj >= N) res[q][p][e] = T(0);
          }
        }
        V* dv = reinterpret_cast<V*>(buf + (x + p) * S::P + 4 + 4 * sg);
#pragma unroll
        for (int k = 0; k < 4 / VEC; ++k) {
          V t4;
#pragma unroll
          for (int e = 0; e < VEC; ++e) t4[e] = res[q][p][VEC * k + e];
          dv[k] = t4;
        }
      }
    }
    __syncthreads();
  }

  // store the tile: window rows HW .., columns HW .. (N % 4 == 0: whole segments)
  constexpr int TSEG = S::TN / 4;
#pragma unroll
  for (int k = 0; k < (S::TM * TSEG + 255) / 256; ++k) {
    const int idx = tid + 256 * k;
    const int x = idx / TSEG, sg = idx - (idx / TSEG) * TSEG;
    const int64_t gi = (int64_t)ti * S::TM + x, gj = (int64_t)tj * S::TN + 4 * sg;
    if (gi >= M || gj >= N) continue;
    const V* sv = reinterpret_cast<const V*>(buf + (S::HW + x) * S::P + 4 + S::HW + 4 * sg);
    V* dv = reinterpret_cast<V*>(out + gi * N + gj);
#pragma unroll
    for (int e = 0; e < 4 / VEC; ++e) dv[e] = sv[e];
  }
}

template <typename T, int R, bool BOX, int TS, int TM_ = 0>
__global__ __launch_bounds__(256) void tb2d_dma_kernel(KArgs a) {
  tb2d_dma_item<T, R, BOX, TS, TM_>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool BOX, int TS, int TM_ = 0>
__global__ __launch_bounds__(256) void tb2d_dma_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { tb2d_dma_item<T, R, BOX, TS, TM_>(x, id); });
}

// The direct-to-LDS kernel for order R and `steps` steps (2 <= steps, halo
// within the limit), empty if not built, with its tile rows; FP32 boxes,
// FP32 stars and FP64 are instantiated in separate translation units.
Kernel tb2d_dma_box(int R, int steps, int64_t items);
Kernel tb2d_dma_star(int R, int steps, int64_t items);
Kernel tb2d_dma_f64(bool box, int R, int steps, int64_t items, bool small_tiles);
constexpr int kTbSmallRows = 16;  // FP64 tile rows on grids of fewer tiles than CUs
template <typename T>
constexpr int tb2d_dma_rows() { return TbDmaShape<T, 1, 2>::TM; }

template <typename T, int R, bool BOX, int TS, int TM_ = 0>
Kernel tb2d_dma_of(int steps, int64_t items) {
  if constexpr (round_up(R * TS, 4) > TbShape<T>::HMAX) {
    return Kernel{};
  } else {
    if (steps == TS)
      return kernel_of<tb2d_dma_kernel<T, R, BOX, TS, TM_>, tb2d_dma_batch<T, R, BOX, TS, TM_>>(items);
    return tb2d_dma_of<T, R, BOX, TS + 1, TM_>(steps, items);
  }
}

template <typename T, bool BOX, int TM_ = 0>
Kernel tb2d_dma_pick(int R, int steps, int64_t items) {
  switch (R) {
    case 1: return tb2d_dma_of<T, 1, BOX, 2, TM_>(steps, items);
    case 2: return tb2d_dma_of<T, 2, BOX, 2, TM_>(steps, items);
    case 3: return tb2d_dma_of<T, 3, BOX, 2, TM_>(steps, items);
    case 4: return tb2d_dma_of<T, 4, BOX, 2, TM_>(steps, items);
  }
  return Kernel{};
}

}  // namespace stencil
