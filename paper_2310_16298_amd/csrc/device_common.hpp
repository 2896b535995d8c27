// Device-side building blocks shared by the stencil kernels (gfx950).
//
// Grids are C order with the rightmost index contiguous (2D: (i, j);
// 3D: (i, j, k)).  A 2D tile is staged into LDS as a halo'd "window": the
// output tile's rows and columns extended by r on every side.  Window row 0
// is output row (tile row 0 - r); window column y is stored at LDS column
// COL0 + y, with COL0 chosen so the tile body (window column r) starts on a
// 16-byte boundary.  The boundary rule is applied here, once, so the compute
// loops run without predicates: ZERO reads 0 outside the grid, PERIODIC wraps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stencil {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Arguments common to every kernel.  Passed by value (kernarg segment).
struct KArgs {
  const void* in;       // input grid (device)
  void* out;            // output grid (device)
  const void* frag;     // packed MFMA operand fragments (device, plan-owned)
  const void* coef;     // dense C^g in the arithmetic dtype (device, plan-owned)
  const void* zeros;    // 256 bytes of zeros (device, plan-owned): source of zero-halo lines
  int64_t d0, d1, d2;   // extents; d2 == 1 for 2D
  int32_t periodic;     // 1 = wrap, 0 = zero halo
  int32_t tiles0;       // tiles along the first tiled axis
  int32_t tiles1;       // tiles along the second tiled axis
  int32_t chunk;        // 3D: planes (i) per workgroup
  int32_t nchunks;      // 3D: number of i-chunks
  float out_scale;      // split-precision paths: exact power-of-two rescale of the result
  float lo_scale;       // split-precision paths: weight of the cross-term accumulator
  int32_t steps;        // time-blocked kernels: Jacobi steps fused in this launch
  int32_t lcode0;       // line-cover kernel: slots 0..5, 5 bits each (bit 4: line along j, bits 0..3: index)
  int32_t lcode1;       // slots 6..8 in bits 0..14, number of lines in bits 27..30
};

// Pointer to data that no lane writes during a kernel (constant address
// space): uniform reads through it compile to scalar loads.
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;

__host__ __device__ constexpr int round_up(int v, int m) { return (v + m - 1) / m * m; }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Destination type of the direct-to-LDS loads (global_load_lds).
typedef __attribute__((address_space(3))) void lds_void_t;

// Workgroup barrier over LDS only: waits for this wave's LDS operations
// (lgkmcnt(0)) and joins the barrier, leaving vector-memory operations in
// flight.  __syncthreads() also waits for those (vmcnt(0)) -- the compiler
// treats pending direct-to-LDS loads as LDS writes -- which would make every
// block wait for the prefetch of the next window as well.  Direct-to-LDS
// windows are published by each wave's own vmcnt wait before this barrier.
// The memory clobber keeps the compiler from moving memory accesses across.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// v_mfma_f32_4x4x1_16b_f32 with the B operand taken from lane group g (the
// B lane-group broadcast, blgp = 4 + g: lanes 16 g .. 16 g + 15 feed all 16
// blocks).  A register can then carry four B vectors, one per lane group;
// g must fold to a constant after unrolling.
__device__ __forceinline__ floatx4 mfma4_group(float a, float b, floatx4 c, int g) {
  switch (g) {
    case 0: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 4);
    case 1: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 5);
    case 2: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 6);
    default: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 7);
  }
}

// v_mfma_f32_4x4x1_16b_f32 with the A operand of block 4 g (lanes 16 g ..
// 16 g + 3) broadcast to all 16 blocks (cbsz = 4, abid = 4 g): with the same
// packing as mfma4_group, a register's lane group g holds one A vector.
__device__ __forceinline__ floatx4 mfma4_agroup(float a, float b, floatx4 c, int g) {
  switch (g) {
    case 0: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 0, 0);
    case 1: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 4, 0);
    case 2: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 8, 0);
    default: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 12, 0);
  }
}

// Index of global coordinate g under the boundary rule, or -1 for a zero-halo
// point outside [0, n).  The modulo branch is taken only at grid faces.
__device__ __forceinline__ int64_t map_index(int64_t g, int64_t n, bool periodic) {
  if (g >= 0 && g < n) return g;
  if (!periodic) return -1;
  int64_t m = g % n;
  return m < 0 ? m + n : m;
}

// Column offset in LDS that puts window column R on a 16-byte boundary.
template <typename T, int R>
__host__ __device__ constexpr int lds_col0() {
  return round_up(R, 16 / (int)sizeof(T)) - R;
}

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; };
template <> struct Vec16<double> { typedef double2 type; };

// Stage a ROWS x (BODY + 2R) window of a 2D slice into LDS.
//   src          : the 2D slice (rows x cols = M x N), C order
//   r0           : global row of window row 0
//   c0           : global column of the tile body (window column R); c0 % VEC == 0
//   lds[row * PITCH + COL0 + y] receives window element (row, y); COL0 + R
//   must be a multiple of VEC.
// All NT threads of the block must call it.
template <typename T, int R, int ROWS, int BODY, int PITCH, int NT, int COL0 = lds_col0<T, R>()>
__device__ __forceinline__ void stage_window(T* __restrict__ lds, const T* __restrict__ src,
                                             int64_t M, int64_t N, int64_t r0, int64_t c0,
                                             bool periodic) {
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int NV = BODY / VEC;
  constexpr int WCOLS = BODY + 2 * R;
  static_assert(BODY % VEC == 0, "tile body must be a whole number of 16-byte vectors");
  typedef typename Vec16<T>::type V;
  const int tid = threadIdx.x;
  const bool fast = (c0 + BODY <= N) && (N % VEC == 0) && ((reinterpret_cast<uintptr_t>(src) & 15) == 0);
  if (fast) {
    for (int idx = tid; idx < ROWS * NV; idx += NT) {
      const int row = idx / NV;
      const int v = idx - row * NV;
      const int64_t g = map_index(r0 + row, M, periodic);
      V val;
      if (g >= 0) {
        val = *reinterpret_cast<const V*>(src + g * N + c0 + v * VEC);
      } else {
        val = V{};
      }
      T* dst = lds + row * PITCH + COL0 + R + v * VEC;
      if constexpr (PITCH % VEC == 0) {
        *reinterpret_cast<V*>(dst) = val;
      } else {
        const T* pv = reinterpret_cast<const T*>(&val);
#pragma unroll
        for (int e = 0; e < VEC; ++e) dst[e] = pv[e];
      }
    }
    for (int idx = tid; idx < ROWS * 2 * R; idx += NT) {
      const int row = idx / (2 * R);
      const int h = idx - row * (2 * R);
      const int64_t gc = (h < R) ? (c0 - R + h) : (c0 + BODY + (h - R));
      const int y = (h < R) ? h : (BODY + h);
      const int64_t g = map_index(r0 + row, M, periodic);
      const int64_t c = map_index(gc, N, periodic);
      lds[row * PITCH + COL0 + y] = (g >= 0 && c >= 0) ? src[g * N + c] : T(0);
    }
  } else {
    for (int idx = tid; idx < ROWS * WCOLS; idx += NT) {
      const int row = idx / WCOLS;
      const int y = idx - row * WCOLS;
      const int64_t g = map_index(r0 + row, M, periodic);
      const int64_t c = map_index(c0 - R + y, N, periodic);
      lds[row * PITCH + COL0 + y] = (g >= 0 && c >= 0) ? src[g * N + c] : T(0);
    }
  }
}

// Fill a rectangular LDS region with zeros (used once per block for the
// padding rows/columns that MFMA K-padding reads but the window never covers).
template <typename T, int NT>
__device__ __forceinline__ void zero_region(T* lds, int rows, int cols, int pitch, int row0, int col0) {
  for (int idx = threadIdx.x; idx < rows * cols; idx += NT) {
    const int rr = idx / cols;
    const int cc = idx - rr * cols;
    lds[(row0 + rr) * pitch + col0 + cc] = T(0);
  }
}

// XCD-aware tile order: workgroups are dispatched round-robin over the 8
// XCDs; give each XCD a contiguous range of tiles so that tiles sharing halo
// rows also share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int NXCD = 8;
  const int per = nblocks / NXCD;
  const int full = per * NXCD;
  if (bid >= full) return bid;
  return (bid % NXCD) * per + bid / NXCD;
}

// Several grids in one launch.  Grid g of a table owns the work items
// (workgroup tiles) [table[g].first, table[g+1].first); the last grid's end
// is `total`.  Its args hold buffer 0 in `in` and buffer 1 in `out`.  Launch
// number `launch` of a sequence advances the grids with launch < limit by one
// step: a grid with (launch + phase) even reads buffer 0 and writes buffer 1,
// odd the reverse, so grids that joined at different steps advance together.
struct BatchGrid {
  KArgs args;
  int32_t first;  // first work item of this grid
  int32_t phase;  // steps the grid had done before launch 0, mod 2
  int32_t limit;  // launches of the sequence that advance this grid
  int32_t pad;
};

struct BatchArgs {
  const BatchGrid* table;
  int32_t ngrids;
  int32_t total;           // work items over all grids
  int32_t launch;          // index of this launch in its sequence
  int32_t pad;
};

// Load a struct whose address is the same in every lane into scalar registers.
template <typename S>
__device__ __forceinline__ S uniform_load(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "dword-sized struct");
  S v;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(S) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
  return v;
}

// Batched launch: a persistent loop over work items blockIdx.x,
// blockIdx.x + gridDim.x, ... of all grids in the table (every workgroup ends
// after the last item); each item finds its grid by binary search over
// `first` and runs item(args, id) with the grid's args in scalar registers.
template <class F>
__device__ __forceinline__ void for_each_batch_item(const BatchArgs& b, F item) {
  for (int it = blockIdx.x; it < b.total; it += gridDim.x) {
    int lo = 0, hi = b.ngrids - 1;  // last grid with first <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (__builtin_amdgcn_readfirstlane(b.table[mid].first) <= it) lo = mid;
      else hi = mid - 1;
    }
    const BatchGrid e = uniform_load(&b.table[lo]);
    if (b.launch >= e.limit) continue;  // this grid has done its steps
    KArgs g = e.args;
    if ((b.launch + e.phase) & 1) {
      g.in = e.args.out;
      g.out = const_cast<void*>(e.args.in);
    }
    __syncthreads();  // the previous item's LDS reads are done
    item(g, it - e.first);
  }
}

}  // namespace stencil
