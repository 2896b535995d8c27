// Time-blocked 3D gather kernel: TS Jacobi steps per launch on a 3D tile held
// whole in LDS (the temporal reuse Section 6 leaves to future work, taken to
// 3D).  A workgroup owns a TI x TJ x TK output tile; its window -- the tile
// plus a halo of r TS planes and rows (r TS rounded up to 4 columns along the
// contiguous k axis) -- is copied from global memory straight into LDS
// (global_load_lds_dwordx4; lines outside a zero-halo grid and the 4-column
// margins read the zero line), the steps update it in place (each thread
// computes its 2 x 4 blocks of a step into registers, a barrier, then writes
// them back), and the tile is stored.  Step s computes the region at least
// r s from the window faces, which depends only on step s - 1's region.
// Zero halo: window points outside the grid are 0 at load and reset to 0
// after every step; periodic: the window is the periodic extension.
//
// Each point sums its taps in the order of the one-step 3D gather kernel
// (box: coefficient planes, rows, columns ascending; star: the lower i arm,
// the j arm with the centre, the k arm, the upper i arm), so a run of fused
// steps equals one-step launches bit for bit.
//
// Requirements (checked on the host): the k extent is a multiple of 4, both
// buffers 16-byte aligned, a zero line.  Built for r = 1 (the 7-point star
// and the 27-point box) and two steps: tiles of 4 x 16 x 64 FP32 or
// 4 x 16 x 32 FP64 points, whose windows (50 / 60 KiB) leave three / two
// workgroups per CU (8-plane FP32 tiles held seven blocks a thread across the
// in-place barrier: 236-256 VGPRs, one or two waves per SIMD).
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "kernels_3d.hpp"
#include "launch.hpp"

namespace stencil {

template <typename T, int R, int TS>
struct Tb3Shape {
  static constexpr int TI = 4, TJ = 16, TK = sizeof(T) == 4 ? 64 : 32;
  static constexpr int VEC = 16 / (int)sizeof(T);  // elements per 16-byte line
  static constexpr int HI = R * TS, HK = round_up(R * TS, 4);
  static constexpr int WI = TI + 2 * HI, WJ = TJ + 2 * HI, WK = TK + 2 * HK;
  static constexpr int P = WK + 8;            // LDS row: window columns -4 .. WK + 3
  static constexpr int LPR = P / VEC;         // 16-byte lines per LDS row
  static constexpr int MARGIN = 4 / VEC;      // lines of each 4-column margin
  static constexpr int ROWS = WI * WJ;        // LDS rows (plane-major)
  static constexpr int NI = (ROWS * LPR + 63) / 64;  // load instructions (1 KiB each)
  static constexpr int NPW = (NI + 3) / 4;           // per wave, at most
  // elements: the loaded lines (whole instructions) and one row past the
  // last plane, which the last 2-row block of a step reads
  static constexpr int BUF = NI * 64 * VEC > (ROWS + 1) * P ? NI * 64 * VEC : (ROWS + 1) * P;
  // 2 x 4 blocks of the first (largest) step, and per thread
  static constexpr int NJB1 = (WJ - 2 * R + 1) / 2, NSG1 = (WK - R + 3) / 4 - R / 4;
  static constexpr int NBLK1 = (WI - 2 * R) * NJB1 * NSG1;
  static constexpr int NBPT = (NBLK1 + 255) / 256;
};

template <typename T> struct Tb3Vec;
template <> struct Tb3Vec<float> { typedef floatx4 type; };
template <> struct Tb3Vec<double> { typedef double __attribute__((ext_vector_type(2))) type; };

// Host-side condition for the kernel: direct-to-LDS lines (k extent a
// multiple of 4, 16-byte aligned buffers) and a zero line.
inline bool tb3d_ok(const KArgs& a) {
  return a.d2 % 4 == 0 && (reinterpret_cast<uintptr_t>(a.in) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(a.out) & 15) == 0 && a.zeros != nullptr;
}

// (j, k) tiles of a plane in the one-step 3D decomposition (kTJ x kTK).
inline int64_t tb3d_plane_tiles(const KArgs& a) {
  return ((a.d1 + kTJ - 1) / kTJ) * ((a.d2 + kTK - 1) / kTK);
}

// Tiles of a launch along i, j, k.
template <typename T, int R, int TS>
__host__ __device__ inline void tb3d_tiles(int64_t d0, int64_t d1, int64_t d2, int64_t* ti, int64_t* tj, int64_t* tk) {
  typedef Tb3Shape<T, R, TS> S;
  *ti = (d0 + S::TI - 1) / S::TI;
  *tj = (d1 + S::TJ - 1) / S::TJ;
  *tk = (d2 + S::TK - 1) / S::TK;
}

template <typename T, int R, bool BOX, int TS>
__device__ __forceinline__ void tb3d_dma_item(const KArgs& a, int item) {
  typedef Tb3Shape<T, R, TS> S;
  typedef typename Tb3Vec<T>::type V;
  constexpr int W = 2 * R + 1, VEC = S::VEC;
  __shared__ __attribute__((aligned(16))) T buf[S::BUF];

  const int64_t Ni = a.d0, Nj = a.d1, Nk = a.d2;
  int64_t nti, ntj, ntk;
  tb3d_tiles<T, R, TS>(Ni, Nj, Nk, &nti, &ntj, &ntk);
  const int64_t tk = item % ntk, tij = item / ntk, tj = tij % ntj, ti = tij / ntj;
  // window origin
  const int64_t i0 = ti * S::TI - S::HI, j0 = tj * S::TJ - S::HI, k0 = tk * S::TK - S::HK;
  const bool periodic = a.periodic != 0;
  const T* __restrict__ in = (const T*)a.in;
  const T* __restrict__ zeros = (const T*)a.zeros;
  T* __restrict__ out = (T*)a.out;
  const ConstPtr<T> c = (ConstPtr<T>)a.coef;  // 27 weights at most: scalar loads
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;

  // window: LDS row (wi, wj) = plane i0 + wi, row j0 + wj; LDS column m =
  // window column m - 4
#pragma unroll
  for (int q = 0; q < S::NPW; ++q) {
    const int inst = q * 4 + w;
    if (inst >= S::NI) break;  // wave-uniform
    const int line = inst * 64 + lane;
    const T* src = zeros;
    const int row = line / S::LPR, lc = line - (line / S::LPR) * S::LPR;
    if (row < S::ROWS && lc >= S::MARGIN && lc < S::LPR - S::MARGIN) {
      const int wi = row / S::WJ, wj = row - (row / S::WJ) * S::WJ;
      const int64_t gi = map_index(i0 + wi, Ni, periodic);
      const int64_t gj = map_index(j0 + wj, Nj, periodic);
      const int64_t gk = map_index(k0 - 4 + VEC * lc, Nk, periodic);
      if (gi >= 0 && gj >= 0 && gk >= 0) src = in + (gi * Nj + gj) * Nk + gk;
    }
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t*)(buf + inst * 64 * VEC), 16, 0, 0);
  }
  __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's lines are in LDS
  __syncthreads();

  // 12 values of LDS row (wi, wj) from LDS column 4 sg, read as whole 16-byte
  // vectors; `lo_e .. hi_e`: the columns used (vectors outside are skipped,
  // a partly used one is kept whole by the empty asm so the compiler does not
  // narrow it into reads that meet a fraction of the LDS banks)
  auto row12 = [&](int wi, int wj, int sg, int lo_e, int hi_e, T v[12]) {
    const V* rp = reinterpret_cast<const V*>(buf + (wi * S::WJ + wj) * S::P + 4 * sg);
#pragma unroll
    for (int q = 0; q < 12 / VEC; ++q) {
      if (VEC * q + VEC - 1 < lo_e || VEC * q > hi_e) continue;
      V t4 = rp[q];
      if (VEC * q < lo_e || VEC * q + VEC - 1 > hi_e) asm volatile("" : "+v"(t4));
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[VEC * q + e] = t4[e];
    }
  };

#pragma unroll
  for (int s = 0; s < TS; ++s) {
    // valid after step s + 1: window planes, rows and columns [lo, W - lo)
    const int lo = R * (s + 1);
    const int njb = (S::WJ - 2 * lo + 1) / 2;
    const int sg0 = lo / 4, nsg = (S::WK - lo + 3) / 4 - sg0;
    const int nblk = (S::WI - 2 * lo) * njb * nsg;
    T res[S::NBPT][2][4];
#pragma unroll
    for (int q = 0; q < S::NBPT; ++q) {
      const int idx = tid + 256 * q;
      if (idx >= nblk) break;
      const int sg = sg0 + idx % nsg, rest = idx / nsg;
      const int x = lo + 2 * (rest % njb), wi = lo + rest / njb;  // rows x, x + 1 of plane wi
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) res[q][p][e] = T(0);
      if constexpr (BOX) {
        // coefficient plane ap, row bb, column cc, in that order
#pragma unroll
        for (int ap = 0; ap < W; ++ap)
#pragma unroll
          for (int dx = 0; dx < 2 + 2 * R; ++dx) {
            T v[12];
            row12(wi + ap - R, x - R + dx, sg, 4 - R, 7 + R, v);
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              const int bb = dx - p;
              if (bb < 0 || bb > 2 * R) continue;
#pragma unroll
              for (int cc = 0; cc < W; ++cc) {
                const T wgt = c[(ap * W + bb) * W + cc];
#pragma unroll
                for (int e = 0; e < 4; ++e) res[q][p][e] += wgt * v[4 - R + e + cc];
              }
            }
          }
      } else {
        // lower i arm
#pragma unroll
        for (int ap = 0; ap < R; ++ap)
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            T v[12];
            row12(wi + ap - R, x + p, sg, 4, 7, v);
            const T wgt = c[(ap * W + R) * W + R];
#pragma unroll
            for (int e = 0; e < 4; ++e) res[q][p][e] += wgt * v[4 + e];
          }
        // j arm with the centre
#pragma unroll
        for (int dx = 0; dx < 2 + 2 * R; ++dx) {
          T v[12];
          row12(wi, x - R + dx, sg, 4, 7, v);
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            const int bb = dx - p;
            if (bb < 0 || bb > 2 * R) continue;
            const T wgt = c[(R * W + bb) * W + R];
#pragma unroll
            for (int e = 0; e < 4; ++e) res[q][p][e] += wgt * v[4 + e];
          }
        }
        // k arm (centre excluded)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          T v[12];
          row12(wi, x + p, sg, 4 - R, 7 + R, v);
#pragma unroll
          for (int cc = 0; cc < W; ++cc) {
            if (cc == R) continue;
            const T wgt = c[(R * W + R) * W + cc];
#pragma unroll
            for (int e = 0; e < 4; ++e) res[q][p][e] += wgt * v[4 - R + e + cc];
          }
        }
        // upper i arm
#pragma unroll
        for (int ap = R + 1; ap < W; ++ap)
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            T v[12];
            row12(wi + ap - R, x + p, sg, 4, 7, v);
            const T wgt = c[(ap * W + R) * W + R];
#pragma unroll
            for (int e = 0; e < 4; ++e) res[q][p][e] += wgt * v[4 + e];
          }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < S::NBPT; ++q) {
      const int idx = tid + 256 * q;
      if (idx >= nblk) break;
      const int sg = sg0 + idx % nsg, rest = idx / nsg;
      const int x = lo + 2 * (rest % njb), wi = lo + rest / njb;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (!periodic) {
          // zero halo: points outside the grid stay 0
          const int64_t gi = i0 + wi, gj = j0 + x + p;
          const bool in_ij = gi >= 0 && gi < Ni && gj >= 0 && gj < Nj;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t gk = k0 + 4 * sg + e;
            if (!in_ij || gk < 0 || gk >= Nk) res[q][p][e] = T(0);
          }
        }
        V* dv = reinterpret_cast<V*>(buf + (wi * S::WJ + x + p) * S::P + 4 + 4 * sg);
#pragma unroll
        for (int m = 0; m < 4 / VEC; ++m) {
          V t4;
#pragma unroll
          for (int e = 0; e < VEC; ++e) t4[e] = res[q][p][VEC * m + e];
          dv[m] = t4;
        }
      }
    }
    __syncthreads();
  }

  // store the tile: window planes / rows HI .., columns HK .. (Nk % 4 == 0:
  // a 4-column segment lies inside the row)
  constexpr int TSEG = S::TK / 4, NSEG = S::TI * S::TJ * TSEG;
#pragma unroll
  for (int q = 0; q < (NSEG + 255) / 256; ++q) {
    const int idx = tid + 256 * q;
    if (idx >= NSEG) break;
    const int sg = idx % TSEG, rest = idx / TSEG, jj = rest % S::TJ, ii = rest / S::TJ;
    const int64_t gi = ti * S::TI + ii, gj = tj * S::TJ + jj, gk = tk * S::TK + 4 * sg;
    if (gi >= Ni || gj >= Nj || gk >= Nk) continue;
    const V* sv = reinterpret_cast<const V*>(buf + ((S::HI + ii) * S::WJ + S::HI + jj) * S::P + 4 + S::HK + 4 * sg);
    V* dv = reinterpret_cast<V*>(out + (gi * Nj + gj) * Nk + gk);
#pragma unroll
    for (int m = 0; m < 4 / VEC; ++m) dv[m] = sv[m];
  }
}

template <typename T, int R, bool BOX, int TS>
__global__ __launch_bounds__(256) void tb3d_dma_kernel(KArgs a) {
  tb3d_dma_item<T, R, BOX, TS>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool BOX, int TS>
__global__ __launch_bounds__(256) void tb3d_dma_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { tb3d_dma_item<T, R, BOX, TS>(x, id); });
}


// ---------------------------------------------------------------------------
// Streaming form (two steps): the work item of the one-step 3D kernels -- a
// kTJ x kTK tile of the (j, k) plane and a chunk of output planes -- with a
// plane ring per time level.  The walk reads input planes ib - 2r ..
// iend + 2r - 1 once each: the window of a plane (rows j0 - 2r .., columns
// k0 - M .. k0 + kTK + M - 1, M = 4 up to order 2 and 8 beyond) is copied
// straight into LDS (double-buffered) and scattered into a ring of 2r+1
// level-1 planes in registers covering the tile plus an r halo (rows
// j0 - r .., columns k0 - 4 .. k0 + kTK + 3).  When level-1 plane p is
// complete it goes to an LDS plane (zero outside a zero-halo grid) and is
// scattered into the ring of level-2 planes (the tile), whose complete plane
// p - r is stored.  Only the 2r-row and M-column halos of the (j, k) window
// are read twice; along i nothing is, apart from the 4r planes at the ends of
// a chunk.  Both levels sum their taps in the order of the one-step kernel
// (its ring scatter), so the result equals two one-step launches bit for bit.
// Built for FP32 stars of order 1 to 4, the FP32 27-point box and FP64
// order 1.
// ---------------------------------------------------------------------------
template <typename T, int R, bool BOX>
struct Tb3Stream {
  static constexpr int W = 2 * R + 1, VEC = 16 / (int)sizeof(T);
  static constexpr int ROWS0 = kTJ + 4 * R;                     // input window rows: global j0 - 2r ..
  // window columns k0 - M .. k0 + kTK + M - 1: level 1 reaches 2r columns
  // past the tile, within a 4-column margin up to order 2, an 8-column one beyond
  static constexpr int M = 2 * R <= 4 ? 4 : 8;
  static constexpr int ROWS1 = kTJ + 2 * R;                     // level-1 rows: global j0 - r ..
  static constexpr int SEG1 = (kTK + 8) / 4;                    // level-1 column blocks: k0 - 4 ..
  static constexpr int NBLK1 = ROWS1 / 2 * SEG1;
  // Workgroup size.  The level-1 pass has 306-360 blocks: with 256 threads
  // one or two waves run a second pass while the others wait at the plane's
  // barrier.  FP32 stars of order 1-2 and the FP32 27-point box take one
  // block per thread (5 / 6 waves, the waves past the fourth sit out level 2;
  // at most two workgroups per CU; 512^3 on MI355X: 1053 vs 938, 784 vs 683
  // and 627 vs 612 GStencil/s, 384^3 box 560 vs 522); FP64 (463 vs 581 at
  // 512^3) and orders 3-4 (406 vs 537) ran slower that way and keep 256.
  static constexpr bool SPREAD = sizeof(T) == 4 && (R == 1 || (!BOX && R == 2));
  static constexpr int NT = SPREAD ? round_up(NBLK1, 64) : 256;
  typedef DmaPlane<T, 2 * R, ROWS0, kTK, NT, M> D;
  static constexpr int P0 = D::PITCH;
  static constexpr int PAD = 4;                                 // elements before the window (16 bytes)
  // with M = 4 a 12-wide read of the first column block starts 4 elements
  // before a row, one of the last ends 4 past it
  static constexpr int BUF0 = round_up(PAD + cmax(D::BUF, ROWS0 * P0) + 4, 4);
  // LDS column (in a window row) where level-1 block s's 12-wide read starts,
  // minus 4 s: global column k0 - 8 + 4 s
  static constexpr int SRC0 = M - 8;
  static constexpr int P1 = kTK + 16;                           // level-1 row: global columns k0 - 8 ..
  static constexpr int BUF1 = ROWS1 * P1;
  static constexpr int NB1 = (NBLK1 + NT - 1) / NT;             // level-1 blocks per thread
  static_assert(kTJ / 2 * (kTK / 4) == 256, "one level-2 block per thread of the first four waves");
  static_assert(NT <= 1024 && NT % 64 == 0, "workgroup of whole waves");
  static_assert(R <= 4, "level-1 blocks k0 - 4 .. cover the level-2 reach");
};

template <typename T, int R, bool BOX>
__device__ __forceinline__ void tb3d_stream_item(const KArgs& a, int item) {
  typedef Tb3Stream<T, R, BOX> S;
  typedef typename S::D D;
  typedef typename Tb3Vec<T>::type V;
  constexpr int W = S::W, VEC = S::VEC;
  __shared__ __attribute__((aligned(16))) T lds[2 * S::BUF0 + S::BUF1];

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Ni = a.d0, Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  const bool periodic = a.periodic != 0;
  const T* __restrict__ in = (const T*)a.in;
  const T* __restrict__ zeros = (const T*)a.zeros;
  T* __restrict__ out = (T*)a.out;
  const ConstPtr<T> c = (ConstPtr<T>)a.coef;  // 27 weights at most: scalar loads
  const int tid = threadIdx.x;
  T* const l1 = lds + 2 * S::BUF0;

  // pads and the level-1 plane start at zero (cells no DMA line writes)
  for (int e = tid; e < 2 * S::BUF0 + S::BUF1; e += S::NT) lds[e] = T(0);
  __syncthreads();

  // ring1[n]: the level-1 ring of this thread's block n; ring2: its level-2 block
  T ring1[S::NB1][W][2][4], ring2[W][2][4];
#pragma unroll
  for (int z = 0; z < W; ++z) {
#pragma unroll
    for (int n = 0; n < S::NB1; ++n)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) ring1[n][z][p][e] = T(0);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) ring2[z][p][e] = T(0);
  }

  // 12 values from LDS (whole 16-byte vectors; `lo_e .. hi_e`: the ones used,
  // a partly used vector kept whole so the compiler does not narrow it)
  auto read12 = [&](const T* src, int lo_e, int hi_e, T v[12]) {
    const V* rp = reinterpret_cast<const V*>(src);
#pragma unroll
    for (int q = 0; q < 12 / VEC; ++q) {
      if (VEC * q + VEC - 1 < lo_e || VEC * q > hi_e) continue;
      V t4 = rp[q];
      if (VEC * q < lo_e || VEC * q + VEC - 1 > hi_e) asm volatile("" : "+v"(t4));
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[VEC * q + e] = t4[e];
    }
  };
  // Scatter one plane from LDS into a ring (the one-step kernel's order):
  // `src` = LDS row of the block's first row minus r, at the first of 12
  // columns (the block's columns are 4 .. 7 of them).
  auto scatter = [&](const T* src, int pitch, T ring[W][2][4]) {
    if constexpr (BOX) {
#pragma unroll
      for (int x = 0; x < 2 + 2 * R; ++x) {
        T v[12];
        read12(src + x * pitch, 4 - R, 7 + R, v);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int bb = x - p;
          if (bb < 0 || bb > 2 * R) continue;
#pragma unroll
          for (int ap = 0; ap < W; ++ap)
#pragma unroll
            for (int cc = 0; cc < W; ++cc) {
              const T wgt = c[(ap * W + bb) * W + cc];
#pragma unroll
              for (int e = 0; e < 4; ++e) ring[2 * R - ap][p][e] += wgt * v[4 - R + e + cc];
            }
        }
      }
    } else {
      // j arm (centre included) into the centre plane's slot r
#pragma unroll
      for (int x = 0; x < 2 + 2 * R; ++x) {
        T v[12];
        read12(src + x * pitch, 4, 7, v);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int bb = x - p;
          if (bb < 0 || bb > 2 * R) continue;
          const T wgt = c[(R * W + bb) * W + R];
#pragma unroll
          for (int e = 0; e < 4; ++e) ring[R][p][e] += wgt * v[4 + e];
        }
      }
      // k arm (centre excluded) and i arm from the block's own rows
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        T v[12];
        read12(src + (p + R) * pitch, 4 - R, 7 + R, v);
#pragma unroll
        for (int cc = 0; cc < W; ++cc) {
          if (cc == R) continue;
          const T wgt = c[(R * W + R) * W + cc];
#pragma unroll
          for (int e = 0; e < 4; ++e) ring[R][p][e] += wgt * v[4 - R + e + cc];
        }
#pragma unroll
        for (int ap = 0; ap < W; ++ap) {
          if (ap == R) continue;
          const T wgt = c[(ap * W + R) * W + R];
#pragma unroll
          for (int e = 0; e < 4; ++e) ring[2 * R - ap][p][e] += wgt * v[4 + e];
        }
      }
    }
  };
  auto shift = [&](T ring[W][2][4]) {
#pragma unroll
    for (int z = 0; z < 2 * R; ++z)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) ring[z][p][e] = ring[z + 1][p][e];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) ring[2 * R][p][e] = T(0);
  };

  typename D::Lines lines;
  D::prepare(lines, Nj, Nk, ch.j0 - 2 * R, ch.k0, periodic);
  const int nu = (int)(ch.iend - ch.ib) + 4 * R;
  {
    const int64_t g0 = map_index(ch.ib - 2 * R, Ni, periodic);
    D::issue(lds + S::PAD, g0 >= 0 ? in + g0 * plane : nullptr, zeros, lines);
  }
  const int rp2 = tid >> 4, q2 = tid & 15;  // level-2 block: rows j0 + 2 rp2 .., columns k0 + 4 q2 ..
  for (int u = 0; u < nu; ++u) {
    T* const win = lds + (u & 1) * S::BUF0 + S::PAD;
    if (u + 1 < nu) {
      const int64_t g1 = map_index(ch.ib - 2 * R + u + 1, Ni, periodic);
      D::issue(lds + ((u + 1) & 1) * S::BUF0 + S::PAD, g1 >= 0 ? in + g1 * plane : nullptr, zeros, lines);
      D::template wait_vm<D::NPW>();
    } else {
      D::template wait_vm<0>();
    }
    lds_barrier();  // window u in LDS; the level-2 reads of the last level-1 plane are done
    // level 1: block (rp, s) = rows j0 - r + 2 rp .., columns k0 - 4 + 4 s ..
#pragma unroll
    for (int n = 0; n < S::NB1; ++n) {
      const int b = tid + S::NT * n;
      if (b >= S::NBLK1) break;
      const int rp = b / S::SEG1, s = b - (b / S::SEG1) * S::SEG1;
      scatter(win + 2 * rp * S::P0 + 4 * s + S::SRC0, S::P0, ring1[n]);
    }
    // level-1 plane ib - 3r + u is complete once its 2r+1 input planes were walked
    const int64_t p1 = ch.ib - 3 * R + u;
    const bool have1 = u >= 2 * R;
    if (have1) {
      const int64_t gp1 = p1;
      const bool plane_in = periodic || (gp1 >= 0 && gp1 < Ni);
#pragma unroll
      for (int n = 0; n < S::NB1; ++n) {
        const int b = tid + S::NT * n;
        if (b >= S::NBLK1) break;
        const int rp = b / S::SEG1, s = b - (b / S::SEG1) * S::SEG1;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          T val[4];
          const int64_t gj = ch.j0 - R + 2 * rp + p;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t gk = ch.k0 - 4 + 4 * s + e;
            const bool inside = periodic || (plane_in && gj >= 0 && gj < Nj && gk >= 0 && gk < Nk);
            val[e] = inside ? ring1[n][0][p][e] : T(0);
          }
          V* dv = reinterpret_cast<V*>(l1 + (2 * rp + p) * S::P1 + 4 + 4 * s);
#pragma unroll
          for (int m = 0; m < 4 / VEC; ++m) {
            V t4;
#pragma unroll
            for (int e = 0; e < VEC; ++e) t4[e] = val[VEC * m + e];
            dv[m] = t4;
          }
        }
      }
    }
#pragma unroll
    for (int n = 0; n < S::NB1; ++n) shift(ring1[n]);
    lds_barrier();  // level-1 plane p1 visible
    if (have1 && tid < 256) {  // level 2: the first four waves
      scatter(l1 + 2 * rp2 * S::P1 + 4 + 4 * q2, S::P1, ring2);
      // level-2 plane p1 - r = ib + u - 4r is complete
      if (u >= 4 * R) {
        const int64_t o = ch.ib + u - 4 * R;
        const int64_t gk = ch.k0 + 4 * q2;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int64_t gj = ch.j0 + 2 * rp2 + p;
          if (gj >= Nj || gk >= Nk) continue;  // Nk % 4 == 0: a 4-column block lies inside the row
          V* dst = reinterpret_cast<V*>(out + o * plane + gj * Nk + gk);
#pragma unroll
          for (int m = 0; m < 4 / VEC; ++m) {
            V t4;
#pragma unroll
            for (int e = 0; e < VEC; ++e) t4[e] = ring2[0][p][VEC * m + e];
            dst[m] = t4;
          }
        }
      }
      shift(ring2);
    }
  }
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__((Tb3Stream<T, R, BOX>::NT)) void tb3d_stream_kernel(KArgs a) {
  tb3d_stream_item<T, R, BOX>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__((Tb3Stream<T, R, BOX>::NT)) void tb3d_stream_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { tb3d_stream_item<T, R, BOX>(x, id); });
}

}  // namespace stencil
