// Asynchronous window loads for the 2D kernels (gfx950 direct-to-LDS).
//
// A workgroup walks a strip of TN columns in blocks of BM rows.  The input
// window of a block -- rows [ib - r, ib + BM + r), columns [j0 - 4, j0 + TN + 4)
// -- is copied from global memory straight into LDS with
// global_load_lds_dwordx4 (16 bytes per lane, 1 KiB per wave instruction, no
// registers), into one of two buffers, while the previous block is computed
// from the other buffer.  Wide strips keep every row segment a workgroup
// reads long and contiguous (TN = 256 FP32 or 128 FP64 columns: 1 KiB),
// which HBM serves far better than short scattered segments.  A 16-byte line
// holds 4 FP32 or 2 FP64 values.
//
// Every wave issues the same number of load instructions per window with all
// lanes active (lanes past the window end read a 16-byte zero line into slack
// at the end of the buffer), so "s_waitcnt vmcnt(n)" with n = the loads just
// issued for window b+1 guarantees that this wave's loads of window b (and
// its older stores) have completed; an LDS-only barrier then makes all
// waves' loads visible while window b+1 stays in flight.  Every window is
// loaded whole (BM + 2r rows); its 2r halo rows were read for the previous
// block moments before and come from L2, not HBM.
//
// Requirements (checked on the host before choosing these kernels): the
// column extent is a multiple of 4 and both grid pointers are 16-byte
// aligned, so every 16-byte line lies entirely inside or outside the grid and
// results can be stored as 16-byte rows.  Lines outside
// the grid come from the zero line (zero halo) or wrap (periodic).
#pragma once

#include "device_common.hpp"
#include "kernels_split2d.hpp"
#include "stream2d.hpp"

namespace stencil {

template <typename T, int R, int BM, int TN, int NT>
struct DmaWindow {
  typedef T elem_t;
  static constexpr int RAD = R;
  static constexpr int VEC = 16 / (int)sizeof(T);  // elements per 16-byte line
  static constexpr int PITCH = TN + 8;          // elements per LDS row: columns j0-4 .. j0+TN+3
  static constexpr int LPR = PITCH / VEC;       // 16-byte lines per row
  static constexpr int WCOL0 = 4 - R;           // LDS column of window column 0 (global j0 - r)
  static constexpr int ROWS = BM + 2 * R;
  static constexpr int NWAVES = NT / 64;
  // Load instructions per window (1 KiB each, all lanes active; lanes past
  // the window end read the zero line into the last instruction's tail),
  // spread round-robin over the waves: waves 0 .. NREM-1 issue NPW_FULL of
  // them, the others NPW_FULL - 1.  The buffer holds exactly NI instructions,
  // which keeps two of the largest windows (FP32 r = 4: 25 KiB each) small
  // enough for three workgroups per CU.
  static constexpr int NI = (ROWS * LPR + 63) / 64;
  static constexpr int NPW_FULL = (NI + NWAVES - 1) / NWAVES;
  static constexpr int NREM = NI - (NPW_FULL - 1) * NWAVES;
  static constexpr int BUF = NI * 64 * VEC;  // elements per buffer
  static_assert(R <= 4, "window covers at most 4 halo columns");
  static_assert(NPW_FULL < 64 && NPW_FULL >= 2, "vmcnt range");

  // Issue the loads of one window, global rows grow0 .. grow0 + ROWS - 1,
  // into the buffer at `dst`.
  static __device__ __forceinline__ void issue(T* dst, const T* __restrict__ src,
                                               const T* __restrict__ zeros, int64_t M, int64_t N,
                                               int64_t grow0, int64_t j0, bool periodic) {
    constexpr int LINES = ROWS * LPR;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NPW_FULL; ++k) {
      const int inst = k * NWAVES + w;
      if (inst >= NI) break;  // wave-uniform
      const int line = inst * 64 + lane;
      const T* s = zeros;
      if (line < LINES) {
        const int row = line / LPR, lc = line - (line / LPR) * LPR;
        const int64_t g = map_index(grow0 + row, M, periodic);
        const int64_t c = map_index(j0 - 4 + VEC * lc, N, periodic);
        if (g >= 0 && c >= 0) s = src + g * N + c;
      }
      __builtin_amdgcn_global_load_lds((const void*)s, (lds_void_t*)(dst + inst * 64 * VEC), 16, 0, 0);
    }
  }

  // After issuing window b+1: wait until this wave's loads of window b (and
  // everything older) have completed.
  static __device__ __forceinline__ void wait_previous() {
    if ((threadIdx.x >> 6) < NREM) wait_vm<NPW_FULL>();
    else wait_vm<NPW_FULL - 1>();
  }

  // s_waitcnt vmcnt(n): vmcnt[3:0] in bits 3:0, vmcnt[5:4] in bits 15:14;
  // expcnt (bits 6:4) and lgkmcnt (bits 11:8) left at their maxima.
  template <int n>
  static __device__ __forceinline__ void wait_vm() {
    __builtin_amdgcn_s_waitcnt((n & 0xf) | ((n >> 4) << 14) | (0x7 << 4) | (0xf << 8));
  }
};

// Default rows per work item of the direct-to-LDS kernels, from a sweep on
// MI355X (8192^2 FP32): short chunks keep many workgroups in flight, at the
// cost of 2r re-read halo rows per chunk, so the best length grows with r.
// Grids too small for ~2048 items of that length use shorter chunks (>= BM).
// kind: 0 star, 1 box (outer products and gather), 2 split-precision kernel
// (128-column strips: its per-block split pass favours long chunks).
inline int32_t dma_chunk(const KArgs& a, int TN, int R, int kind, int32_t chunk) {
  if (chunk > 0) return chunk;
  static const int32_t kBox[5] = {0, 16, 64, 64, 64}, kStar[5] = {0, 16, 16, 32, 64};
  const int64_t strips = (a.d1 + TN - 1) / TN;
  const int64_t fill = a.d0 * strips / 2048;
  const int64_t best = kind == 2 ? 128 : kind == 1 ? kBox[R] : kStar[R];
  return (int32_t)(fill < best ? (fill < 16 ? 16 : fill) : best);
}

// Host-side condition for the direct-to-LDS kernels.
inline bool dma2d_ok(const KArgs& a) {
  return a.d1 % 4 == 0 && (reinterpret_cast<uintptr_t>(a.in) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(a.out) & 15) == 0 && a.zeros != nullptr;
}

// Block loop shared by the DMA kernels: body(cur, ib) computes and stores the
// block of rows [ib, min(ib + BM, i1)) from the window in `cur` (window row 0
// = global row ib - r).  The loads of window b+1 (all BM + 2r rows; its 2r
// halo rows were just read for window b and come from L2) are issued before
// block b is computed.  Nothing else writes LDS inside the loop, so the
// compiler has no LDS store to order behind the loads in flight and the LDS
// barriers leave them outstanding across the compute of block b.
template <class D, int BM, class Body>
__device__ __forceinline__ void dma_block_loop(typename D::elem_t* bufs, const KArgs& a, const Strip2D& sp, Body body) {
  typedef typename D::elem_t T;
  constexpr int R = D::RAD;
  const T* __restrict__ in = (const T*)a.in;
  const T* __restrict__ zeros = (const T*)a.zeros;
  const bool periodic = a.periodic != 0;
  const int nb = (int)((sp.i1 - sp.i0 + BM - 1) / BM);
  D::issue(bufs, in, zeros, a.d0, a.d1, sp.i0 - R, sp.j0, periodic);
  for (int bi = 0; bi < nb; ++bi) {
    const int64_t ib = sp.i0 + (int64_t)bi * BM;
    T* cur = bufs + (bi & 1) * D::BUF;
    T* nxt = bufs + ((bi + 1) & 1) * D::BUF;
    if (bi + 1 < nb) {
      D::issue(nxt, in, zeros, a.d0, a.d1, ib + BM - R, sp.j0, periodic);
      D::wait_previous();
    } else {
      D::template wait_vm<0>();
    }
    lds_barrier();
    body(cur, ib);
    lds_barrier();
  }
}

// Block loop with one barrier per block, for kernels whose body issues NST
// store instructions per wave when the block is whole: wait for this wave's
// loads of window b (the stores of block b - 1, issued after them, may stay
// in flight), barrier (window b visible; every wave is past block b - 1,
// whose buffer then takes window b + 1), issue window b + 1, compute and
// store block b.  body(cur, ib) returns NST when all its stores were issued,
// else -1 (the next wait then waits for everything).
template <class D, int BM, int NST, class Body>
__device__ __forceinline__ void dma_block_loop1(typename D::elem_t* bufs, const KArgs& a, const Strip2D& sp, Body body) {
  typedef typename D::elem_t T;
  constexpr int R = D::RAD;
  const T* __restrict__ in = (const T*)a.in;
  const T* __restrict__ zeros = (const T*)a.zeros;
  const bool periodic = a.periodic != 0;
  const int nb = (int)((sp.i1 - sp.i0 + BM - 1) / BM);
  D::issue(bufs, in, zeros, a.d0, a.d1, sp.i0 - R, sp.j0, periodic);
  int pend = 0;
  for (int bi = 0; bi < nb; ++bi) {
    const int64_t ib = sp.i0 + (int64_t)bi * BM;
    T* cur = bufs + (bi & 1) * D::BUF;
    if (pend == NST) D::template wait_vm<NST>();
    else D::template wait_vm<0>();
    lds_barrier();
    if (bi + 1 < nb) D::issue(bufs + ((bi + 1) & 1) * D::BUF, in, zeros, a.d0, a.d1, ib + BM - R, sp.j0, periodic);
    pend = body(cur, ib);
  }
}

// ---------------------------------------------------------------------------
// n = 4 block outer products on DMA-fed windows.  Register tile (the i and j
// unrolling of Section 4.2): wave w owns 64 columns (lane 4 beta + j of block
// beta) and 4 UI rows (UI accumulators of 4 rows); the workgroup's four waves
// are WR rows x (4 / WR) columns of such tiles, so its strip is 256 / WR
// columns wide and its row block BM = 4 UI WR.  Default UI = 4, WR = 1:
// 256-column strips of 16-row blocks.  The input row segment is the MFMA A
// operand and the coefficient vector the B operand, so block beta of the
// instruction holds D[i][j] = input column 4 beta + i times the weight for
// block row j: lane 4 beta + j then owns four consecutive columns of one
// output row and stores them with one 16-byte write.
//
// Every block of the instruction uses the same B vector, so one VGPR carries
// four of them, one per 16-lane group, and the instruction's B lane-group
// broadcast (blgp = 4 + g: lanes 16 g .. 16 g + 15 feed all 16 blocks)
// selects one: the coefficient fragments take NL NB / 4 registers, not NL NB.
// ---------------------------------------------------------------------------
constexpr int kDmaTN = 256, kDmaBM = 16;

// Scheduling pattern of one line: X LDS reads, each followed by its share of
// the line's NM MFMAs (the group sizes must be constants, hence the recursion).
template <int X, int NM, int K = 0>
__device__ __forceinline__ void interleave_reads_mfma() {
  if constexpr (K < X) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                              // one LDS read
    __builtin_amdgcn_sched_group_barrier(0x008, (K + 1) * NM / X - K * NM / X, 0);  // MFMAs
    interleave_reads_mfma<X, NM, K + 1>();
  }
}

template <int R, bool BOX, int UI = 4, int WR = 1>
__device__ __forceinline__ void mfma2d_b4_dma_item(const KArgs& a, int item) {
  constexpr int NWC = 4 / WR, TN = 64 * NWC, BM = 4 * UI * WR;
  constexpr int NB = 4 + 2 * R, NL = BOX ? 2 * R + 1 : 1;
  constexpr int NC = NL * NB, NP = (NC + 3) / 4;  // coefficient vectors, packed registers
  static_assert(WR == 1 || WR == 2, "one or two rows of wave tiles");
  typedef DmaWindow<float, R, BM, TN, 256> D;
  __shared__ __attribute__((aligned(16))) float bufs[2 * D::BUF];

  const int64_t N = a.d1;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wc = w % NWC, wr = w / NWC;
  const Strip2D sp = decode_strip(a, item, TN);

  // vector c's value for lane l sits at frag[64 c + l] (it depends on l mod 4
  // only); register k holds vector 4 k + g in lane group g
  const float* __restrict__ frag = (const float*)a.frag;
  float af[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int c = 4 * k + (lane >> 4);
    af[k] = c < NC ? frag[c * 64 + lane] : 0.0f;
  }
  float cw[2 * R + 1];
  if constexpr (!BOX) {
    const float* __restrict__ c = (const float*)a.coef;
#pragma unroll
    for (int b = 0; b <= 2 * R; ++b) cw[b] = c[R * (2 * R + 1) + b];
  }
  const int orow = lane & 3;                             // block row owned by this lane
  const int64_t gj = sp.j0 + 64 * wc + 4 * (lane >> 2);  // first of its four columns
  const int row0 = 4 * UI * wr;                          // the wave's first row in the block

  dma_block_loop1<D, BM, UI>(bufs, a, sp, [&](const float* cur, int64_t ib) {
    const float* rowp = cur + row0 * D::PITCH + D::WCOL0 + 64 * wc + lane;
    floatx4 acc[UI];
#pragma unroll
    for (int s = 0; s < UI; ++s) acc[s] = floatx4{0, 0, 0, 0};
    // the window rows of line li + 1 are read while line li's MFMAs run (two
    // register sets), the reads spread evenly between the MFMAs
    constexpr int X = 4 * UI + 2 * R, NM = UI * NB;  // rows read and MFMAs per line
    float hv[2][X];
#pragma unroll
    for (int x = 0; x < X; ++x) hv[0][x] = rowp[x * D::PITCH + (BOX ? 0 : R)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int li = 0; li < NL; ++li) {
      if (li + 1 < NL) {
#pragma unroll
        for (int x = 0; x < X; ++x) hv[(li + 1) & 1][x] = rowp[x * D::PITCH + li + 1];
      }
#pragma unroll
      for (int x = 0; x < X; ++x)
#pragma unroll
        for (int s = 0; s < UI; ++s) {
          const int d = x - 4 * s, c = li * NB + d;
          if (d < 0 || d >= NB) continue;
          acc[s] = mfma4_group(hv[li & 1][x], af[c >> 2], acc[s], c & 3);
        }
      if (li + 1 < NL) interleave_reads_mfma<X, NM>();
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (!BOX) {
      // single-weight lines b != r: D[row][col] += C^g[r][b] * H[row + r][col + b]
#pragma unroll
      for (int s = 0; s < UI; ++s) {
        const float* rp = cur + (row0 + 4 * s + orow + R) * D::PITCH + D::WCOL0 + 64 * wc + 4 * (lane >> 2);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float sum = 0.0f;
#pragma unroll
          for (int b = 0; b <= 2 * R; ++b) {
            if (b == R) continue;
            sum += cw[b] * rp[v + b];
          }
          acc[s][v] += sum;
        }
      }
    }
    if (gj < N) {
#pragma unroll
      for (int s = 0; s < UI; ++s) {
        const int64_t gi = ib + row0 + 4 * s + orow;
        if (gi < sp.i1) *reinterpret_cast<float4*>(out + gi * N + gj) = float4{acc[s][0], acc[s][1], acc[s][2], acc[s][3]};
      }
    }
    // all UI stores issued: the wave's columns lie inside the grid and its rows inside the block
    return (sp.j0 + 64 * wc + 64 <= N && ib + row0 + 4 * UI <= sp.i1) ? UI : -1;
  });
}

template <int R, bool BOX, int UI = 4, int WR = 1>
__global__ __launch_bounds__(256) void mfma2d_b4_dma_kernel(KArgs a) {
  mfma2d_b4_dma_item<R, BOX, UI, WR>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int R, bool BOX, int UI = 4, int WR = 1>
__global__ __launch_bounds__(256) void mfma2d_b4_dma_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { mfma2d_b4_dma_item<R, BOX, UI, WR>(x, id); });
}

// ---------------------------------------------------------------------------
// n = 4 blocks over a minimum line cover of any C^g (Section 3.5): up to 2r+1
// slots, each a line along i (C^g column b, as above) or along j (C^g row a).
// A line along j uses the same accumulator layout: for window column offset
// e = 0 .. 3 + 2r, lane 4 beta + i supplies the band value w[e - i] (the A
// operand, packed like a column line's) and lane 4 beta + j the input
// H[4 s + j + a][4 beta + e], so block beta accumulates output (row 4 s + j,
// column 4 beta + i) += w[e - i] * input (row + a - r, column + e - i - r).
// Slot kinds and indices: KArgs.lcode0 / lcode1.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void mfma2d_b4c_dma_item(const KArgs& a, int item) {
  constexpr int BM = kDmaBM, TN = kDmaTN, NB = 4 + 2 * R, W = 2 * R + 1;
  typedef DmaWindow<float, R, BM, TN, 256> D;
  __shared__ __attribute__((aligned(16))) float bufs[2 * D::BUF];

  const int64_t N = a.d1;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const Strip2D sp = decode_strip(a, item, TN);
  // band vectors packed four to a register (lane group g holds vector 4 k + g),
  // selected by the B lane-group broadcast (lines along i) or the A block
  // broadcast (lines along j)
  constexpr int NC = W * NB, NP = (NC + 3) / 4;
  const float* __restrict__ frag = (const float*)a.frag;
  float af[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int c = 4 * k + (lane >> 4);
    af[k] = c < NC ? frag[c * 64 + lane] : 0.0f;
  }
  const int nlines = (a.lcode1 >> 27) & 15;
  const int orow = lane & 3;
  const int64_t gj = sp.j0 + 64 * w + 4 * (lane >> 2);

  dma_block_loop<D, BM>(bufs, a, sp, [&](const float* cur, int64_t ib) {
    floatx4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = floatx4{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < W; ++k) {
      if (k >= nlines) break;
      const int code = k < 6 ? (a.lcode0 >> (5 * k)) & 31 : (a.lcode1 >> (5 * (k - 6))) & 31;
      const int idx = code & 15;
      if ((code & 16) == 0) {
        const float* rowp = cur + D::WCOL0 + 64 * w + lane + idx;
#pragma unroll
        for (int x = 0; x < 16 + 2 * R; ++x) {
          const float hv = rowp[x * D::PITCH];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int d = x - 4 * s;
            if (d < 0 || d >= NB) continue;
            const int c = k * NB + d;
            acc[s] = mfma4_group(hv, af[c >> 2], acc[s], c & 3);
          }
        }
      } else {
        const float* colp = cur + (orow + idx) * D::PITCH + D::WCOL0 + 64 * w + 4 * (lane >> 2);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int e = 0; e < NB; ++e)
            acc[s] = mfma4_agroup(af[(k * NB + e) >> 2], colp[4 * s * D::PITCH + e], acc[s], (k * NB + e) & 3);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (gj < N) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t gi = ib + 4 * s + orow;
        if (gi < sp.i1) *reinterpret_cast<float4*>(out + gi * N + gj) = float4{acc[s][0], acc[s][1], acc[s][2], acc[s][3]};
      }
    }
  });
}

template <int R>
__global__ __launch_bounds__(256) void mfma2d_b4c_dma_kernel(KArgs a) {
  mfma2d_b4c_dma_item<R>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int R>
__global__ __launch_bounds__(256) void mfma2d_b4c_dma_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { mfma2d_b4c_dma_item<R>(x, id); });
}

// ---------------------------------------------------------------------------
// Gather-form baseline on DMA-fed windows: strips of 256 (FP32) or 128 (FP64)
// columns; thread t owns a block of 4 (FP32) or 2 (FP64) rows x 4 columns,
// reads each input row it needs as 12 values (three 16-byte LDS vectors FP32,
// six FP64) covering the column offsets -r .. r of its four columns, applies
// the taps with wave-uniform coefficients and stores 16-byte rows.
// ---------------------------------------------------------------------------
template <typename T> struct Gather2DDma;
template <> struct Gather2DDma<float> { static constexpr int TN = 256; };
template <> struct Gather2DDma<double> { static constexpr int TN = 128; };

template <typename T, int R, bool BOX>
__device__ __forceinline__ void gather2d_dma_item(const KArgs& a, int item) {
  constexpr int BM = kDmaBM, TN = Gather2DDma<T>::TN, W = 2 * R + 1;
  constexpr int CT = TN / 4, NRG = 256 / CT, PR = BM / NRG;  // column groups, row groups, rows per thread
  typedef DmaWindow<T, R, BM, TN, 256> D;
  typedef typename Vec16<T>::type V;
  constexpr int VEC = D::VEC;
  constexpr int XU = BOX && (sizeof(T) == 8 || R >= 3) ? 2 : 0;  // unroll of the middle rows (0: all)
  __shared__ __attribute__((aligned(16))) T bufs[2 * D::BUF];

  const int64_t N = a.d1;
  T* __restrict__ out = (T*)a.out;
  const ConstPtr<T> c = (ConstPtr<T>)a.coef;  // uniform reads: scalar loads
  const int rg = threadIdx.x / CT, c4 = 4 * (threadIdx.x % CT);
  const Strip2D sp = decode_strip(a, item, TN);
  const int64_t gj = sp.j0 + c4;

  dma_block_loop<D, BM>(bufs, a, sp, [&](const T* cur, int64_t ib) {
    T acc[PR][4];
#pragma unroll
    for (int p = 0; p < PR; ++p)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) acc[p][qq] = T(0);
    // window row x feeds output rows p with coefficient row x - p; `edge`
    // rows (the first and last PR - 1) have some p out of range
    auto row = [&](int x, auto edge) {
      // LDS columns c4 .. c4 + 11 hold window columns c4 - 4 + r .. c4 + 7 + r
      const V* rp = reinterpret_cast<const V*>(cur + (PR * rg + x) * D::PITCH + c4);
      T vv[12];
      if constexpr (sizeof(T) == 4 && R < 4) {
        // FP32 below r = 4: a row uses 4 + 2r of the 12 columns (a star row
        // off every output row's centre only the middle four), and a partly
        // used 16-byte vector would be narrowed into 4- or 8-byte reads that
        // meet a quarter or half of the banks at this 16-byte lane stride;
        // the empty asm keeps the vector whole
        const bool full = BOX || (x >= R && x < R + PR);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (!full && k != 1) continue;
          floatx4 t4 = reinterpret_cast<const floatx4*>(rp)[k];
          asm volatile("" : "+v"(t4));
#pragma unroll
          for (int e = 0; e < 4; ++e) vv[4 * k + e] = t4[e];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 12 / VEC; ++k) {
          const V t = rp[k];
          const T* pt = reinterpret_cast<const T*>(&t);
#pragma unroll
          for (int e = 0; e < VEC; ++e) vv[k * VEC + e] = pt[e];
        }
      }
#pragma unroll
      for (int p = 0; p < PR; ++p) {
        const int aa = x - p;
        if constexpr (decltype(edge)::value) {
          if (aa < 0 || aa > 2 * R) continue;
        }
#pragma unroll
        for (int b = 0; b < W; ++b) {
          if (!BOX && aa != R && b != R) continue;
          const T cf = c[aa * W + b];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) acc[p][qq] += cf * vv[D::WCOL0 + qq + b];
        }
      }
    };
    if constexpr (XU == 0) {  // fully unrolled: every row index a constant
#pragma unroll
      for (int x = 0; x < PR + 2 * R; ++x) row(x, std::true_type{});
    } else {  // large boxes: a rolled middle keeps registers and scalar coefficients in budget
      static_assert(PR - 1 <= 2 * R + 1, "edge rows overlap");
#pragma unroll
      for (int x = 0; x < PR - 1; ++x) row(x, std::true_type{});
#pragma unroll XU
      for (int x = PR - 1; x <= 2 * R; ++x) row(x, std::false_type{});
#pragma unroll
      for (int x = 2 * R + 1; x < PR + 2 * R; ++x) row(x, std::true_type{});
    }
    if (gj < N) {  // column extent a multiple of 4: the four columns lie inside the row
#pragma unroll
      for (int p = 0; p < PR; ++p) {
        const int64_t gi = ib + PR * rg + p;
        if (gi >= sp.i1) continue;
        V* dst = reinterpret_cast<V*>(out + gi * N + gj);
#pragma unroll
        for (int k = 0; k < 4 / VEC; ++k) {
          V t;
          T* pt = reinterpret_cast<T*>(&t);
#pragma unroll
          for (int e = 0; e < VEC; ++e) pt[e] = acc[p][k * VEC + e];
          dst[k] = t;
        }
      }
    }
  });
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__(256) void gather2d_dma_kernel(KArgs a) {
  gather2d_dma_item<T, R, BOX>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__(256) void gather2d_dma_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { gather2d_dma_item<T, R, BOX>(x, id); });
}

// ---------------------------------------------------------------------------
// Split-precision outer products on DMA-fed FP32 windows: 128-column strips,
// 16-row blocks, wave w owns columns 32 w .. 32 w + 31 (two 16 x 16 blocks).
// After a window lands, one pass splits it into the hi/lo 16-bit LDS planes.
// The band is the MFMA A operand and the input the B operand, so
// D[m][n] = sum_y S_a[y][m] H[n + a][y]: lane l holds output row l % 16 and
// four consecutive columns, stored with one 16-byte write.
// ---------------------------------------------------------------------------
constexpr int kSplitTN = 128;

template <int KIND, int R>
__device__ __forceinline__ void split2d_dma_item(const KArgs& a, int item) {
  constexpr int NL = 2 * R + 1, BM = kDmaBM, TN = kSplitTN;
  constexpr int WROWS = BM + 2 * R, WEND = TN + 2 * R;
  constexpr int P = 152;  // 16-bit pitch: multiple of 8, odd number of 16-byte units, >= 96 + 16 + 32
  static_assert(WEND <= P && 32 * 3 + 16 + 32 <= P, "pitch too small");
  typedef DmaWindow<float, R, BM, TN, 256> D;
  // one LDS object (separate ones make the compiler wait for the window in
  // flight before LDS accesses): the two windows, then the hi and lo planes
  constexpr int PLANE = (WROWS * P * 2 + 15) / 16 * 4;  // floats per 16-bit plane, 16-byte multiple
  __shared__ __attribute__((aligned(16))) float bufs[2 * D::BUF + 2 * PLANE];
  uint16_t* lhi = reinterpret_cast<uint16_t*>(bufs + 2 * D::BUF);
  uint16_t* llo = reinterpret_cast<uint16_t*>(bufs + 2 * D::BUF + PLANE);

  const int64_t N = a.d1;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, q = lane & 15;
  const Strip2D sp = decode_strip(a, item, TN);

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
    lds_barrier();
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
        acc[t] = Split16<KIND>::mma(bh[l], ah, acc[t]);
        acx[t] = Split16<KIND>::mma(bl[l], ah, acx[t]);
        acx[t] = Split16<KIND>::mma(bh[l], al, acx[t]);
      }
    }
    const int64_t gi = ib + q;
    if (gi < sp.i1) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int64_t gj = sp.j0 + 32 * w + 16 * t + 4 * g;
        if (gj < N)
          *reinterpret_cast<float4*>(out + gi * N + gj) =
              float4{(acc[t][0] + ls * acx[t][0]) * os, (acc[t][1] + ls * acx[t][1]) * os,
                     (acc[t][2] + ls * acx[t][2]) * os, (acc[t][3] + ls * acx[t][3]) * os};
      }
    }
  });
}

template <int KIND, int R>
__global__ __launch_bounds__(256) void split2d_dma_kernel(KArgs a) {
  split2d_dma_item<KIND, R>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int KIND, int R>
__global__ __launch_bounds__(256) void split2d_dma_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { split2d_dma_item<KIND, R>(x, id); });
}

}  // namespace stencil
