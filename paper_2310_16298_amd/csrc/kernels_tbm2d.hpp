// Two Jacobi steps per launch on the n = 4 box outer products (FP32, 2D).
//
// The one-step kernel (mfma2d_b4_dma_item) spends its launch on the matrix
// work and on the grid's HBM traffic one after the other; here the traffic
// of two steps is paid once.  A workgroup walks a chunk of rows down a strip
// of 256 computed columns in blocks of 16 rows:
//
//   level 1  the outer products of the block's direct-to-LDS input window
//            give 16 rows of the intermediate state (step 1) for all 256
//            columns; they are masked to zero outside a zero-halo grid and
//            written to an LDS plane laid out like an input window;
//   level 2  the same outer products over that plane (the 2r rows above the
//            block's 16 come from the previous level-1 block) give 16 output
//            rows of step 2.
//
// Level-1 rows run r ahead of level-2 rows, so a chunk starts with one
// level-1 block of warm-up.  Level 2 at a column needs step-1 values r
// columns either side, which exist inside the 256 computed columns only: the
// strips therefore overlap, each storing its inner 248 columns (the first and
// last 4-column groups are recomputed by the neighbours).  Two level-1 planes
// alternate: block k goes to plane k mod 2 (rows 2r ..) and its last 2r rows
// also to the head of plane (k + 1) mod 2, where level 2 of block k reads
// them as the rows above block k + 1.  Both levels run the one-step kernel's
// MFMA sequence, so a launch equals two one-step launches bit for bit.
#pragma once

#include "dma2d.hpp"
#include "launch.hpp"
#include "stream2d.hpp"

namespace stencil {

constexpr int kTbmStride = 248;  // stored columns per strip (256 computed)

template <int R>
struct TbmShape {
  static constexpr int UI = 4, BM = 16, TN = 256;
  static constexpr int NB = 4 + 2 * R, NL = 2 * R + 1, NC = NL * NB, NP = (NC + 3) / 4;
  static constexpr int X = BM + 2 * R;  // rows one line reads
  typedef DmaWindow<float, R, BM, TN, 256> D;
  static constexpr int PITCH = D::PITCH;
  static constexpr int PLANE = X * PITCH;  // a level-1 plane: rows ib - r .. ib + BM + r - 1
  static_assert(2 * R <= BM, "the rows above a block come from one level-1 block");
  static_assert(TN - kTbmStride == 8, "each strip drops one 4-column group at either edge");
};

// acc[s] (rows row0 + 4 s .., lane's four columns) = the outer products of
// a window-layout buffer `src` (row 0 = the block's first row minus r,
// LDS column D::WCOL0 + c = strip column c - r), the one-step kernel's
// order: lines li = 0 .. 2r, rows x, accumulator blocks s.
template <int R>
__device__ __forceinline__ void tbm_outer_products(const float* src, const float* af, int row0, int wc, int lane,
                                                   floatx4* acc) {
  typedef TbmShape<R> S;
  constexpr int X = S::X, NB = S::NB, NL = S::NL, UI = S::UI, NM = UI * NB;
  const float* rowp = src + row0 * S::PITCH + S::D::WCOL0 + 64 * wc + lane;
#pragma unroll
  for (int s = 0; s < UI; ++s) acc[s] = floatx4{0, 0, 0, 0};
  float hv[2][X];
#pragma unroll
  for (int x = 0; x < X; ++x) hv[0][x] = rowp[x * S::PITCH];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int li = 0; li < NL; ++li) {
    if (li + 1 < NL) {
#pragma unroll
      for (int x = 0; x < X; ++x) hv[(li + 1) & 1][x] = rowp[x * S::PITCH + li + 1];
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
}

template <int R>
__device__ __forceinline__ void tbm2d_item(const KArgs& a, int item) {
  typedef TbmShape<R> S;
  typedef typename S::D D;
  constexpr int UI = S::UI, BM = S::BM, NC = S::NC, NP = S::NP, PITCH = S::PITCH;
  __shared__ __attribute__((aligned(16))) float win[D::BUF];
  __shared__ __attribute__((aligned(16))) float l1[2 * S::PLANE];

  const int64_t M = a.d0, N = a.d1;
  const bool periodic = a.periodic != 0;
  const float* __restrict__ in = (const float*)a.in;
  const float* __restrict__ zeros = (const float*)a.zeros;
  float* __restrict__ out = (float*)a.out;
  const int tid = threadIdx.x, lane = tid & 63, wc = tid >> 6;
  const Strip2D sp = decode_strip(a, item, kTbmStride);
  const int64_t j0 = sp.j0 - 4;  // first computed column

  // the planes' edge columns (strip columns -4 .. -1 and 256 .. 259) are
  // never written: zero, so the outputs next to them (not stored) stay finite
  for (int e = tid; e < 2 * S::PLANE; e += 256) l1[e] = 0.0f;

  const float* __restrict__ frag = (const float*)a.frag;
  float af[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int c = 4 * k + (lane >> 4);
    af[k] = c < NC ? frag[c * 64 + lane] : 0.0f;
  }
  const int orow = lane & 3;                          // block row owned by this lane
  const int64_t gj = j0 + 64 * wc + 4 * (lane >> 2);  // first of its four columns
  // columns this lane may store: inside the strip's 248 and the grid
  const bool store_cols = gj >= sp.j0 && gj < sp.j0 + kTbmStride && gj < N;
  bool col_in[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) col_in[v] = periodic || (gj + v >= 0 && gj + v < N);

  const int nb = (int)((sp.i1 - sp.i0 + BM - 1) / BM);  // level-2 blocks
  // level-1 block k: rows g_k = i0 - BM + r + BM k .. + BM - 1; its input
  // window starts at row g_k - r
  D::issue(win, in, zeros, M, N, sp.i0 - BM, j0, periodic);
  int pend = 0;  // store instructions this wave issued after the loads in flight
  for (int k = 0; k <= nb; ++k) {
    if (pend == UI) D::template wait_vm<UI>();
    else D::template wait_vm<0>();
    lds_barrier();  // window k visible; every wave is past level 2 of block k - 2
    floatx4 acc[UI];
    tbm_outer_products<R>(win, af, 0, wc, lane, acc);
    // step-1 rows g_k + 4 s + orow: zero outside a zero-halo grid; plane k & 1
    // rows 2r + (4 s + orow), and the last 2r rows also plane (k + 1) & 1 rows
    // 4 s + orow - (BM - 2r)
    const int64_t gk = sp.i0 - BM + R + (int64_t)BM * k;
    float* const pk = l1 + (k & 1) * S::PLANE;
    float* const pn = l1 + ((k + 1) & 1) * S::PLANE;
#pragma unroll
    for (int s = 0; s < UI; ++s) {
      const int t = 4 * s + orow;
      const int64_t gi = gk + t;
      const bool row_in = periodic || (gi >= 0 && gi < M);
      float4 v;
      v.x = row_in && col_in[0] ? acc[s][0] : 0.0f;
      v.y = row_in && col_in[1] ? acc[s][1] : 0.0f;
      v.z = row_in && col_in[2] ? acc[s][2] : 0.0f;
      v.w = row_in && col_in[3] ? acc[s][3] : 0.0f;
      const int col = 4 + 64 * wc + 4 * (lane >> 2);  // LDS column of strip column 64 wc + 4 (lane / 4)
      *reinterpret_cast<float4*>(pk + (2 * R + t) * PITCH + col) = v;
      if (t >= BM - 2 * R) *reinterpret_cast<float4*>(pn + (t - (BM - 2 * R)) * PITCH + col) = v;
    }
    lds_barrier();  // plane k & 1 complete; every wave is done with window k
    if (k < nb) D::issue(win, in, zeros, M, N, sp.i0 + (int64_t)BM * k, j0, periodic);
    pend = -1;
    if (k == 0) continue;  // warm-up block: level 1 only
    // level 2: output block b = k - 1, rows ib .. ib + BM - 1, from the plane
    // whose rows are step-1 rows ib - r .. ib + BM + r - 1
    const int64_t ib = sp.i0 + (int64_t)BM * (k - 1);
    tbm_outer_products<R>(pk, af, 0, wc, lane, acc);
    if (store_cols) {
#pragma unroll
      for (int s = 0; s < UI; ++s) {
        const int64_t gi = ib + 4 * s + orow;
        if (gi < sp.i1) *reinterpret_cast<float4*>(out + gi * N + gj) = float4{acc[s][0], acc[s][1], acc[s][2], acc[s][3]};
      }
    }
    // the wave issued UI store instructions when the block is whole and one
    // of its lanes stores: every wave's columns meet the strip's stored
    // range, so that lane exists unless the first of them is past the grid
    const int64_t first = j0 + 64 * wc > sp.j0 ? j0 + 64 * wc : sp.j0;
    pend = (ib + BM <= sp.i1 && first < N) ? UI : -1;
  }
}

template <int R>
__global__ __launch_bounds__(256) void tbm2d_kernel(KArgs a) {
  tbm2d_item<R>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int R>
__global__ __launch_bounds__(256) void tbm2d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { tbm2d_item<R>(x, id); });
}

}  // namespace stencil
