// 2D stencil kernels: the gather-form baseline and the outer-product form on
// MFMA in the grid dtype (FP32 or FP64).
//
// Both walk a 64-column strip in blocks of 64 rows (four waves per
// workgroup), stream the input rows through an LDS window with an r-wide
// halo (stream2d.hpp), and differ only in how each block's sum is formed.
#pragma once

#include "device_common.hpp"
#include "mfma_traits.hpp"
#include "stream2d.hpp"

namespace stencil {

enum Variant2D { VAR_BOX = 0, VAR_STAR_PARALLEL = 1, VAR_STAR_ORTHO = 2, VAR_COVER = 3 };

constexpr int kTile2D = 64;   // output tile edge of one workgroup
constexpr int kThreads = 256; // four waves

// LDS pitch (elements) with a bank-friendly residue.
template <typename T, bool ROWREAD>
__host__ __device__ constexpr int pick_pitch(int cols) {
  // FP32: 16 lanes read 16 consecutive words of one row and the next 16 lanes
  // the next row, so rows offset by half the banks avoid conflicts; when
  // lanes also walk down a column (row-line reads), an odd residue spreads them.
  constexpr int mod = sizeof(T) == 4 ? 32 : 16;
  constexpr int res = sizeof(T) == 4 ? (ROWREAD ? 17 : 16) : (ROWREAD ? 9 : 8);
  int p = cols;
  while (p % mod != res) ++p;
  return p;
}

// ---------------------------------------------------------------------------
// Gather-form baseline (Section 3.2, Eq. (1)): each thread owns a 16-row strip
// of one column and slides a register window down the LDS tile; coefficient
// reads are wave-uniform (scalar loads).  Box: all (2r+1)^2 taps; star: the
// on-axis taps only.
// ---------------------------------------------------------------------------
template <typename T, int R, bool BOX>
__device__ __forceinline__ void gather2d_item(const KArgs& a, int item) {
  constexpr int BM = kTile2D, TN = kTile2D, W = 2 * R + 1;
  constexpr int WROWS = BM + 2 * R, WCOLS = TN + 2 * R;
  constexpr int COL0 = lds_col0<T, R>();
  constexpr int PITCH = pick_pitch<T, false>(COL0 + WCOLS);
  constexpr int STRIP = 16;
  __shared__ __attribute__((aligned(16))) T lds[WROWS * PITCH];

  const int64_t M = a.d0, N = a.d1;
  const bool periodic = a.periodic != 0;
  const T* __restrict__ in = (const T*)a.in;
  T* __restrict__ out = (T*)a.out;
  const Strip2D sp = decode_strip(a, item, TN);
  const bool fast = strip_fast(in, N, sp.j0, TN);
  PlainWriter<T, R, PITCH> wr{lds};
  stage_window<T, R, WROWS, TN, PITCH, kThreads>(lds, in, M, N, sp.i0 - R, sp.j0, periodic);
  __syncthreads();

  const T* __restrict__ c = (const T*)a.coef;
  const int q = threadIdx.x & 63;  // column within the strip
  const int s = threadIdx.x >> 6;  // rows 16 s .. 16 s + 15 of each block
  const T* base = lds + (STRIP * s) * PITCH + COL0 + q;
  RowPrefetch<T, R, BM, TN, kThreads> pf;
  RowMover<T, R, WCOLS, kThreads> mv;
  for (int64_t ib = sp.i0; ib < sp.i1; ib += BM) {
    const bool more = ib + BM < sp.i1;
    if (more) pf.fetch(in, M, N, ib + BM + R, sp.j0, periodic, fast);
    T acc[STRIP];
#pragma unroll
    for (int p = 0; p < STRIP; ++p) acc[p] = T(0);
#pragma unroll
    for (int x = 0; x < STRIP + 2 * R; ++x) {
      T h[W];
#pragma unroll
      for (int b = 0; b < W; ++b) h[b] = base[x * PITCH + b];
#pragma unroll
      for (int p = 0; p < STRIP; ++p) {
        const int aa = x - p;  // input row x reaches output row p through C^g[x-p][.]
        if (aa < 0 || aa > 2 * R) continue;
#pragma unroll
        for (int b = 0; b < W; ++b) {
          if (!BOX && aa != R && b != R) continue;
          acc[p] += c[aa * W + b] * h[b];
        }
      }
    }
    const int64_t gj = sp.j0 + q;
#pragma unroll
    for (int p = 0; p < STRIP; ++p) {
      const int64_t gi = ib + STRIP * s + p;
      if (gi < sp.i1 && gj < N) out[gi * N + gj] = acc[p];
    }
    if (more) mv.load([&](int rr, int cc) { return lds[(BM + rr) * PITCH + COL0 + cc]; });
    __syncthreads();
    if (more) {
      mv.store([&](int rr, int cc, T v) { lds[rr * PITCH + COL0 + cc] = v; });
      pf.commit(2 * R, wr);
    }
    __syncthreads();
  }
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__(kThreads) void gather2d_kernel(KArgs a) {
  gather2d_item<T, R, BOX>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__(kThreads) void gather2d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { gather2d_item<T, R, BOX>(x, id); });
}

// ---------------------------------------------------------------------------
// Outer-product form on MFMA (Section 3.2, Eq. (7)-(12); Section 3.3 for star
// stencils; Table 1 for the line options).
//
// Each wave owns a 16-row x 64-column strip of the tile = four 16x16 output
// blocks held in MFMA accumulators.  A coefficient line along i (C^g column b)
// is the band T_b[p][x] = C^g[x-p][b] (the zero-padded vectors of Eq. (9)-
// (11)); the rank-1 updates of Eq. (12) for that line are
//      D[p][q] += sum_x T_b[p][x] * H[x][q + b]
// with H the halo'd input window: MFMA A operand = band (kept in VGPRs for
// the whole kernel), B operand = one LDS row segment per K row, read with an
// immediate offset.  One band fragment feeds the four blocks of the strip.
//
// VAR_BOX:           2r+1 lines along i (all columns of C^g).
// VAR_STAR_PARALLEL: the centre line b = r on MFMA; the 2r single-weight lines
//                    are scalar-times-vector updates, done as vector FMAs.
// VAR_STAR_ORTHO:    the centre line along i on MFMA, plus the line along j
//                    (C^g row r, centre excluded) in the transposed form
//                    D[p][q] += sum_y H[p + r][y] * S[y][q], S[y][q] = C^g[r][y-q]
//                    (Eq. (14)): the input column segment is the A operand.
// VAR_COVER:         any C^g (Section 3.5): up to 2r+1 lines of a minimum
//                    axis-parallel cover, each along i (C^g column b, first
//                    form) or along j (C^g row a, second form); the slot
//                    kinds and indices come from KArgs.lcode0 / lcode1.
// K is padded to a multiple of 4 per line; padded rows carry zero weights.
// ---------------------------------------------------------------------------
template <typename T, int R, int VAR>
struct Mfma2DShape {
  static constexpr int KL = round_up(16 + 2 * R, 4);   // K rows per line incl. padding
  static constexpr int CPL = KL / 4;                    // MFMA chunks per line
  static constexpr int NLC = (VAR == VAR_BOX || VAR == VAR_COVER) ? 2 * R + 1 : 1;
  static constexpr int NLR = VAR == VAR_STAR_ORTHO ? 1 : 0;
  static constexpr bool ROWREAD = VAR == VAR_STAR_ORTHO || VAR == VAR_COVER;  // lines along j read columns
  static constexpr int NCH = (NLC + NLR) * CPL;         // band fragments per lane
  static constexpr int TM = kTile2D, TN = kTile2D;
  static constexpr int WROWS = TM + 2 * R;
  static constexpr int LROWS = TM - 16 + KL;            // rows touched by padded K reads
  static constexpr int COL0 = lds_col0<T, R>();
  static constexpr int WEND = COL0 + TN + 2 * R;        // one past the window's last column
  static constexpr int REND = COL0 + (TN - 16) + KL;    // one past the row-line reads' last column
  static constexpr int LCOLS = cmax(WEND, ROWREAD ? REND : 0);
  static constexpr int PITCH = pick_pitch<T, ROWREAD>(LCOLS);
};

template <typename T, int R, int VAR>
__device__ __forceinline__ void mfma2d_item(const KArgs& a, int item) {
  typedef Mfma16<T> MM;
  typedef typename MM::acc_t acc_t;
  typedef Mfma2DShape<T, R, VAR> S;
  constexpr int BM = S::TM, WCOLS = S::TN + 2 * R;
  __shared__ __attribute__((aligned(16))) T lds[S::LROWS * S::PITCH];

  const int64_t M = a.d0, N = a.d1;
  const bool periodic = a.periodic != 0;
  const T* __restrict__ in = (const T*)a.in;
  T* __restrict__ out = (T*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, q = lane & 15;
  const Strip2D sp = decode_strip(a, item, S::TN);
  const bool fast = strip_fast(in, N, sp.j0, S::TN);

  // Band fragments for this lane (packed by the plan in lane order).
  const T* __restrict__ frag = (const T*)a.frag;
  T af[S::NCH];
#pragma unroll
  for (int c = 0; c < S::NCH; ++c) af[c] = frag[c * 64 + lane];
  T cw[2 * R + 1];  // parallel star: single-weight lines C^g[r][b]
  if constexpr (VAR == VAR_STAR_PARALLEL) {
    const T* __restrict__ c = (const T*)a.coef;
#pragma unroll
    for (int b = 0; b <= 2 * R; ++b) cw[b] = c[R * (2 * R + 1) + b];
  }

  if constexpr (S::LROWS > S::WROWS)
    zero_region<T, kThreads>(lds, S::LROWS - S::WROWS, S::PITCH, S::PITCH, S::WROWS, 0);
  if constexpr (S::LCOLS > S::WEND)
    zero_region<T, kThreads>(lds, S::WROWS, S::LCOLS - S::WEND, S::PITCH, 0, S::WEND);
  stage_window<T, R, S::WROWS, S::TN, S::PITCH, kThreads>(lds, in, M, N, sp.i0 - R, sp.j0, periodic);
  __syncthreads();

  PlainWriter<T, R, S::PITCH> wr{lds};
  RowPrefetch<T, R, BM, S::TN, kThreads> pf;
  RowMover<T, R, WCOLS, kThreads> mv;
  // Lines along i: B operand row x = 4 cc + g of the wave's window rows.
  const T* colbase = lds + (16 * w + g) * S::PITCH + S::COL0 + q;
  const T* rowbase = lds + (16 * w + R + q) * S::PITCH + S::COL0 + g;
  for (int64_t ib = sp.i0; ib < sp.i1; ib += BM) {
    const bool more = ib + BM < sp.i1;
    if (more) pf.fetch(in, M, N, ib + BM + R, sp.j0, periodic, fast);
    acc_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = acc_t{};
    if constexpr (VAR != VAR_COVER) {
#pragma unroll
      for (int li = 0; li < S::NLC; ++li) {
        const int b = VAR == VAR_BOX ? li : R;
#pragma unroll
        for (int cc = 0; cc < S::CPL; ++cc) {
          const T av = af[li * S::CPL + cc];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const T bv = colbase[(4 * cc) * S::PITCH + 16 * t + b];
            acc[t] = MM::mma(av, bv, acc[t]);
          }
        }
      }
    } else {
      const int nlines = (a.lcode1 >> 27) & 15;
#pragma unroll
      for (int k = 0; k < S::NLC; ++k) {
        if (k >= nlines) break;
        const int code = k < 6 ? (a.lcode0 >> (5 * k)) & 31 : (a.lcode1 >> (5 * (k - 6))) & 31;
        const int idx = code & 15;
        if ((code & 16) == 0) {
          // line along i, C^g column idx: A = band, B = input row segment shifted by idx
#pragma unroll
          for (int cc = 0; cc < S::CPL; ++cc) {
            const T av = af[k * S::CPL + cc];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = MM::mma(av, colbase[(4 * cc) * S::PITCH + 16 * t + idx], acc[t]);
          }
        } else {
          // line along j, C^g row idx: A = input column segment of rows shifted by idx, B = band
          const T* rb = lds + (16 * w + idx + q) * S::PITCH + S::COL0 + g;
#pragma unroll
          for (int cc = 0; cc < S::CPL; ++cc) {
            const T sv = af[k * S::CPL + cc];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = MM::mma(rb[16 * t + 4 * cc], sv, acc[t]);
          }
        }
      }
    }
    if constexpr (VAR == VAR_STAR_ORTHO) {
      // Line along j: A operand = input column segment H[r + p][y], y = 4 cc + g.
#pragma unroll
      for (int cc = 0; cc < S::CPL; ++cc) {
        const T sv = af[S::NLC * S::CPL + cc];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const T hv = rowbase[16 * t + 4 * cc];
          acc[t] = MM::mma(hv, sv, acc[t]);
        }
      }
    }
    if constexpr (VAR == VAR_STAR_PARALLEL) {
      // Single-weight lines b != r: D[p][q] += C^g[r][b] * H[p + r][q + b].
      const int col = MM::col(lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T* rp = lds + (16 * w + R + MM::row(lane, v)) * S::PITCH + S::COL0 + col;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          T sum = T(0);
#pragma unroll
          for (int b = 0; b <= 2 * R; ++b) {
            if (b == R) continue;
            sum += cw[b] * rp[16 * t + b];
          }
          acc[t][v] += sum;
        }
      }
    }
    const int64_t gj = sp.j0 + MM::col(lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = ib + 16 * w + MM::row(lane, v);
      if (gi >= sp.i1) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (gj + 16 * t < N) out[gi * N + gj + 16 * t] = acc[t][v];
      }
    }
    if (more) mv.load([&](int rr, int cc) { return lds[(BM + rr) * S::PITCH + S::COL0 + cc]; });
    __syncthreads();
    if (more) {
      mv.store([&](int rr, int cc, T v) { lds[rr * S::PITCH + S::COL0 + cc] = v; });
      pf.commit(2 * R, wr);
    }
    __syncthreads();
  }
}

template <typename T, int R, int VAR>
__global__ __launch_bounds__(kThreads) void mfma2d_kernel(KArgs a) {
  mfma2d_item<T, R, VAR>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, int VAR>
__global__ __launch_bounds__(kThreads) void mfma2d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { mfma2d_item<T, R, VAR>(x, id); });
}

// ---------------------------------------------------------------------------
// Outer-product form with n = 4 blocks on v_mfma_f32_4x4x1_16b_f32 (FP32).
//
// One instruction performs sixteen independent rank-1 updates of 4 x 4 output
// blocks: exactly the vector outer product of Eq. (8) with n = 4.  The sixteen
// blocks of a wave sit side by side along j, so a wave covers 4 rows x 64
// columns per accumulator; with four accumulators (the i unrolling of
// Section 4.2, ui = 4) a wave owns 16 rows x 64 columns.
//   A operand (lane l): the coefficient vector of Eq. (9)-(10) for line b and
//     band offset d: T_b[l % 4][d] = C^g[d - l % 4][b] (zero outside the band);
//     all (2r+1) x (4 + 2r) vectors stay in VGPRs.
//   B operand (lane l): window row x, column l + b -- one conflict-free LDS
//     read of 64 consecutive floats, scattered to every accumulator whose rows
//     it reaches (Section 4.3: group the outer products by input vector).
//   D (lane l, register v): row 4 s + v, column l -- full 256-byte rows.
// Padding per line is (4 + 2r) / (2r + 1) instead of (16 + 2r) / (2r + 1).
// BOX: all 2r+1 lines along i; STAR (parallel option, Table 1): the centre
// line on MFMA, the single-weight lines as vector FMAs.
// ---------------------------------------------------------------------------
template <int R, bool BOX>
struct MfmaB4Shape {
  static constexpr int NB = 4 + 2 * R;              // band offsets per line
  static constexpr int NL = BOX ? 2 * R + 1 : 1;    // lines on MFMA
  static constexpr int NF = NL * NB;                // coefficient vectors per lane
  static constexpr int TM = kTile2D, TN = kTile2D;
  static constexpr int WROWS = TM + 2 * R, WCOLS = TN + 2 * R;
  static constexpr int COL0 = lds_col0<float, R>();
  static constexpr int PITCH = round_up(COL0 + WCOLS, 4);
};

template <int R, bool BOX>
__device__ __forceinline__ void mfma2d_b4_item(const KArgs& a, int item) {
  typedef MfmaB4Shape<R, BOX> S;
  constexpr int BM = S::TM;
  __shared__ __attribute__((aligned(16))) float lds[S::WROWS * S::PITCH];

  const int64_t M = a.d0, N = a.d1;
  const bool periodic = a.periodic != 0;
  const float* __restrict__ in = (const float*)a.in;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const Strip2D sp = decode_strip(a, item, S::TN);
  const bool fast = strip_fast(in, N, sp.j0, S::TN);

  const float* __restrict__ frag = (const float*)a.frag;
  float af[S::NF];
#pragma unroll
  for (int c = 0; c < S::NF; ++c) af[c] = frag[c * 64 + lane];
  float cw[2 * R + 1];
  if constexpr (!BOX) {
    const float* __restrict__ c = (const float*)a.coef;
#pragma unroll
    for (int b = 0; b <= 2 * R; ++b) cw[b] = c[R * (2 * R + 1) + b];
  }

  stage_window<float, R, S::WROWS, S::TN, S::PITCH, kThreads>(lds, in, M, N, sp.i0 - R, sp.j0, periodic);
  __syncthreads();

  PlainWriter<float, R, S::PITCH> wr{lds};
  RowPrefetch<float, R, BM, S::TN, kThreads> pf;
  RowMover<float, R, S::WCOLS, kThreads> mv;
  const float* rowp = lds + (16 * w) * S::PITCH + S::COL0 + lane;
  for (int64_t ib = sp.i0; ib < sp.i1; ib += BM) {
    const bool more = ib + BM < sp.i1;
    if (more) pf.fetch(in, M, N, ib + BM + R, sp.j0, periodic, fast);
    floatx4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = floatx4{0, 0, 0, 0};
#pragma unroll
    for (int li = 0; li < S::NL; ++li) {
      const int b = BOX ? li : R;
#pragma unroll
      for (int x = 0; x < 16 + 2 * R; ++x) {
        const float bv = rowp[x * S::PITCH + b];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int d = x - 4 * s;
          if (d < 0 || d >= S::NB) continue;
          acc[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(af[li * S::NB + d], bv, acc[s], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // keep each line's LDS reads next to its MFMAs
    }
    if constexpr (!BOX) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float* rp = rowp + (4 * s + v + R) * S::PITCH;
          float sum = 0.0f;
#pragma unroll
          for (int b = 0; b <= 2 * R; ++b) {
            if (b == R) continue;
            sum += cw[b] * rp[b];
          }
          acc[s][v] += sum;
        }
    }
    const int64_t gj = sp.j0 + lane;
    if (gj < N) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t gi = ib + 16 * w + 4 * s + v;
          if (gi < sp.i1) out[gi * N + gj] = acc[s][v];
        }
    }
    if (more) mv.load([&](int rr, int cc) { return lds[(BM + rr) * S::PITCH + S::COL0 + cc]; });
    __syncthreads();
    if (more) {
      mv.store([&](int rr, int cc, float v) { lds[rr * S::PITCH + S::COL0 + cc] = v; });
      pf.commit(2 * R, wr);
    }
    __syncthreads();
  }
}

template <int R, bool BOX>
__global__ __launch_bounds__(kThreads) void mfma2d_b4_kernel(KArgs a) {
  mfma2d_b4_item<R, BOX>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int R, bool BOX>
__global__ __launch_bounds__(kThreads) void mfma2d_b4_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { mfma2d_b4_item<R, BOX>(x, id); });
}

}  // namespace stencil
