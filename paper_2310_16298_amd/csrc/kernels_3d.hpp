// 3D stencil kernels (grid (i, j, k), k contiguous).
//
// Plane order of Algorithm 1 (Section 4.4): a workgroup owns a TJ x TK tile
// of the (j, k) plane and a chunk of CH output planes along i.  It walks the
// input planes i = ib - r .. ib + CH + r - 1 once; each plane is staged into
// LDS with its in-plane halo and scattered into the 2r+1 output planes it
// reaches, whose accumulators form a ring in registers (the i-direction
// unrolling of Section 4.2: an input element is loaded once and used by all
// its neighbours along i).  While input plane i is scattered, ring slot z
// holds output plane i - r + z, so coefficient plane a (output plane
// i - a + r) goes to the compile-time slot 2r - a; afterwards output plane
// i - r is complete in slot 0: it is stored and the ring shifts down by one.
//
// Staging: with DMA = true the window of plane i+1 is loaded straight into
// LDS (dma3d.hpp) while plane i is computed; otherwise (extents or pointers
// that do not allow 16-byte lines) each plane is staged synchronously.
#pragma once

#include <type_traits>
#include <utility>

#include "device_common.hpp"
#include "dma3d.hpp"
#include "kernels_2d.hpp"
#include "kernels_split2d.hpp"
#include "launch.hpp"
#include "mfma_traits.hpp"

namespace stencil {

constexpr int kTJ = 32;   // workgroup tile along j
constexpr int kTK = 64;   // workgroup tile along k

struct Chunk3D {
  int64_t ib, iend, j0, k0;  // output planes [ib, iend), tile origin
};

// Work items of a 3D grid: (j, k) tiles x i-chunks (set by the plan).
inline int64_t chunk3d_items(const KArgs& a) { return (int64_t)a.tiles0 * a.tiles1 * a.nchunks; }

// Work items of a single-grid launch of `kernel`.  When the chunk is the
// library's choice, the kernel keeps at most three workgroups per CU and the
// plan-time decomposition needs more than one wave of them, the planes are
// re-cut into the most chunks of equal depth (at least 4r planes) whose items
// still fit one wave: every (tile, chunk) item then runs at once (no partial
// last wave), and the items an XCD receives are neighbours in the plane, so
// the halo rows one reads are in L2 when the next reads them.  Measured on
// MI355X: FP32 stars of order 4 +8-19 % (384^3, 512^3), FP64 stars of order
// 4 at 384^3 +60 %; kernels with four or more workgroups per CU ran 2-4 %
// slower re-cut and keep the plan's chunks.  cap_per_cu > 0 counts at most
// that many workgroups per CU (a kernel that runs slower with more of them
// resident: its items are re-cut to fill the CUs evenly at the cap).
inline int64_t balanced_items3d(KArgs& a, const void* kernel, int R, int32_t chunk_req, int threads = 256,
                                int cap_per_cu = 0) {
  const int64_t items = chunk3d_items(a);
  if (chunk_req > 0) return items;
  const Residency res = resident_workgroups(kernel, threads);
  const int per_cu = cap_per_cu > 0 && res.per_cu > cap_per_cu ? cap_per_cu : res.per_cu;
  if (per_cu <= 0 || res.cus <= 0) return items;
  const int64_t tiles = (int64_t)a.tiles0 * a.tiles1;
  auto recut = [&](int64_t nch) {
    if (nch < 1) nch = 1;
    int64_t chunk = (a.d0 + nch - 1) / nch;
    const int64_t minc = 4 * R < a.d0 ? 4 * R : a.d0;
    if (chunk < minc) chunk = minc;
    a.chunk = (int32_t)chunk;
    a.nchunks = (int32_t)((a.d0 + chunk - 1) / chunk);
    return chunk3d_items(a);
  };
  const int64_t slots = (int64_t)per_cu * res.cus;
  if (per_cu <= 3 && items > slots) return recut(slots / tiles);
  // Even fill: the plan rounds its chunk count up from an item target, which
  // on extents that are not powers of two leaves some CUs one workgroup more
  // than the rest (FP64 7-point star at 384^3: 576 items, 2.25 per CU, the
  // CUs with three setting the launch time).  Round the items per CU to the
  // nearest whole number and re-cut the planes into at most that many.
  if (items >= res.cus) {
    const int64_t target = (items + res.cus / 2) / res.cus * res.cus;
    if (items > target && target / tiles >= 1) return recut(target / tiles);
  }
  return items;
}

// A 3D kernel (single-grid K, batched B) for its plan's args: items as above.
template <auto K, auto B, int NT = 256>
inline Kernel kernel3d(KArgs& a, int R, int32_t chunk_req, int cap_per_cu = 0) {
  Kernel k = kernel_of<K, B, NT>(0);
  k.items = balanced_items3d(a, k.single_id, R, chunk_req, NT, cap_per_cu);
  return k;
}

__device__ __forceinline__ Chunk3D decode_chunk(const KArgs& a, int id) {
  const int per_plane = a.tiles0 * a.tiles1;
  const int chunk = id / per_plane;
  const int t = id - chunk * per_plane;
  const int tj = t / a.tiles1, tk = t - tj * a.tiles1;
  Chunk3D c;
  c.ib = (int64_t)chunk * a.chunk;
  c.iend = c.ib + a.chunk < a.d0 ? c.ib + a.chunk : a.d0;
  c.j0 = (int64_t)tj * kTJ;
  c.k0 = (int64_t)tk * kTK;
  return c;
}

// Walk the input planes of a chunk.  LROWS window rows (global j0 - r ..) of
// each plane are staged into a buffer of pitch PITCH, window column y at LDS
// column COL0 + y.
template <typename T, int R, int LROWS, bool DMA, bool BODY4 = false>
struct PlaneWalk {
  static constexpr int W = 2 * R + 1;
  typedef DmaPlane<T, R, LROWS, kTK, kThreads> D;
  // BODY4: the tile body (window column r) sits at LDS column 4 in both
  // staging modes, as in the direct-to-LDS layout.
  static constexpr int PITCH = (DMA || BODY4) ? D::PITCH : pick_pitch<T, true>(lds_col0<T, R>() + kTK + 2 * R + 8);
  static constexpr int COL0 = (DMA || BODY4) ? D::COL0 : lds_col0<T, R>();
  static constexpr int BUF = DMA ? D::BUF : LROWS * PITCH;  // elements per buffer
  static constexpr int NBUF = DMA ? 2 : 1;

  // body(win, valid) scatters input plane i (win = its window; valid = false
  // for a zero-halo plane outside the grid), then finish(o, live) completes
  // output plane o = i - r (live = o lies in the chunk; warm-up planes reach
  // outputs below it): the caller stores its ring's slot 0 when live and
  // shifts the ring down by one.
  template <class Body, class Finish>
  static __device__ __forceinline__ void walk(T* bufs, const KArgs& a, const Chunk3D& ch, Body body, Finish finish) {
    const int64_t Ni = a.d0, Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
    const bool periodic = a.periodic != 0;
    const T* __restrict__ in = (const T*)a.in;
    const T* __restrict__ zeros = (const T*)a.zeros;
    const int nu = (int)(ch.iend - ch.ib) + 2 * R;
    typename D::Lines lines;
    if constexpr (DMA) {
      D::prepare(lines, Nj, Nk, ch.j0 - R, ch.k0, periodic);
      const int64_t g0 = map_index(ch.ib - R, Ni, periodic);
      D::issue(bufs, g0 >= 0 ? in + g0 * plane : nullptr, zeros, lines);
    } else {
      // rows and columns past the window (K padding of the MFMA kernels) are
      // read with zero weights: keep them finite
      zero_region<T, kThreads>(bufs, LROWS, PITCH, PITCH, 0, 0);
    }
    for (int u = 0; u < nu; ++u) {
      const int64_t gi = map_index(ch.ib - R + u, Ni, periodic);
      const T* win;
      if constexpr (DMA) {
        win = bufs + (u & 1) * BUF;
        if (u + 1 < nu) {
          const int64_t g1 = map_index(ch.ib - R + u + 1, Ni, periodic);
          D::issue(bufs + ((u + 1) & 1) * BUF, g1 >= 0 ? in + g1 * plane : nullptr, zeros, lines);
          D::template wait_vm<D::NPW>();
        } else {
          D::template wait_vm<0>();
        }
        lds_barrier();
      } else {
        win = bufs;
        __syncthreads();
        if (gi >= 0)
          stage_window<T, R, kTJ + 2 * R, kTK, PITCH, kThreads, COL0>(bufs, in + gi * plane, Nj, Nk, ch.j0 - R,
                                                                     ch.k0, periodic);
        __syncthreads();
      }
      body(win, gi >= 0);
      finish(ch.ib + u - 2 * R, u >= 2 * R);
      if constexpr (DMA) lds_barrier();
    }
  }

  // As walk, with the loop over planes unrolled by W: body(win, valid, ph)
  // and finish(o, live, ph) receive ph = u mod W as a std::integral_constant,
  // so a caller can keep its ring of 2r+1 output planes in place and rotate
  // the slot it names (slot z of plane u in register (z + ph) mod W) instead
  // of moving every accumulator down one slot after each plane.
  template <class Body, class Finish>
  static __device__ __forceinline__ void walk_phased(T* bufs, const KArgs& a, const Chunk3D& ch, Body body,
                                                     Finish finish) {
    const int64_t Ni = a.d0, Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
    const bool periodic = a.periodic != 0;
    const T* __restrict__ in = (const T*)a.in;
    const T* __restrict__ zeros = (const T*)a.zeros;
    const int nu = (int)(ch.iend - ch.ib) + 2 * R;
    typename D::Lines lines;
    if constexpr (DMA) {
      D::prepare(lines, Nj, Nk, ch.j0 - R, ch.k0, periodic);
      const int64_t g0 = map_index(ch.ib - R, Ni, periodic);
      D::issue(bufs, g0 >= 0 ? in + g0 * plane : nullptr, zeros, lines);
    } else {
      zero_region<T, kThreads>(bufs, LROWS, PITCH, PITCH, 0, 0);
    }
    auto step = [&](int u, auto ph) __attribute__((always_inline)) {
      const int64_t gi = map_index(ch.ib - R + u, Ni, periodic);
      const T* win;
      if constexpr (DMA) {
        win = bufs + (u & 1) * BUF;
        if (u + 1 < nu) {
          const int64_t g1 = map_index(ch.ib - R + u + 1, Ni, periodic);
          D::issue(bufs + ((u + 1) & 1) * BUF, g1 >= 0 ? in + g1 * plane : nullptr, zeros, lines);
          D::template wait_vm<D::NPW>();
        } else {
          D::template wait_vm<0>();
        }
        lds_barrier();
      } else {
        win = bufs;
        __syncthreads();
        if (gi >= 0)
          stage_window<T, R, kTJ + 2 * R, kTK, PITCH, kThreads, COL0>(bufs, in + gi * plane, Nj, Nk, ch.j0 - R,
                                                                     ch.k0, periodic);
        __syncthreads();
      }
      body(win, gi >= 0, ph);
      finish(ch.ib + u - 2 * R, u >= 2 * R, ph);
      if constexpr (DMA) lds_barrier();
    };
    for (int u0 = 0; u0 < nu; u0 += W) phases(step, u0, nu, std::make_integer_sequence<int, W>{});
  }

  template <class Step, int... P>
  static __device__ __forceinline__ void phases(Step& step, int u0, int nu, std::integer_sequence<int, P...>) {
    ((u0 + P < nu ? step(u0 + P, std::integral_constant<int, P>{}) : void()), ...);
  }
};

// ---------------------------------------------------------------------------
// Gather-form baseline (Eq. (1) in 3D).  Thread t owns a 2 x 4 register
// block: j rows 2 (t / 16) .. +1 and k columns 4 (t % 16) .. +3 of the tile.
// Each window row it needs is read as 12 consecutive values (16-byte LDS
// vectors, columns 4 (t % 16) - 4 .. + 7 around the block), which cover
// the k offsets -r .. r of all four columns.  Box: each input plane adds its
// (2r+1)^2 in-plane taps to the 2r+1 output planes it reaches; star: the
// centre plane adds the j and k arms, every plane adds its i-arm weight.
// Ring: ring[z] accumulates output plane i - r + z while input plane i is
// scattered (coefficient plane a reaches z = 2r - a); afterwards ring[0] is
// complete and the ring shifts down by one.
// ---------------------------------------------------------------------------
template <typename T, int R, bool BOX, bool DMA>
__device__ __forceinline__ void gather3d_item(const KArgs& a, int item) {
  constexpr int W = 2 * R + 1, VEC = 16 / (int)sizeof(T), NV = 12 / VEC;
  typedef typename Vec16<T>::type V;
  typedef PlaneWalk<T, R, kTJ + 2 * R, DMA, true> PW;
  static_assert(PW::COL0 + R == 4, "tile body at LDS column 4");
  __shared__ __attribute__((aligned(16))) T bufs[PW::NBUF * PW::BUF];

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  T* __restrict__ out = (T*)a.out;
  const ConstPtr<T> c = (ConstPtr<T>)a.coef;  // uniform reads: scalar loads
  const int q4 = threadIdx.x & 15, rg = threadIdx.x >> 4;

  T ring[W][2][4];
#pragma unroll
  for (int z = 0; z < W; ++z)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) ring[z][p][e] = T(0);

  // v[m] = window row x, LDS column 4 q4 + m (tile column 4 q4 + m - 4)
  auto row12 = [&](const T* win, int x, T v[12]) {
    const V* rp = reinterpret_cast<const V*>(win + (2 * rg + x) * PW::PITCH + 4 * q4);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const V t = rp[k];
      const T* pt = reinterpret_cast<const T*>(&t);
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[k * VEC + e] = pt[e];
    }
  };

  // Stars and the 27-point box rotate the ring: at plane phase PH (input
  // plane u, PH = u mod W) slot z sits in register set (z + PH) mod W, and
  // the stored set is cleared for the next plane's top slot.  Larger boxes
  // (up to 5832 FMAs per plane) keep one copy of the plane code and shift.
  constexpr bool ROT = !BOX || R == 1;
  auto body = [&](const T* win, bool valid, auto phase) __attribute__((always_inline)) {
        constexpr int PH = ROT ? decltype(phase)::value : 0;
        if (!valid) return;  // a zero-halo plane adds nothing
        if constexpr (BOX) {
#pragma unroll
          for (int x = 0; x < 2 + 2 * R; ++x) {
            T v[12];
            row12(win, x, v);
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              const int bb = x - p;
              if (bb < 0 || bb > 2 * R) continue;
#pragma unroll
              for (int ap = 0; ap < W; ++ap)
#pragma unroll
                for (int cc = 0; cc < W; ++cc) {
                  const T w = c[(ap * W + bb) * W + cc];
#pragma unroll
                  for (int e = 0; e < 4; ++e) ring[(2 * R - ap + PH) % W][p][e] += w * v[4 - R + e + cc];
                }
            }
          }
        } else {
          // j arm into the centre plane's slot r: column block at LDS columns 4 q4 + 4 ..
#pragma unroll
          for (int x = 0; x < 2 + 2 * R; ++x) {
            const V* rp = reinterpret_cast<const V*>(win + (2 * rg + x) * PW::PITCH + 4 * q4 + 4);
            T v[4];
#pragma unroll
            for (int k = 0; k < 4 / VEC; ++k) {
              const V t = rp[k];
              const T* pt = reinterpret_cast<const T*>(&t);
#pragma unroll
              for (int e = 0; e < VEC; ++e) v[k * VEC + e] = pt[e];
            }
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              const int bb = x - p;
              if (bb < 0 || bb > 2 * R) continue;
              const T w = c[(R * W + bb) * W + R];
#pragma unroll
              for (int e = 0; e < 4; ++e) ring[(R + PH) % W][p][e] += w * v[e];
            }
          }
          // k arm (centre excluded) and i arm from the block's own rows
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            T v[12];
            row12(win, p + R, v);
#pragma unroll
            for (int cc = 0; cc < W; ++cc) {
              if (cc == R) continue;
              const T w = c[(R * W + R) * W + cc];
#pragma unroll
              for (int e = 0; e < 4; ++e) ring[(R + PH) % W][p][e] += w * v[4 - R + e + cc];
            }
#pragma unroll
            for (int ap = 0; ap < W; ++ap) {
              if (ap == R) continue;
              const T w = c[(ap * W + R) * W + R];
#pragma unroll
              for (int e = 0; e < 4; ++e) ring[(2 * R - ap + PH) % W][p][e] += w * v[4 + e];
            }
          }
        }
  };
  auto finish = [&](int64_t o, bool live, auto phase) __attribute__((always_inline)) {
        constexpr int Z0 = ROT ? decltype(phase)::value : 0;  // register set of slot 0
        const int64_t gk = ch.k0 + 4 * q4;
        if (live) {
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            const int64_t gj = ch.j0 + 2 * rg + p;
            if (gj >= Nj) continue;
            T* dst = out + o * plane + gj * Nk + gk;
            if constexpr (DMA) {
              // k extent a multiple of the vector and output 16-byte aligned:
              // a vector starting inside the row lies inside it
#pragma unroll
              for (int k = 0; k < 4 / VEC; ++k) {
                if (gk + k * VEC >= Nk) break;
                V t;
                T* pt = reinterpret_cast<T*>(&t);
#pragma unroll
                for (int e = 0; e < VEC; ++e) pt[e] = ring[Z0][p][k * VEC + e];
                reinterpret_cast<V*>(dst)[k] = t;
              }
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (gk + e < Nk) dst[e] = ring[Z0][p][e];
            }
          }
        }
        if constexpr (!ROT) {
#pragma unroll
          for (int z = 0; z < 2 * R; ++z)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
              for (int e = 0; e < 4; ++e) ring[z][p][e] = ring[z + 1][p][e];
        }
        constexpr int ZT = ROT ? Z0 : 2 * R;  // the next plane's top slot
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int e = 0; e < 4; ++e) ring[ZT][p][e] = T(0);
  };
  if constexpr (ROT) {
    PW::walk_phased(bufs, a, ch, body, finish);
  } else {
    PW::walk(
        bufs, a, ch, [&](const T* win, bool valid) { body(win, valid, std::integral_constant<int, 0>{}); },
        [&](int64_t o, bool live) { finish(o, live, std::integral_constant<int, 0>{}); });
  }
}

template <typename T, int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads) void gather3d_kernel(KArgs a) {
  gather3d_item<T, R, BOX, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads) void gather3d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { gather3d_item<T, R, BOX, DMA>(x, id); });
}

// ---------------------------------------------------------------------------
// Whole-grid gather for small 3D grids (the paper's Table 3 sizes, 8^3 and
// up): one workgroup stages the grid with its r halo (zero or wrapped) in
// LDS and computes every point as Eq. (1), one point per thread and pass.
// The tiled kernels give such a grid 32 x 64 (j, k) tiles of which an 8 x 8
// plane fills one lane in 32; a batch of many small grids then keeps every
// lane of every workgroup busy instead.  VOL: LDS elements (16 to 128 KiB).
// ---------------------------------------------------------------------------
template <typename T, int VOL>
__host__ __device__ constexpr bool whole3d_fits(int64_t Ni, int64_t Nj, int64_t Nk, int R) {
  return (Ni + 2 * R) * (Nj + 2 * R) * (Nk + 2 * R) <= VOL;
}

// e / d for 0 <= e < 2^20 and 0 < d: a float estimate from the reciprocal,
// corrected by one either way (cheaper than the integer division sequence)
__device__ __forceinline__ int div_small(int e, int d, float rd) {
  int q = (int)((float)e * rd);
  if (q * d > e) --q;
  else if ((q + 1) * d <= e) ++q;
  return q;
}

template <typename T, int R, bool BOX, int VOL>
__device__ __forceinline__ void gather3d_whole_item(const KArgs& a) {
  constexpr int W = 2 * R + 1;
  __shared__ T g[VOL];
  const int Ni = (int)a.d0, Nj = (int)a.d1, Nk = (int)a.d2;
  const int PJ = Nj + 2 * R, PK = Nk + 2 * R, PP = PJ * PK;
  const bool periodic = a.periodic != 0;
  const T* __restrict__ in = (const T*)a.in;
  T* __restrict__ out = (T*)a.out;
  const ConstPtr<T> c = (ConstPtr<T>)a.coef;  // uniform reads: scalar loads
  const int vol = (Ni + 2 * R) * PP;
  const float rPP = 1.0f / (float)PP, rPK = 1.0f / (float)PK;
  // several loads in flight per thread before their LDS stores (one memory
  // round trip per UNR elements, not per element); four in the 16 KiB class
  constexpr int UNR = VOL * (int)sizeof(T) <= 16384 ? 4 : 8;
  for (int e0 = threadIdx.x; e0 < vol; e0 += UNR * kThreads) {
    T v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = e0 + u * kThreads;
      v[u] = T(0);
      if (e < vol) {
        const int i = div_small(e, PP, rPP), rem = e - i * PP, j = div_small(rem, PK, rPK), k = rem - j * PK;
        const int64_t gi = map_index(i - R, Ni, periodic), gj = map_index(j - R, Nj, periodic),
                      gk = map_index(k - R, Nk, periodic);
        if (gi >= 0 && gj >= 0 && gk >= 0) v[u] = in[(gi * Nj + gj) * Nk + gk];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      if (e0 + u * kThreads < vol) g[e0 + u * kThreads] = v[u];
  }
  __syncthreads();
  const int plane = Nj * Nk, n = Ni * plane;
  const float rplane = 1.0f / (float)plane, rNk = 1.0f / (float)Nk;
  for (int p = threadIdx.x; p < n; p += kThreads) {
    const int i = div_small(p, plane, rplane), rem = p - i * plane, j = div_small(rem, Nk, rNk), k = rem - j * Nk;
    const T* base = g + i * PP + j * PK + k;  // padded (i, j, k) = neighbourhood corner
    // the tiled kernel's order per point (input planes ascending; a star's
    // centre plane: the j arm with the centre, then the k arm), so a grid
    // gives the same bits on either kernel and under the time-blocked ones
    T sum = T(0);
#pragma unroll
    for (int x = 0; x < W; ++x) {
      if constexpr (BOX) {
#pragma unroll
        for (int y = 0; y < W; ++y)
#pragma unroll
          for (int z = 0; z < W; ++z) sum += c[(x * W + y) * W + z] * base[x * PP + y * PK + z];
      } else if (x != R) {
        sum += c[(x * W + R) * W + R] * base[x * PP + R * PK + R];
      } else {
#pragma unroll
        for (int y = 0; y < W; ++y) sum += c[(R * W + y) * W + R] * base[R * PP + y * PK + R];
#pragma unroll
        for (int z = 0; z < W; ++z)
          if (z != R) sum += c[(R * W + R) * W + z] * base[R * PP + R * PK + z];
      }
    }
    out[p] = sum;
  }
}

template <typename T, int R, bool BOX, int VOL>
__global__ __launch_bounds__(kThreads) void gather3d_whole_kernel(KArgs a) {
  gather3d_whole_item<T, R, BOX, VOL>(a);
}

template <typename T, int R, bool BOX, int VOL>
__global__ __launch_bounds__(kThreads) void gather3d_whole_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int) { gather3d_whole_item<T, R, BOX, VOL>(x); });
}

// The whole-grid kernel for a grid that fits 16, 32, 64 or 128 KiB of LDS
// with its halo (the smallest: more workgroups per CU) and leaves the chunk
// to the library, else none.
template <typename T, int R, bool BOX>
inline Kernel whole3d_kernel(const KArgs& a, int32_t chunk) {
  constexpr int SMALL = 16384 / (int)sizeof(T), MEDIUM = 32768 / (int)sizeof(T), LARGE = 65536 / (int)sizeof(T),
                HUGE = 131072 / (int)sizeof(T);
  if (chunk != 0) return Kernel{};
  if (whole3d_fits<T, SMALL>(a.d0, a.d1, a.d2, R))
    return kernel_of<gather3d_whole_kernel<T, R, BOX, SMALL>, gather3d_whole_batch<T, R, BOX, SMALL>>(1);
  if (whole3d_fits<T, MEDIUM>(a.d0, a.d1, a.d2, R))
    return kernel_of<gather3d_whole_kernel<T, R, BOX, MEDIUM>, gather3d_whole_batch<T, R, BOX, MEDIUM>>(1);
  if (whole3d_fits<T, LARGE>(a.d0, a.d1, a.d2, R))
    return kernel_of<gather3d_whole_kernel<T, R, BOX, LARGE>, gather3d_whole_batch<T, R, BOX, LARGE>>(1);
  // 128 KiB (one workgroup per CU) only for grids of at most 16^3 points:
  // larger ones keep the tiled kernel's parallelism when launched alone
  if (a.d0 * a.d1 * a.d2 <= 4096 && whole3d_fits<T, HUGE>(a.d0, a.d1, a.d2, R))
    return kernel_of<gather3d_whole_kernel<T, R, BOX, HUGE>, gather3d_whole_batch<T, R, BOX, HUGE>>(1);
  return Kernel{};
}

// ---------------------------------------------------------------------------
// Outer-product form on MFMA (FP32 / FP64).  Waves form a 2 x 2 grid over the
// 32 x 64 tile; each wave owns two 16 x 16 blocks (16 j-rows x 32 k-columns)
// in each of the 2r+1 ring slots.
//
// Box (3D box stencils, Section 3.3: the (2r+1)^2 lines CLS(a, *, c) along j):
// input plane i adds, for every coefficient plane a and k-shift c, the band
// T_{a,c}[p][x] = C^g[a][x - p][c] times the window rows shifted by c to output
// plane i - a + r.  The band fragments of all lines stay in VGPRs.
// Star (hybrid cover of Table 2): on the centre plane the line CLS(r, *, r)
// along j (band, rows of the window as B operand) and CLS(r, r, *) along k
// (window column segments as A operand, centre excluded); the lines CLS(a, *, r)
// with a != r hold one weight each and are the vector FMAs of the i arm.
// K padding reads rows and columns past the band; they carry zero weights
// (rows are loaded or zeroed; columns past a row end read the next row).
// ---------------------------------------------------------------------------
template <typename T, int R, bool BOX>
struct Mfma3DShape {
  static constexpr int W = 2 * R + 1;
  static constexpr int KL = round_up(16 + 2 * R, 4);
  static constexpr int CPL = KL / 4;
  static constexpr int NLINES = BOX ? W * W : 2;
  static constexpr int NCH = NLINES * CPL;
  static constexpr int LROWS = cmax(kTJ + 2 * R, (kTJ - 16) + KL);
};

template <typename T, int R, bool BOX, bool DMA>
__device__ __forceinline__ void mfma3d_item(const KArgs& a, int item) {
  typedef Mfma16<T> MM;
  typedef typename MM::acc_t acc_t;
  typedef Mfma3DShape<T, R, BOX> S;
  typedef PlaneWalk<T, R, S::LROWS, DMA> PW;
  constexpr int W = S::W;
  __shared__ __attribute__((aligned(16))) T bufs[PW::NBUF * PW::BUF];

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  T* __restrict__ out = (T*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wj = w >> 1, wk = w & 1;
  const int g = lane >> 4, q = lane & 15;

  const T* __restrict__ frag = (const T*)a.frag;
  T af[S::NCH];
#pragma unroll
  for (int cidx = 0; cidx < S::NCH; ++cidx) af[cidx] = frag[cidx * 64 + lane];
  T ci[W];  // i-arm weights C^g[a][r][r] (star)
  if constexpr (!BOX) {
    const T* __restrict__ c = (const T*)a.coef;
#pragma unroll
    for (int ap = 0; ap < W; ++ap) ci[ap] = c[(ap * W + R) * W + R];
  }

  acc_t ring[W][2];
#pragma unroll
  for (int z = 0; z < W; ++z) {
    ring[z][0] = acc_t{};
    ring[z][1] = acc_t{};
  }
  // ring[z] accumulates output plane i - r + z while input plane i is
  // scattered (coefficient plane a reaches z = 2r - a); then ring[0] is
  // complete and the ring shifts down by one.
  PW::walk(
      bufs, a, ch,
      [&](const T* win, bool valid) {
        if (!valid) return;
        const T* colbase = win + (16 * wj + g) * PW::PITCH + PW::COL0 + 32 * wk + q;
        const T* rowbase = win + (16 * wj + R + q) * PW::PITCH + PW::COL0 + 32 * wk + g;
        if constexpr (BOX) {
#pragma unroll
          for (int ap = 0; ap < W; ++ap) {
            const int slot = 2 * R - ap;
#pragma unroll
            for (int cs = 0; cs < W; ++cs) {
#pragma unroll
              for (int cc = 0; cc < S::CPL; ++cc) {
                const T av = af[(ap * W + cs) * S::CPL + cc];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                  const T bv = colbase[(4 * cc) * PW::PITCH + 16 * t + cs];
                  ring[slot][t] = MM::mma(av, bv, ring[slot][t]);
                }
              }
            }
          }
        } else {
          const int slot = R;
#pragma unroll
          for (int cc = 0; cc < S::CPL; ++cc) {
            const T av = af[cc];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const T bv = colbase[(4 * cc) * PW::PITCH + 16 * t + R];
              ring[slot][t] = MM::mma(av, bv, ring[slot][t]);
            }
          }
#pragma unroll
          for (int cc = 0; cc < S::CPL; ++cc) {
            const T sv = af[S::CPL + cc];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const T hv = rowbase[16 * t + 4 * cc];
              ring[slot][t] = MM::mma(hv, sv, ring[slot][t]);
            }
          }
          // i arm: lines CLS(a, *, r), a != r, one weight each
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T* cp = win + (16 * wj + R + MM::row(lane, v)) * PW::PITCH + PW::COL0 + 32 * wk + MM::col(lane) + R;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const T ctr = cp[16 * t];
#pragma unroll
              for (int ap = 0; ap < W; ++ap) {
                if (ap == R) continue;
                ring[2 * R - ap][t][v] += ci[ap] * ctr;
              }
            }
          }
        }
      },
      [&](int64_t o, bool live) {
        if (live) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t gj = ch.j0 + 16 * wj + MM::row(lane, v);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const int64_t gk = ch.k0 + 32 * wk + 16 * t + MM::col(lane);
              if (gj < Nj && gk < Nk) out[o * plane + gj * Nk + gk] = ring[0][t][v];
            }
          }
        }
#pragma unroll
        for (int z = 0; z < 2 * R; ++z) {
          ring[z][0] = ring[z + 1][0];
          ring[z][1] = ring[z + 1][1];
        }
        ring[2 * R][0] = acc_t{};
        ring[2 * R][1] = acc_t{};
      });
}

template <typename T, int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads) void mfma3d_kernel(KArgs a) {
  mfma3d_item<T, R, BOX, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <typename T, int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads) void mfma3d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { mfma3d_item<T, R, BOX, DMA>(x, id); });
}

// ---------------------------------------------------------------------------
// Outer-product form on n = 4 blocks (v_mfma_f32_4x4x1_16b_f32, FP32), as the
// 2D kernel of dma2d.hpp: wave w owns tile rows 8 w .. 8 w + 7 (two 4-row
// blocks s) and all 64 columns; block beta of an instruction holds output
// (row 4 s + j, column 4 beta + i), lane 4 beta + j owning four consecutive
// columns.  Lines along j (CLS(a, *, c)): A = input row segment of window
// row x (column lane + c), B = band value w[x - 4 s - j].  Line along k
// (CLS(r, r, *), centre excluded): A = band value w[e - i], B = input
// H[4 s + j + r][4 beta + e].  Star: the j and k lines through the centre on
// MFMA, the i arm as vector FMAs into the other ring slots.  Box: the 27-point
// box (r = 1), all nine lines along j.
// ---------------------------------------------------------------------------
template <int R, bool BOX, bool DMA>
__device__ __forceinline__ void mfma3d_b4_item(const KArgs& a, int item) {
  constexpr int W = 2 * R + 1, NB = 4 + 2 * R, NL = BOX ? W * W : 2;
  typedef PlaneWalk<float, R, kTJ + 2 * R, DMA, true> PW;
  static_assert(PW::COL0 + R == 4, "tile body at LDS column 4");
  __shared__ __attribute__((aligned(16))) float bufs[PW::NBUF * PW::BUF];

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int orow = lane & 3, beta = lane >> 2;

  // band vectors packed four to a register (lane group g holds vector 4 k + g)
  constexpr int NC = NL * NB, NP = (NC + 3) / 4;
  const float* __restrict__ frag = (const float*)a.frag;
  float af[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int c = 4 * k + (lane >> 4);
    af[k] = c < NC ? frag[c * 64 + lane] : 0.0f;
  }
  float ci[W];  // star: i-arm weights C^g[a][r][r]
  if constexpr (!BOX) {
    const float* __restrict__ c = (const float*)a.coef;
#pragma unroll
    for (int ap = 0; ap < W; ++ap) ci[ap] = c[(ap * W + R) * W + R];
  }

  // ring[z][s]: output plane i - r + z while input plane i is scattered
  floatx4 ring[W][2];
#pragma unroll
  for (int z = 0; z < W; ++z)
#pragma unroll
    for (int t = 0; t < 2; ++t) ring[z][t] = floatx4{0, 0, 0, 0};

  PW::walk(
      bufs, a, ch,
      [&](const float* win, bool valid) {
        if (!valid) return;
        // lines along j: CLS(ap, *, cs) into slot 2r - ap
#pragma unroll
        for (int l = 0; l < (BOX ? W * W : 1); ++l) {
          const int ap = BOX ? l / W : R, cs = BOX ? l % W : R;
          const float* rowp = win + (8 * w) * PW::PITCH + PW::COL0 + lane + cs;
#pragma unroll
          for (int x = 0; x < 8 + 2 * R; ++x) {
            const float hv = rowp[x * PW::PITCH];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              const int d = x - 4 * s;
              if (d < 0 || d >= NB) continue;
              const int c = l * NB + d;
              ring[2 * R - ap][s] = mfma4_group(hv, af[c >> 2], ring[2 * R - ap][s], c & 3);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (!BOX) {
          // line along k through the centre (row offset r), centre excluded
          const float* colp = win + (8 * w + orow + R) * PW::PITCH + PW::COL0 + 4 * beta;
#pragma unroll
          for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int e = 0; e < NB; ++e)
              ring[R][s] = mfma4_agroup(af[(NB + e) >> 2], colp[4 * s * PW::PITCH + e], ring[R][s], (NB + e) & 3);
          // i arm: this plane's centre values reach output plane i - ap + r
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const float4 ctr =
                *reinterpret_cast<const float4*>(win + (8 * w + 4 * s + orow + R) * PW::PITCH + 4 + 4 * beta);
#pragma unroll
            for (int ap = 0; ap < W; ++ap) {
              if (ap == R) continue;
              ring[2 * R - ap][s][0] += ci[ap] * ctr.x;
              ring[2 * R - ap][s][1] += ci[ap] * ctr.y;
              ring[2 * R - ap][s][2] += ci[ap] * ctr.z;
              ring[2 * R - ap][s][3] += ci[ap] * ctr.w;
            }
          }
        }
      },
      [&](int64_t o, bool live) {
        if (live) {
          const int64_t gk = ch.k0 + 4 * beta;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const int64_t gj = ch.j0 + 8 * w + 4 * s + orow;
            if (gj >= Nj) continue;
            float* dst = out + o * plane + gj * Nk + gk;
            if constexpr (DMA) {  // k extent a multiple of 4, output 16-byte aligned
              if (gk < Nk) *reinterpret_cast<float4*>(dst) = float4{ring[0][s][0], ring[0][s][1], ring[0][s][2], ring[0][s][3]};
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (gk + e < Nk) dst[e] = ring[0][s][e];
            }
          }
        }
#pragma unroll
        for (int z = 0; z < 2 * R; ++z)
#pragma unroll
          for (int t = 0; t < 2; ++t) ring[z][t] = ring[z + 1][t];
#pragma unroll
        for (int t = 0; t < 2; ++t) ring[2 * R][t] = floatx4{0, 0, 0, 0};
      });
}

template <int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads) void mfma3d_b4_kernel(KArgs a) {
  mfma3d_b4_item<R, BOX, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads) void mfma3d_b4_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { mfma3d_b4_item<R, BOX, DMA>(x, id); });
}

// ---------------------------------------------------------------------------
// 3D boxes of radius >= 2 on n = 4 blocks.  The (2r+1)^2 lines along j,
// CLS(a, *, c), scatter input plane i into output plane i - a + r (ring slot
// 2r - a).  For one column offset c the lines of all 2r+1 planes a read the
// same input column, so each window row value is read from LDS once and feeds
// (2r+1) x 2 MFMAs.  The (2r+1)^2 (4 + 2r) band vectors (972 at r = 4) do not
// fit in registers: a table in LDS holds them in the packed lane order (four
// vectors per register, one per 16-lane group, selected with the B lane-group
// broadcast), and the 2r+1 planes' vectors of one column offset are loaded
// before its rows.  Ring and tile layout as mfma3d_b4_item.
// ---------------------------------------------------------------------------
template <int R, bool DMA>
__device__ __forceinline__ void mfma3d_b4box_item(const KArgs& a, int item) {
  constexpr int W = 2 * R + 1, NB = 4 + 2 * R;
  constexpr int NQ = W * NB, NPC = (NQ + 3) / 4;  // vectors and packed registers per column offset
  typedef PlaneWalk<float, R, kTJ + 2 * R, DMA, true> PW;
  static_assert(PW::COL0 + R == 4, "tile body at LDS column 4");
  // one LDS object (separate ones make the compiler wait for the plane in
  // flight before LDS accesses): the plane buffers, then ptab[(c NPC + k) 16 +
  // 4 g + j], vector q = 4 k + g of column offset c (plane a = q / NB, band
  // row d = q % NB) for block row j
  __shared__ __attribute__((aligned(16))) float bufs[PW::NBUF * PW::BUF + W * NPC * 16];
  float* ptab = bufs + PW::NBUF * PW::BUF;

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int orow = lane & 3, beta = lane >> 2;

  // the plan's compact fragments: line l = a (2r+1) + c, vector l NB + d,
  // its value for block row j at frag[4 (l NB + d) + j]
  const float* __restrict__ frag = (const float*)a.frag;
  for (int e = threadIdx.x; e < W * NPC * 16; e += kThreads) {
    const int j = e & 3, g = (e >> 2) & 3, k = (e >> 4) % NPC, c = (e >> 4) / NPC;
    const int q = 4 * k + g;
    ptab[e] = q < NQ ? frag[(((q / NB) * W + c) * NB + q % NB) * 4 + j] : 0.0f;
  }
  __syncthreads();
  const float* lanetab = ptab + 4 * (lane >> 4) + (lane & 3);

  floatx4 ring[W][2];
#pragma unroll
  for (int z = 0; z < W; ++z)
#pragma unroll
    for (int t = 0; t < 2; ++t) ring[z][t] = floatx4{0, 0, 0, 0};

  PW::walk(
      bufs, a, ch,
      [&](const float* win, bool valid) {
        if (!valid) return;
#pragma unroll
        for (int cs = 0; cs < W; ++cs) {
          float pf[NPC];
#pragma unroll
          for (int k = 0; k < NPC; ++k) pf[k] = lanetab[(cs * NPC + k) * 16];
          const float* rowp = win + (8 * w) * PW::PITCH + PW::COL0 + lane + cs;
#pragma unroll
          for (int x = 0; x < 8 + 2 * R; ++x) {
            const float hv = rowp[x * PW::PITCH];
#pragma unroll
            for (int ap = 0; ap < W; ++ap)
#pragma unroll
              for (int s = 0; s < 2; ++s) {
                const int d = x - 4 * s, q = ap * NB + d;
                if (d < 0 || d >= NB) continue;
                ring[2 * R - ap][s] = mfma4_group(hv, pf[q >> 2], ring[2 * R - ap][s], q & 3);
              }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      },
      [&](int64_t o, bool live) {
        if (live) {
          const int64_t gk = ch.k0 + 4 * beta;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const int64_t gj = ch.j0 + 8 * w + 4 * s + orow;
            if (gj >= Nj) continue;
            float* dst = out + o * plane + gj * Nk + gk;
            if constexpr (DMA) {  // k extent a multiple of 4, output 16-byte aligned
              if (gk < Nk) *reinterpret_cast<float4*>(dst) = float4{ring[0][s][0], ring[0][s][1], ring[0][s][2], ring[0][s][3]};
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (gk + e < Nk) dst[e] = ring[0][s][e];
            }
          }
        }
#pragma unroll
        for (int z = 0; z < 2 * R; ++z)
#pragma unroll
          for (int t = 0; t < 2; ++t) ring[z][t] = ring[z + 1][t];
#pragma unroll
        for (int t = 0; t < 2; ++t) ring[2 * R][t] = floatx4{0, 0, 0, 0};
      });
}

template <int R, bool DMA>
__global__ __launch_bounds__(kThreads) void mfma3d_b4box_kernel(KArgs a) {
  mfma3d_b4box_item<R, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int R, bool DMA>
__global__ __launch_bounds__(kThreads) void mfma3d_b4box_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { mfma3d_b4box_item<R, DMA>(x, id); });
}

// ---------------------------------------------------------------------------
// Outer-product form with 16-bit split operands (see kernels_split2d.hpp) in
// the plane order of Algorithm 1.  Lines run along k: CLS(a, b, *) adds
// D[p][q] += sum_y H[p + b][y] * S_{a,b}[y][q], S_{a,b}[y][q] = C^g[a][b][y - q],
// to output plane i - a + r (window rows shifted by b as the A operand).
// Box: all (2r+1)^2 lines on MFMA; at r = 1 their 27 x 2 band fragments
// stay in registers.  From r = 2 (25 to 81 lines) they come from an LDS
// table: lane (g, q) of line (a, b) holds S_{a,b}[8 g + e][q] = C^g[a][b][d + e]
// (e = 0..7, d = 8 g - q), which is zero unless d lies in -7 .. 2r, so a line
// has only 2r + 8 distinct nonzero fragments per hi / lo part.  The parts'
// blocks follow each other, a zero fragment before each and after the last,
// and a lane reads entry clamp(d + 8, 0, 2r + 9) of every block (the last is
// the next block's zero): one lane address, the blocks at immediate
// offsets.  The A operand (window rows shifted by b) is read once per b and
// feeds the lines of all 2r + 1 planes a; the reads of a line go out two
// lines ahead of its products.  Star: the k line
// CLS(r, r, *) on MFMA; the other 4r lines hold one weight each and are vector
// FMAs on the FP32 window (j arm on the centre plane, i arm into the other
// ring slots), pre-multiplied by the plan's coefficient scale.  Each staged
// FP32 window is split once into hi/lo 16-bit planes.
// ---------------------------------------------------------------------------
template <int R, bool BOX>
struct Split3DShape {
  static constexpr int W = 2 * R + 1;
  static constexpr int NL = BOX ? W * W : 1;
  static constexpr int WROWS = kTJ + 2 * R;
  static constexpr int WEND = kTK + 2 * R;
  // 16-bit pitch: multiple of 8, covers the columns read by K = 32; 88
  // spreads a read's 16 rows over all LDS banks, 80 leaves the order-4 box
  // (with its fragment table) under half the LDS: two workgroups per CU
  static constexpr int P = BOX && R == 4 ? 80 : 88;
  static_assert((kTK - 32) + 16 + 32 <= P && WEND <= P, "pitch too small");
};

// Issue order of the box lines' LDS reads and MFMAs (line n = plane a =
// n mod W, row shift b = n / W): the reads of line n + 2 (its two band
// fragments, and the four A operands of its b when it opens one) go out
// ahead of the six products of line n, so the products of two lines cover
// the LDS latency of every read.
template <int W>
constexpr int split_box_reads(int n) { return n >= W * W ? 0 : 2 + (n % W == 0 ? 4 : 0); }

template <int W, int N = 0>
__device__ __forceinline__ void split_box_schedule() {
  constexpr int L = W * W, P = 2;
  if constexpr (N == 0) __builtin_amdgcn_sched_group_barrier(0x100, split_box_reads<W>(0) + split_box_reads<W>(1), 0);
  if constexpr (N < L) {
    if constexpr (N + P < L) __builtin_amdgcn_sched_group_barrier(0x100, split_box_reads<W>(N + P), 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
    split_box_schedule<W, N + 1>();
  }
}

template <int KIND, int R, bool BOX, bool DMA>
__device__ __forceinline__ void split3d_item(const KArgs& a, int item) {
  typedef Split3DShape<R, BOX> S;
  typedef PlaneWalk<float, R, S::WROWS, DMA> PW;
  constexpr int W = S::W;
  // one LDS object (separate ones make the compiler wait for the plane in
  // flight before LDS accesses): the plane buffers, then the hi and lo
  // planes, then (box, r >= 2) the band fragment table
  constexpr bool TABLE = BOX && R >= 2;
  constexpr int ND = 2 * R + 8;                                 // nonzero fragments of a line, d = -7 .. 2r
  constexpr int NB = ND + 1;                                    // stride of a line's part: zero, d = -7 .. 2r
  static_assert(ND <= 16, "a fragment's source lane is 16 + 15 - (d + 7)");
  constexpr int PLANE = (S::WROWS * S::P * 2 + 15) / 16 * 4;  // floats per 16-bit plane
  // stars from order 2 split their k line's A operand in registers (order 1:
  // 588 vs 554 GStencil/s at 512^3 with the LDS planes, order 4: 439 vs 455
  // at 384^3 without them)
  constexpr bool REGA = !BOX && R >= 2;
  constexpr int NPLANE = REGA ? 0 : 2;  // hi/lo planes
  constexpr int TAB0 = round_up(PW::NBUF * PW::BUF + NPLANE * PLANE, 4);
  constexpr int NTAB = TABLE ? S::NL * 2 * NB + 1 : 0;         // fragments, a zero one last
  __shared__ __attribute__((aligned(16))) float bufs[TAB0 + 4 * NTAB];
  uint16_t* lhi = reinterpret_cast<uint16_t*>(bufs + PW::NBUF * PW::BUF);
  uint16_t* llo = reinterpret_cast<uint16_t*>(bufs + PW::NBUF * PW::BUF + PLANE);
  u16x8* tab = reinterpret_cast<u16x8*>(bufs + TAB0);

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wj = w >> 1, wk = w & 1;
  const int g = lane >> 4, q = lane & 15;

  const u16x8* __restrict__ frag = (const u16x8*)a.frag;
  constexpr int NLR = TABLE ? 1 : S::NL;  // lines whose fragments sit in registers
  u16x8 bh[NLR], bl[NLR];
  // table: fragment (line l, part h, d) at (2 l + h) NB + d + 8, copied from
  // lane 16 + 8 - d of the packed fragments (g = 1, q = 8 - d); the entries
  // at multiples of NB are zero
  const u16x8* tlane = tab;
  if constexpr (TABLE) {
    for (int e = threadIdx.x; e < NTAB; e += kThreads) {
      u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
      const int lh = e / NB, i = e - lh * NB;
      if (i != 0) v = frag[lh * 64 + 32 - i];
      tab[e] = v;
    }
    const int di = 8 * g - q + 8;
    tlane = tab + (di < 0 ? 0 : di > NB ? NB : di);
  } else {
#pragma unroll
    for (int l = 0; l < S::NL; ++l) {
      bh[l] = frag[(l * 2 + 0) * 64 + lane];
      bl[l] = frag[(l * 2 + 1) * 64 + lane];
    }
  }
  const float cscale = 1.0f / a.out_scale;  // exact power of two
  float cj[W], ci[W];                        // star: j-arm and i-arm weights, scaled
  if constexpr (!BOX) {
    const float* __restrict__ c = (const float*)a.coef;
#pragma unroll
    for (int b = 0; b < W; ++b) {
      cj[b] = c[(R * W + b) * W + R] * cscale;
      ci[b] = c[(b * W + R) * W + R] * cscale;
    }
  }
  if constexpr (!REGA) {
    zero_region<uint16_t, kThreads>(lhi, S::WROWS, S::P - S::WEND, S::P, 0, S::WEND);
    zero_region<uint16_t, kThreads>(llo, S::WROWS, S::P - S::WEND, S::P, 0, S::WEND);
  }
  const float lo_mul = 1.0f / a.lo_scale;
  const float ls = a.lo_scale, os = a.out_scale;

  // Box: every ring slot takes MFMA products, so the cross terms (hi*lo +
  // lo*hi) keep a ring of their own.  Star: only the centre plane's slot takes
  // the k line's products, so its cross terms are folded into acc at once.
  constexpr int WX = BOX ? W : 1;
  floatx4 acc[W][2], acx[WX][2];
#pragma unroll
  for (int z = 0; z < W; ++z)
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[z][t] = floatx4{0, 0, 0, 0};
#pragma unroll
  for (int z = 0; z < WX; ++z)
#pragma unroll
    for (int t = 0; t < 2; ++t) acx[z][t] = floatx4{0, 0, 0, 0};
  // ring slot z holds output plane i - r + z while input plane i is
  // scattered; slot 0 is stored after the plane.  Stars and the 27-point box
  // rotate the ring: at plane phase PH (input plane u, PH = u mod W) slot z
  // sits in register set (z + PH) mod W, and the stored set is cleared for
  // the next plane's top slot.  The table boxes (order >= 2: up to 486 MFMAs
  // per plane) keep one copy of the plane code and shift the ring down.
  constexpr bool ROT = !TABLE;
  auto body = [&](const float* win, bool valid, auto phase) __attribute__((always_inline)) {
        constexpr int PH = ROT ? decltype(phase)::value : 0;
        if (!valid) return;
        if constexpr (!REGA) {
          // split the FP32 window into hi/lo planes, read by every wave (a
          // star's k line reads the rows r .. r + TJ - 1)
          constexpr int HALF = S::WEND / 2;
          constexpr int SROW0 = BOX ? 0 : R, SROWS = BOX ? S::WROWS : kTJ;
          for (int idx = threadIdx.x; idx < SROWS * HALF; idx += kThreads) {
            const int row = SROW0 + idx / HALF, y = 2 * (idx - (idx / HALF) * HALF);
            const float* src = win + row * PW::PITCH + PW::COL0 + y;
            uint16_t h0, l0, h1, l1;
            Split16<KIND>::split(src[0], lo_mul, h0, l0);
            Split16<KIND>::split(src[1], lo_mul, h1, l1);
            *reinterpret_cast<uint32_t*>(lhi + row * S::P + y) = (uint32_t)h0 | ((uint32_t)h1 << 16);
            *reinterpret_cast<uint32_t*>(llo + row * S::P + y) = (uint32_t)l0 | ((uint32_t)l1 << 16);
          }
          lds_barrier();
        }
        if constexpr (TABLE) {
          // per accumulator the products come in the order of the loop below
          // (b ascending; hi*lo before lo*hi)
#pragma unroll
          for (int b = 0; b < W; ++b) {
            const uint16_t* ph = lhi + (16 * wj + b + q) * S::P + 32 * wk + 8 * g;
            const uint16_t* pl = llo + (16 * wj + b + q) * S::P + 32 * wk + 8 * g;
            u16x8 ah[2], al[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              ah[t] = *reinterpret_cast<const u16x8*>(ph + 16 * t);
              al[t] = *reinterpret_cast<const u16x8*>(pl + 16 * t);
            }
#pragma unroll
            for (int ap = 0; ap < W; ++ap) {
              const int slot = (2 * R - ap + PH) % W, l = ap * W + b;
              const u16x8 vh = tlane[2 * l * NB], vl = tlane[(2 * l + 1) * NB];
#pragma unroll
              for (int t = 0; t < 2; ++t) {
                acc[slot][t] = Split16<KIND>::mma(ah[t], vh, acc[slot][t]);
                acx[slot][t] = Split16<KIND>::mma(ah[t], vl, acx[slot][t]);
                acx[slot][t] = Split16<KIND>::mma(al[t], vh, acx[slot][t]);
              }
            }
          }
          split_box_schedule<W>();
          __builtin_amdgcn_sched_barrier(0);
        } else if constexpr (REGA) {
          // the k line's A operand straight from the FP32 window: lane (g, q)
          // takes row 16 wj + r + q, window columns 32 wk + 16 t + 8 g .. + 7
          // (zero from the window's end on, where the band is zero too), and
          // splits them in registers -- the same values the box path stages
          // in LDS, without the planes and their barrier
          const int slot = (R + PH) % W;
          const float* arow = win + (16 * wj + R + q) * PW::PITCH + PW::COL0 + 32 * wk + 8 * g;
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            u16x8 ah, al;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int y = 32 * wk + 16 * t + 8 * g + e;
              const float x = y < S::WEND ? arow[16 * t + e] : 0.0f;
              uint16_t h, l;
              Split16<KIND>::split(x, lo_mul, h, l);
              ah[e] = h;
              al[e] = l;
            }
            acc[slot][t] = Split16<KIND>::mma(ah, bh[0], acc[slot][t]);
            acx[0][t] = Split16<KIND>::mma(ah, bl[0], acx[0][t]);
            acx[0][t] = Split16<KIND>::mma(al, bh[0], acx[0][t]);
          }
        } else {
#pragma unroll
          for (int ap = 0; ap < W; ++ap) {
            if (!BOX && ap != R) continue;
            const int slot = (2 * R - ap + PH) % W;
#pragma unroll
            for (int b = 0; b < W; ++b) {
              if (!BOX && b != R) continue;
              const int l = BOX ? ap * W + b : 0;
              const uint16_t* ph = lhi + (16 * wj + b + q) * S::P + 32 * wk + 8 * g;
              const uint16_t* pl = llo + (16 * wj + b + q) * S::P + 32 * wk + 8 * g;
#pragma unroll
              for (int t = 0; t < 2; ++t) {
                const u16x8 ah = *reinterpret_cast<const u16x8*>(ph + 16 * t);
                const u16x8 al = *reinterpret_cast<const u16x8*>(pl + 16 * t);
                const int xs = BOX ? slot : 0;
                acc[slot][t] = Split16<KIND>::mma(ah, bh[l], acc[slot][t]);
                acx[xs][t] = Split16<KIND>::mma(ah, bl[l], acx[xs][t]);
                acx[xs][t] = Split16<KIND>::mma(al, bh[l], acx[xs][t]);
              }
            }
          }
        }
        if constexpr (!BOX) {
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            acc[(R + PH) % W][t] += ls * acx[0][t];
            acx[0][t] = floatx4{0, 0, 0, 0};
          }
        }
        if constexpr (!BOX) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float* cp = win + (16 * wj + 4 * g + v) * PW::PITCH + PW::COL0 + 32 * wk + q + R;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              float sj = 0.0f;
#pragma unroll
              for (int b = 0; b < W; ++b) {
                if (b == R) continue;
                sj += cj[b] * cp[b * PW::PITCH + 16 * t];
              }
              acc[(R + PH) % W][t][v] += sj;
              const float ctr = cp[R * PW::PITCH + 16 * t];
#pragma unroll
              for (int ap = 0; ap < W; ++ap) {
                if (ap == R) continue;
                acc[(2 * R - ap + PH) % W][t][v] += ci[ap] * ctr;
              }
            }
          }
        }
  };
  auto finish = [&](int64_t o, bool live, auto phase) __attribute__((always_inline)) {
        constexpr int Z0 = ROT ? decltype(phase)::value : 0;  // register set of slot 0
        if (live) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t gj = ch.j0 + 16 * wj + 4 * g + v;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const int64_t gk = ch.k0 + 32 * wk + 16 * t + q;
              const float v0 = BOX ? acc[Z0][t][v] + ls * acx[Z0][t][v] : acc[Z0][t][v];
              if (gj < Nj && gk < Nk) out[o * plane + gj * Nk + gk] = v0 * os;
            }
          }
        }
        if constexpr (!ROT) {
#pragma unroll
          for (int z = 0; z < 2 * R; ++z)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              acc[z][t] = acc[z + 1][t];
              if constexpr (BOX) acx[z][t] = acx[z + 1][t];
            }
        }
        constexpr int ZT = ROT ? Z0 : 2 * R;  // the next plane's top slot
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          acc[ZT][t] = floatx4{0, 0, 0, 0};
          if constexpr (BOX) acx[ZT][t] = floatx4{0, 0, 0, 0};
        }
  };
  if constexpr (ROT) {
    PW::walk_phased(bufs, a, ch, body, finish);
  } else {
    PW::walk(
        bufs, a, ch, [&](const float* win, bool valid) { body(win, valid, std::integral_constant<int, 0>{}); },
        [&](int64_t o, bool live) { finish(o, live, std::integral_constant<int, 0>{}); });
  }
}

// ---------------------------------------------------------------------------
// Split-precision star in the hybrid cover of Table 2 (the line assignment of
// the FP32 n = 4 kernel): on every input plane the two in-plane lines through
// the centre run as BF16/FP16 hi/lo products on 16x16x32 MFMAs -- the line
// along k, CLS(r, r, *) (centre included), as D[p][q] += sum_y H[p][y] S[y][q]
// (A = eight consecutive k values of one row: one 16-byte LDS read), and the
// line along j, CLS(r, *, r) (centre excluded), as D[p][q] += sum_x T[p][x]
// H[x][q] with the band T[p][x] = C^g[r][x - p][r] as the A operand and B =
// eight consecutive j values of one column, read as 16-bit elements (lanes of
// a row read neighbouring elements: no bank conflicts) -- and the 2r lines
// CLS(a, *, r), a != r, one weight each, are the vector FMAs of the i arm into
// the other ring slots.  Each FP32 window is split once into row-major hi/lo
// planes.  Both lines' products land in the same accumulator layout; their
// cross terms (hi*lo + lo*hi) are summed apart and folded into the centre
// plane's slot.
// ---------------------------------------------------------------------------
template <int R>
struct SplitStar3DShape {
  static constexpr int W = 2 * R + 1;
  static constexpr int WROWS = kTJ + 2 * R;   // window rows (global j0 - r ..)
  static constexpr int WCOLS = kTK + 2 * R;   // window columns (global k0 - r ..)
  static constexpr int PR = kTJ + 16;         // plane rows: the j line's K = 32 reads rows up to 47
  static constexpr int P = 88;                // 16-bit pitch: the k line's K = 32 reads columns up to 79
  static_assert((kTK - 32) + 16 + 32 <= P && WCOLS <= P && WROWS <= PR, "plane too small");
};

template <int KIND, int R, bool DMA>
__device__ __forceinline__ void split3d_hybrid_item(const KArgs& a, int item) {
  typedef SplitStar3DShape<R> S;
  typedef PlaneWalk<float, R, S::WROWS, DMA, true> PW;
  static_assert(PW::COL0 + R == 4, "tile body at LDS column 4");
  constexpr int W = S::W;
  // one LDS object (separate ones make the compiler wait for the plane in
  // flight before LDS accesses): the plane buffers, then the hi and lo planes
  constexpr int PLANE = (S::PR * S::P * 2 + 15) / 16 * 4;  // floats per 16-bit plane
  __shared__ __attribute__((aligned(16))) float bufs[PW::NBUF * PW::BUF + 2 * PLANE];
  uint16_t* lhi = reinterpret_cast<uint16_t*>(bufs + PW::NBUF * PW::BUF);
  uint16_t* llo = reinterpret_cast<uint16_t*>(bufs + PW::NBUF * PW::BUF + PLANE);

  const Chunk3D ch = decode_chunk(a, item);
  const int64_t Nj = a.d1, Nk = a.d2, plane = Nj * Nk;
  float* __restrict__ out = (float*)a.out;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wj = w >> 1, wk = w & 1;
  const int g = lane >> 4, q = lane & 15;

  // line 0: along k (B operand S[y][q]); line 1: along j (A operand T[p][x]);
  // both bands pack as w[8 (l / 16) + e - l % 16] in lane l, element e
  const u16x8* __restrict__ frag = (const u16x8*)a.frag;
  const u16x8 kh = frag[0 * 64 + lane], kl = frag[1 * 64 + lane];
  const u16x8 jh = frag[2 * 64 + lane], jl = frag[3 * 64 + lane];
  const float cscale = 1.0f / a.out_scale;  // exact power of two
  float ci[W];                               // i-arm weights C^g[a][r][r], scaled
  {
    const float* __restrict__ c = (const float*)a.coef;
#pragma unroll
    for (int b = 0; b < W; ++b) ci[b] = c[(b * W + R) * W + R] * cscale;
  }
  // padding the MFMAs read with zero weights (columns past the window, rows
  // past it): keep it finite
  zero_region<uint16_t, kThreads>(lhi, S::WROWS, S::P - S::WCOLS, S::P, 0, S::WCOLS);
  zero_region<uint16_t, kThreads>(llo, S::WROWS, S::P - S::WCOLS, S::P, 0, S::WCOLS);
  zero_region<uint16_t, kThreads>(lhi, S::PR - S::WROWS, S::P, S::P, S::WROWS, 0);
  zero_region<uint16_t, kThreads>(llo, S::PR - S::WROWS, S::P, S::P, S::WROWS, 0);
  const float lo_mul = 1.0f / a.lo_scale;
  const float ls = a.lo_scale, os = a.out_scale;

  floatx4 acc[W][2], acx[2];
#pragma unroll
  for (int z = 0; z < W; ++z)
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[z][t] = floatx4{0, 0, 0, 0};
  // ring slot z holds output plane i - r + z while input plane i is
  // scattered, in register set (z + PH) mod W at plane phase PH (the ring
  // rotates: slot 0 is stored after the plane and its set cleared for the
  // next plane's top slot)
  PW::walk_phased(
      bufs, a, ch,
      [&](const float* win, bool valid, auto phase) __attribute__((always_inline)) {
        constexpr int PH = decltype(phase)::value;
        if (!valid) return;
        // split the FP32 window into hi/lo planes, two columns per thread and step
        constexpr int HALF = S::WCOLS / 2;
        for (int idx = threadIdx.x; idx < S::WROWS * HALF; idx += kThreads) {
          const int row = idx / HALF, y = 2 * (idx - (idx / HALF) * HALF);
          const float* src = win + row * PW::PITCH + PW::COL0 + y;
          uint16_t h0, l0, h1, l1;
          Split16<KIND>::split(src[0], lo_mul, h0, l0);
          Split16<KIND>::split(src[1], lo_mul, h1, l1);
          *reinterpret_cast<uint32_t*>(lhi + row * S::P + y) = (uint32_t)h0 | ((uint32_t)h1 << 16);
          *reinterpret_cast<uint32_t*>(llo + row * S::P + y) = (uint32_t)l0 | ((uint32_t)l1 << 16);
        }
        lds_barrier();
#pragma unroll
        for (int t = 0; t < 2; ++t) acx[t] = floatx4{0, 0, 0, 0};
        // k line: rows r + 16 wj + q, columns 32 wk + 16 t + 8 g ..
        const uint16_t* pkh = lhi + (R + 16 * wj + q) * S::P + 32 * wk + 8 * g;
        const uint16_t* pkl = llo + (R + 16 * wj + q) * S::P + 32 * wk + 8 * g;
        // j line: rows 16 wj + 8 g + e, column r + 32 wk + 16 t + q
        const uint16_t* pjh = lhi + (16 * wj + 8 * g) * S::P + R + 32 * wk + q;
        const uint16_t* pjl = llo + (16 * wj + 8 * g) * S::P + R + 32 * wk + q;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const u16x8 ah = *reinterpret_cast<const u16x8*>(pkh + 16 * t);
          const u16x8 al = *reinterpret_cast<const u16x8*>(pkl + 16 * t);
          acc[(R + PH) % W][t] = Split16<KIND>::mma(ah, kh, acc[(R + PH) % W][t]);
          acx[t] = Split16<KIND>::mma(ah, kl, acx[t]);
          acx[t] = Split16<KIND>::mma(al, kh, acx[t]);
          u16x8 bh, bl;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            bh[e] = pjh[e * S::P + 16 * t];
            bl[e] = pjl[e * S::P + 16 * t];
          }
          acc[(R + PH) % W][t] = Split16<KIND>::mma(jh, bh, acc[(R + PH) % W][t]);
          acx[t] = Split16<KIND>::mma(jl, bh, acx[t]);
          acx[t] = Split16<KIND>::mma(jh, bl, acx[t]);
        }
        // i arm: this plane's centre values reach output plane i - ap + r
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float* cp = win + (16 * wj + 4 * g + v + R) * PW::PITCH + PW::COL0 + R + 32 * wk + q;
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const float ctr = cp[16 * t];
#pragma unroll
            for (int ap = 0; ap < W; ++ap) {
              if (ap == R) continue;
              acc[(2 * R - ap + PH) % W][t][v] += ci[ap] * ctr;
            }
          }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[(R + PH) % W][t] += ls * acx[t];
      },
      [&](int64_t o, bool live, auto phase) __attribute__((always_inline)) {
        constexpr int Z0 = decltype(phase)::value;  // register set of slot 0
        if (live) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t gj = ch.j0 + 16 * wj + 4 * g + v;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const int64_t gk = ch.k0 + 32 * wk + 16 * t + q;
              if (gj < Nj && gk < Nk) out[o * plane + gj * Nk + gk] = acc[Z0][t][v] * os;
            }
          }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[Z0][t] = floatx4{0, 0, 0, 0};
      });
}

template <int KIND, int R, bool DMA>
__global__ __launch_bounds__(kThreads) void split3d_hybrid_kernel(KArgs a) {
  split3d_hybrid_item<KIND, R, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int KIND, int R, bool DMA>
__global__ __launch_bounds__(kThreads) void split3d_hybrid_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { split3d_hybrid_item<KIND, R, DMA>(x, id); });
}

// Boxes of order 3 and 4 (direct-to-LDS planes): registers for two waves
// per SIMD (order 2 fits them anyway)
template <int R, bool BOX, bool DMA>
constexpr int split3d_waves() { return BOX && (R == 3 || (R == 4 && DMA)) ? 2 : 1; }

template <int KIND, int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads, (split3d_waves<R, BOX, DMA>())) void split3d_kernel(KArgs a) {
  split3d_item<KIND, R, BOX, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int KIND, int R, bool BOX, bool DMA>
__global__ __launch_bounds__(kThreads, (split3d_waves<R, BOX, DMA>())) void split3d_batch(BatchArgs b) {
  for_each_batch_item(b, [&](const KArgs& x, int id) { split3d_item<KIND, R, BOX, DMA>(x, id); });
}

}  // namespace stencil
