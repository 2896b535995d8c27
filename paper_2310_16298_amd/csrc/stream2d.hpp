// Row streaming for the 2D kernels.
//
// A workgroup owns a strip of TN columns and walks down it in blocks of BM
// output rows.  The LDS window holds BM + 2r input rows (+ r halo columns on
// each side).  Between blocks the bottom 2r rows move to the top (the input
// rows shared by consecutive blocks are loaded from HBM once), and the BM new
// rows -- prefetched into registers while the previous block was being
// computed -- are written below them.  The boundary rule (zero or periodic)
// is applied while fetching, exactly as in stage_window.
#pragma once

#include "device_common.hpp"

namespace stencil {

// Registers holding BM new window rows (body TN columns + 2r halo columns).
template <typename T, int R, int BM, int TN, int NT>
struct RowPrefetch {
  static constexpr int VEC = 16 / (int)sizeof(T);
  static constexpr int NV = TN / VEC;                    // vectors per row
  static constexpr int NB = (BM * NV + NT - 1) / NT;     // body vectors per thread
  static constexpr int NH = (BM * 2 * R + NT - 1) / NT;  // halo values per thread
  typedef typename Vec16<T>::type V;
  V body[NB];
  T halo[NH];

  // Fetch global rows grow0 .. grow0 + BM - 1 of the strip starting at
  // column c0 (window column r).  `fast`: the strip's body lies inside the
  // grid and rows are 16-byte aligned.
  __device__ __forceinline__ void fetch(const T* __restrict__ src, int64_t M, int64_t N, int64_t grow0, int64_t c0,
                                        bool periodic, bool fast) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int idx = tid + k * NT;
      const int row = idx / NV, v = idx - (idx / NV) * NV;
      V val = V{};
      if (idx < BM * NV) {
        const int64_t g = map_index(grow0 + row, M, periodic);
        if (g >= 0) {
          if (fast) {
            val = *reinterpret_cast<const V*>(src + g * N + c0 + v * VEC);
          } else {
            T* pv = reinterpret_cast<T*>(&val);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
              const int64_t c = map_index(c0 + v * VEC + e, N, periodic);
              pv[e] = c >= 0 ? src[g * N + c] : T(0);
            }
          }
        }
      }
      body[k] = val;
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int idx = tid + k * NT;
      T val = T(0);
      if (idx < BM * 2 * R) {
        const int row = idx / (2 * R), h = idx - (idx / (2 * R)) * (2 * R);
        const int64_t gc = (h < R) ? (c0 - R + h) : (c0 + TN + (h - R));
        const int64_t g = map_index(grow0 + row, M, periodic);
        const int64_t c = map_index(gc, N, periodic);
        if (g >= 0 && c >= 0) val = src[g * N + c];
      }
      halo[k] = val;
    }
  }

  // Write the fetched rows to LDS window rows lrow0 .. lrow0 + BM - 1 through
  // `put(row, y, value)` (y = window column) or `put_vec(row, y, V)`.
  template <class Writer>
  __device__ __forceinline__ void commit(int lrow0, Writer& wr) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int idx = tid + k * NT;
      if (idx < BM * NV) {
        const int row = idx / NV, v = idx - (idx / NV) * NV;
        wr.put_vec(lrow0 + row, R + v * VEC, body[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int idx = tid + k * NT;
      if (idx < BM * 2 * R) {
        const int row = idx / (2 * R), h = idx - (idx / (2 * R)) * (2 * R);
        const int y = (h < R) ? h : (TN + h);
        wr.put(lrow0 + row, y, halo[k]);
      }
    }
  }
};

// Writer for a plain LDS window: element (row, y) at lds[row * PITCH + COL0 + y].
template <typename T, int R, int PITCH>
struct PlainWriter {
  T* lds;
  static constexpr int COL0 = lds_col0<T, R>();
  static constexpr int VEC = 16 / (int)sizeof(T);
  typedef typename Vec16<T>::type V;
  __device__ __forceinline__ void put(int row, int y, T v) { lds[row * PITCH + COL0 + y] = v; }
  __device__ __forceinline__ void put_vec(int row, int y, const V& v) {
    T* dst = lds + row * PITCH + COL0 + y;
    if constexpr (PITCH % VEC == 0) {
      *reinterpret_cast<V*>(dst) = v;  // COL0 + r is a multiple of VEC
    } else {
      const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int e = 0; e < VEC; ++e) dst[e] = pv[e];
    }
  }
};

// Registers carrying the bottom 2r window rows of one LDS array to the top
// between blocks: loaded before the block's final barrier, stored after it.
template <typename U, int R, int COLS, int NT>
struct RowMover {
  static constexpr int NM = (2 * R * COLS + NT - 1) / NT;
  U v[NM];
  // get(rr, cc): element cc of window row BM + rr
  template <class Get>
  __device__ __forceinline__ void load(Get get) {
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int idx = threadIdx.x + k * NT;
      if (idx < 2 * R * COLS) v[k] = get(idx / COLS, idx - (idx / COLS) * COLS);
    }
  }
  // put(rr, cc, value): element cc of window row rr
  template <class Put>
  __device__ __forceinline__ void store(Put put) const {
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int idx = threadIdx.x + k * NT;
      if (idx < 2 * R * COLS) put(idx / COLS, idx - (idx / COLS) * COLS, v[k]);
    }
  }
};

// Whether a strip at column c0 can use the vectorised fetch.
template <typename T>
__device__ __forceinline__ bool strip_fast(const T* src, int64_t N, int64_t c0, int TN) {
  return (c0 + TN <= N) && (N % (16 / (int)sizeof(T)) == 0) && ((reinterpret_cast<uintptr_t>(src) & 15) == 0);
}

// Work items (column strip x row chunk) for strips of TN columns walked in
// blocks of BM rows.  Chunks hold `chunk` rows when chunk > 0 (rounded up to
// BM), else are sized for about `target` items.  Fills a.tiles0 (chunks),
// a.tiles1 (strips), a.chunk (rows) and returns the number of items.
inline int64_t strip_grid(KArgs& a, int TN, int BM, int64_t target, int32_t chunk_req = 0) {
  const int64_t strips = (a.d1 + TN - 1) / TN;
  const int64_t rows = (a.d0 + BM - 1) / BM * BM;
  int64_t chunk = chunk_req > 0 ? chunk_req : a.d0 * strips / target;
  chunk = (chunk < BM ? BM : chunk + BM - 1) / BM * BM;
  if (chunk > rows) chunk = rows;
  const int64_t nch = (a.d0 + chunk - 1) / chunk;
  a.tiles0 = (int32_t)nch;
  a.tiles1 = (int32_t)strips;
  a.chunk = (int32_t)chunk;
  a.nchunks = (int32_t)nch;
  return strips * nch;
}

// Strip decomposition of a 2D grid: tiles0 = row chunks, tiles1 = column strips.
struct Strip2D {
  int64_t i0, i1, j0;  // output rows [i0, i1), strip column origin j0
};
__device__ __forceinline__ Strip2D decode_strip(const KArgs& a, int id, int TN) {
  const int chunk = id / a.tiles1;
  const int strip = id - chunk * a.tiles1;
  Strip2D s;
  s.i0 = (int64_t)chunk * a.chunk;
  s.i1 = s.i0 + a.chunk < a.d0 ? s.i0 + a.chunk : a.d0;
  s.j0 = (int64_t)strip * TN;
  return s;
}

}  // namespace stencil
