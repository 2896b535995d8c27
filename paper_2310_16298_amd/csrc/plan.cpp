// Host-side plan construction.
//
// A coefficient line (Section 3.2, "coefficient line summation", Eq. (9)) is
// turned into a banded operand: for an output block of edge n and a line
// along i holding C^g column b, T_b[p][x] = C^g[x - p][b] for 0 <= x - p <= 2r
// (zero elsewhere), x indexing the n + 2r rows of the halo'd input.  These
// are exactly the zero-padded coefficient vectors of Eq. (10)-(11): column x
// of T_b is the vector that multiplies input row x.  Eq. (12) as printed pairs
// the C^o column j with the input segment starting at column j; reading Eq. (1)
// and Eq. (3)-(5) together, the segment shifted by j - r from the output must
// carry C^g column j (C^s column 2r - j), which is what is built here (the two
// agree for stencils symmetric in j, the case of the paper's examples).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "kernels_3d.hpp"

namespace stencil {

namespace {

int dtype_size(int dtype) { return dtype == STENCIL_F64 ? 8 : 4; }

bool on_axis(int ndim, int R, const int* idx) {
  int nz = 0;
  for (int d = 0; d < ndim; ++d)
    if (idx[d] != R) ++nz;
  return nz <= 1;
}

template <typename T>
void put(std::vector<uint8_t>& buf, size_t index, T v) {
  std::memcpy(buf.data() + index * sizeof(T), &v, sizeof(T));
}

// Round-to-nearest-even conversions to 16-bit formats, written out from the
// IEEE-754 encodings (binary32 -> bfloat16 / binary16).
uint16_t to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
float from_bf16_bits(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t to_f16_bits(float f) {
  _Float16 h = (_Float16)f;  // host conversion rounds to nearest even
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}
float from_f16_bits(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (float)h;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

double band_value(const double* cg2d, int R, int n, int axis, int index, int i, int j) {
  const int W = 2 * R + 1;
  if (axis == 0) {  // T_index[p = i][x = j]
    const int p = i, x = j, a = x - p;
    if (x < 0 || x >= n + 2 * R || p < 0 || p >= n || a < 0 || a > 2 * R) return 0.0;
    return cg2d[a * W + index];
  }
  // S_index[y = i][q = j]
  const int y = i, q = j, b = y - q;
  if (y < 0 || y >= n + 2 * R || q < 0 || q >= n || b < 0 || b > 2 * R) return 0.0;
  return cg2d[index * W + b];
}

int line_cover(const double* cg2d, int R, int* rows_out, int* cols_out) {
  // Maximum matching by augmenting paths (Kuhn), then König's construction:
  // Z = vertices reachable from unmatched rows by alternating paths; the
  // cover is (rows not in Z) + (columns in Z).
  const int W = 2 * R + 1;
  std::vector<int> match_col(W, -1), match_row(W, -1);
  auto edge = [&](int i, int j) { return cg2d[i * W + j] != 0.0; };
  for (int i = 0; i < W; ++i) {
    std::vector<char> seen(W, 0);
    std::vector<int> stack;
    // iterative DFS for an augmenting path from row i
    std::vector<int> parent_col(W, -1), via_row(W, -1);
    bool found = false;
    int end_col = -1;
    stack.push_back(i);
    while (!stack.empty() && !found) {
      const int u = stack.back();
      stack.pop_back();
      for (int j = 0; j < W && !found; ++j) {
        if (!edge(u, j) || seen[j]) continue;
        seen[j] = 1;
        via_row[j] = u;
        if (match_row[j] < 0) {
          found = true;
          end_col = j;
        } else {
          stack.push_back(match_row[j]);
        }
      }
    }
    if (found) {
      int j = end_col;
      while (j >= 0) {
        const int u = via_row[j];
        const int prev = match_col[u];
        match_col[u] = j;
        match_row[j] = u;
        j = (u == i) ? -1 : prev;
      }
    }
    (void)parent_col;
  }
  std::vector<char> zr(W, 0), zc(W, 0);
  std::vector<int> queue;
  for (int i = 0; i < W; ++i)
    if (match_col[i] < 0) {
      zr[i] = 1;
      queue.push_back(i);
    }
  while (!queue.empty()) {
    const int u = queue.back();
    queue.pop_back();
    for (int j = 0; j < W; ++j) {
      if (!edge(u, j) || zc[j] || match_col[u] == j) continue;
      zc[j] = 1;
      const int v = match_row[j];
      if (v >= 0 && !zr[v]) {
        zr[v] = 1;
        queue.push_back(v);
      }
    }
  }
  int count = 0;
  for (int i = 0; i < W; ++i) {
    rows_out[i] = zr[i] ? 0 : 1;
    cols_out[i] = zc[i] ? 1 : 0;
    count += rows_out[i] + cols_out[i];
  }
  return count;
}

static int validate(const stencil_desc_t* d) {
  if (!d || !d->coeffs) return STENCIL_EINVAL;
  if (d->ndim != 2 && d->ndim != 3) return STENCIL_EINVAL;
  if (d->radius < 1 || d->radius > 4) return STENCIL_EINVAL;
  if (d->shape != STENCIL_STAR && d->shape != STENCIL_BOX && d->shape != STENCIL_GENERAL) return STENCIL_EINVAL;
  if (d->boundary != STENCIL_BC_ZERO && d->boundary != STENCIL_BC_PERIODIC) return STENCIL_EINVAL;
  if (d->dtype != STENCIL_F32 && d->dtype != STENCIL_F64) return STENCIL_EINVAL;
  if (d->path < STENCIL_PATH_AUTO || d->path > STENCIL_PATH_MFMA_F16X3) return STENCIL_EINVAL;
  if (d->lines < STENCIL_LINES_AUTO || d->lines > STENCIL_LINES_HYBRID) return STENCIL_EINVAL;
  if (d->block_n != 0 && d->block_n != 4 && d->block_n != 16) return STENCIL_EINVAL;
  if (d->chunk < 0 || d->time_block < 0) return STENCIL_EINVAL;
  if (d->reg_rows != 0 && d->reg_rows != 8 && d->reg_rows != 16 && d->reg_rows != 32) return STENCIL_EINVAL;
  if (d->tile_width != 0 && d->tile_width != 128 && d->tile_width != 256) return STENCIL_EINVAL;
  if (d->time_block > 1) {
    // outer products: FP32 2D boxes on n = 4 blocks (library tiles), two
    // steps, column extent a multiple of 4
    const bool mfma_tb = d->path == STENCIL_PATH_MFMA && d->ndim == 2 && d->shape == STENCIL_BOX &&
                         d->dtype == STENCIL_F32 && d->time_block == 2 && d->dims[1] % 4 == 0 &&
                         d->block_n != 16 && (d->reg_rows == 0 || d->reg_rows == 16) &&
                         (d->tile_width == 0 || d->tile_width == 256);
    if (d->path != STENCIL_PATH_AUTO && d->path != STENCIL_PATH_GATHER && !mfma_tb) return STENCIL_EUNSUPPORTED;
    if (d->ndim == 3) {
      // 3D: two steps, direct-to-LDS lines; FP32 stars of order 1 and 2 and the
      // 27-point box, FP64 order 1
      if (d->shape == STENCIL_GENERAL || !tb3d_built(d->dtype, d->radius, d->shape == STENCIL_BOX) ||
          d->time_block > 2 || d->dims[2] % 4 != 0)
        return STENCIL_EUNSUPPORTED;
    } else if (d->time_block > tb2d_max_steps(d->dtype, d->radius)) {
      return STENCIL_EUNSUPPORTED;
    }
  }
  int64_t total = 1;
  for (int k = 0; k < d->ndim; ++k) {
    if (d->dims[k] < 1 || d->dims[k] > (int64_t(1) << 31) - 1) return STENCIL_EINVAL;
    total *= d->dims[k];
    if (total > (int64_t(1) << 40)) return STENCIL_EINVAL;
  }
  const int R = d->radius, W = 2 * R + 1;
  const int ncoef = d->ndim == 2 ? W * W : W * W * W;
  for (int t = 0; t < ncoef; ++t) {
    const double c = d->coeffs[t];
    if (!std::isfinite(c)) return STENCIL_EINVAL;
    if (d->shape == STENCIL_STAR && c != 0.0) {
      int idx[3] = {t / W % W, t % W, 0};
      if (d->ndim == 3) {
        idx[0] = t / (W * W);
        idx[1] = t / W % W;
        idx[2] = t % W;
      }
      if (!on_axis(d->ndim, R, idx)) return STENCIL_EINVAL;
    }
  }
  const bool split = d->path == STENCIL_PATH_MFMA_BF16X3 || d->path == STENCIL_PATH_MFMA_F16X3;
  if (split && d->dtype != STENCIL_F32) return STENCIL_EUNSUPPORTED;
  if (d->shape == STENCIL_GENERAL && d->lines != STENCIL_LINES_AUTO) return STENCIL_EUNSUPPORTED;
  if (d->shape == STENCIL_BOX && d->lines != STENCIL_LINES_AUTO && d->lines != STENCIL_LINES_PARALLEL)
    return STENCIL_EUNSUPPORTED;
  if (d->shape == STENCIL_STAR && d->ndim == 2 && d->lines == STENCIL_LINES_HYBRID)
    return STENCIL_EUNSUPPORTED;
  if (d->shape == STENCIL_STAR && d->ndim == 3 && d->lines == STENCIL_LINES_ORTHOGONAL)
    return STENCIL_EUNSUPPORTED;  // needs a second output block shape (Table 2); not built
  return STENCIL_OK;
}

// ------------------------------------------------------------------ packing
//
// A line is given by its 2r+1 weights w[d], d = 0..2r.  A line along the
// block's row axis ("column line", Eq. (9)-(12)) becomes the band
// T[p][x] = w[x - p]; a line along the column axis ("row line", Eq. (14))
// becomes S[y][q] = w[y - q]; x, y < n + 2r, zero elsewhere.
typedef std::vector<double> Line;

// FP32 / FP64 16x16x4 fragments.  Column lines are MFMA A operands (lane
// holds T[p = lane % 16][x = 4 cc + lane / 16]); row lines are B operands
// (lane holds S[y = 4 cc + lane / 16][q = lane % 16]).  Each line is padded to
// KL = round_up(n + 2r, 4) K rows (CPL chunks of 4).
static void pack_mfma(Resolved* rs, int R, int dtype, const std::vector<Line>& col,
                      const std::vector<Line>& row) {
  const int n = 16, K = n + 2 * R;
  const int KL = round_up(K, 4), CPL = KL / 4;
  const int NCH = (int)(col.size() + row.size()) * CPL;
  const int es = dtype_size(dtype);
  rs->frag.assign((size_t)NCH * 64 * es, 0);
  for (int c = 0; c < NCH; ++c) {
    const int li = c / CPL, cc = c % CPL;
    for (int lane = 0; lane < 64; ++lane) {
      const int a = lane % 16, k = 4 * cc + lane / 16;  // (p, x) or (q, y)
      const int d = k - a;
      const Line& w = li < (int)col.size() ? col[li] : row[li - col.size()];
      const double v = (k < K && d >= 0 && d <= 2 * R) ? w[d] : 0.0;
      if (es == 8)
        put<double>(rs->frag, (size_t)c * 64 + lane, v);
      else
        put<float>(rs->frag, (size_t)c * 64 + lane, (float)v);
    }
  }
  rs->info.k_rows = NCH * 4;
}

// FP32 fragments for n = 4 blocks on 4x4x1 (16 blocks): lane l of vector
// (line, d) holds T[p = l % 4][d] = w[d - p], d = 0 .. 3 + 2r.
static void pack_mfma_b4(Resolved* rs, int R, const std::vector<Line>& col) {
  const int NB = 4 + 2 * R;
  const int NF = (int)col.size() * NB;
  rs->frag.assign((size_t)NF * 64 * 4, 0);
  for (int li = 0; li < (int)col.size(); ++li)
    for (int dd = 0; dd < NB; ++dd)
      for (int lane = 0; lane < 64; ++lane) {
        const int e = dd - lane % 4;
        const double v = (e >= 0 && e <= 2 * R) ? col[li][e] : 0.0;
        put<float>(rs->frag, (size_t)(li * NB + dd) * 64 + lane, (float)v);
      }
  rs->info.k_rows = NF;
}

// Compact n = 4 fragments: vector li NB + dd holds only its four distinct
// values (block row j = lane mod 4) at 4 (li NB + dd) + j; kernels that build
// the packed lane order themselves (the 3D box table) read this form.
static void pack_mfma_b4_compact(Resolved* rs, int R, const std::vector<Line>& col) {
  const int NB = 4 + 2 * R;
  const int NF = (int)col.size() * NB;
  rs->frag.assign((size_t)NF * 4 * 4, 0);
  for (int li = 0; li < (int)col.size(); ++li)
    for (int dd = 0; dd < NB; ++dd)
      for (int j = 0; j < 4; ++j) {
        const int e = dd - j;
        const double v = (e >= 0 && e <= 2 * R) ? col[li][e] : 0.0;
        put<float>(rs->frag, (size_t)(li * NB + dd) * 4 + j, (float)v);
      }
  rs->info.k_rows = NF;
}

// 16-bit split fragments for row lines on 16x16x32 (B operand: lane l,
// element e holds S[y = 8 (l / 16) + e][q = l % 16]); hi and lo parts.  For
// FP16 the coefficients are scaled by 2^e (max weight in [2^14, 2^15)) and the
// lo parts by 2^11; out_scale / lo_scale undo both exactly.
static void pack_split(Resolved* rs, int R, int kind, const std::vector<Line>& row) {
  const int K = 16 + 2 * R;
  const int NL = (int)row.size();
  rs->frag.assign((size_t)NL * 2 * 64 * 8 * 2, 0);
  double cmax = 0.0;
  for (double c : rs->cg) cmax = std::fmax(cmax, std::fabs(c));
  float cscale = 1.0f, lscale = 1.0f;
  if (kind == 1) {
    int e = 0;
    if (cmax > 0.0) e = 14 - (int)std::floor(std::log2(cmax));
    cscale = std::ldexp(1.0f, e);
    lscale = std::ldexp(1.0f, 11);
  }
  for (int l = 0; l < NL; ++l) {
    for (int lane = 0; lane < 64; ++lane) {
      for (int e = 0; e < 8; ++e) {
        const int y = 8 * (lane / 16) + e, q = lane % 16, d = y - q;
        const float c = (float)((y < K && d >= 0 && d <= 2 * R) ? row[l][d] : 0.0) * cscale;
        uint16_t hi, lo;
        if (kind == 0) {
          hi = to_bf16_bits(c);
          lo = to_bf16_bits(c - from_bf16_bits(hi));
        } else {
          hi = to_f16_bits(c);
          lo = to_f16_bits((c - from_f16_bits(hi)) * lscale);
        }
        put<uint16_t>(rs->frag, ((size_t)(l * 2 + 0) * 64 + lane) * 8 + e, hi);
        put<uint16_t>(rs->frag, ((size_t)(l * 2 + 1) * 64 + lane) * 8 + e, lo);
      }
    }
  }
  rs->out_scale = 1.0f / cscale;
  rs->lo_scale = 1.0f / lscale;
  rs->info.k_rows = NL * 32;
}

// Weights of the line through C^g along one axis.  `fixed` gives the other
// indices (entry for `axis` ignored).
static Line line_of(const std::vector<double>& cg, int nd, int R, int axis, const int* fixed, bool drop_centre) {
  const int W = 2 * R + 1;
  Line w(W);
  for (int d = 0; d < W; ++d) {
    int idx[3] = {fixed[0], fixed[1], fixed[2]};
    idx[axis] = d;
    const size_t flat = nd == 2 ? (size_t)idx[0] * W + idx[1] : ((size_t)idx[0] * W + idx[1]) * W + idx[2];
    w[d] = cg[flat];
  }
  if (drop_centre) w[R] = 0.0;
  return w;
}

static void fill_2d_counts(Resolved* rs, int R, int variant, bool split) {
  stencil_plan_info_t& in = rs->info;
  const int n = 16, W = 2 * R + 1;
  if (split) {
    in.mfma_lines = W;
    in.valu_lines = 0;
    in.rank1_per_block = (int64_t)W * (2 * R + n);
    return;
  }
  in.mfma_lines = variant == VAR_BOX ? W : (variant == VAR_STAR_ORTHO ? 2 : 1);
  in.valu_lines = variant == VAR_STAR_PARALLEL ? 2 * R : 0;
  if (variant == VAR_BOX) in.rank1_per_block = (int64_t)W * (2 * R + n);  // Section 3.4
  else if (variant == VAR_STAR_PARALLEL) in.rank1_per_block = (2 * R + n) + (int64_t)2 * R * n;  // Table 1
  else in.rank1_per_block = 2 * (2 * R + n);                                                      // Table 1
}

// Lines covering the nonzero weights of a 2D C^g: a minimum axis-parallel
// cover (König).  For the n = 4 kernel (c4) a line along j costs about 1.5
// lines along i (one LDS read per MFMA instead of one per four), so the
// nonzero columns alone are taken when they are not dearer.  Returns the
// number of lines; rows / cols flag the chosen lines.
static int general_cover(const std::vector<double>& cg, int R, bool c4, int* rows, int* cols) {
  const int W = 2 * R + 1;
  int ncov = line_cover(cg.data(), R, rows, cols);
  if (!c4) return ncov;
  int nzc = 0, nr = 0, nc = 0, colnz[9] = {0};
  for (int b = 0; b < W; ++b) {
    for (int a0 = 0; a0 < W; ++a0) colnz[b] |= cg[(size_t)a0 * W + b] != 0.0;
    nzc += colnz[b];
    nr += rows[b];
    nc += cols[b];
  }
  if (nr > 0 && 2 * nzc <= 2 * nc + 3 * nr) {
    for (int b = 0; b < W; ++b) {
      rows[b] = 0;
      cols[b] = colnz[b];
    }
    ncov = nzc;
  }
  return ncov;
}

// Largest nonzero-tap count of a GENERAL 2D stencil on the nonzero-tap gather
// (measured on MI355X, 8192^2; FP32 / FP64, orders 1..4): beyond it the
// all-tap gather is as fast, so that kernel runs every tap instead.
static const int kSparseMax[2][5] = {{0, 3, 10, 27, 43}, {0, 5, 10, 27, 31}};

// Largest nonzero-tap count of a GENERAL 3D stencil on the nonzero-tap
// gather; beyond it the all-tap gather is as fast (measured on MI355X,
// 256^3; FP32 / FP64, orders 1..4).
static const int kSparse3DMax[2][5] = {{0, 5, 44, 128, 128}, {0, 3, 40, 128, 128}};

int resolve_plan(const stencil_desc_t* desc, Resolved* rs, bool pack) {
  const int st = validate(desc);
  if (st != STENCIL_OK) return st;
  const stencil_desc_t& d = *desc;
  const int R = d.radius, W = 2 * R + 1, nd = d.ndim;
  const int ncoef = nd == 2 ? W * W : W * W * W;
  rs->cg.resize(ncoef);
  for (int t = 0; t < ncoef; ++t)
    rs->cg[t] = d.dtype == STENCIL_F32 ? (double)(float)d.coeffs[t] : d.coeffs[t];
  const std::vector<double>& cg = rs->cg;

  stencil_plan_info_t& in = rs->info;
  std::memset(&in, 0, sizeof(in));
  in.ndim = nd;
  in.radius = R;
  in.shape = d.shape;
  in.boundary = d.boundary;
  in.dtype = d.dtype;
  // GENERAL (any C^g) runs on the box kernels, except for the 2D outer-product
  // form, which takes a minimum line cover (Section 3.5).
  const bool general = d.shape == STENCIL_GENERAL;
  const bool box = d.shape == STENCIL_BOX || general;
  in.taps = box ? (nd == 2 ? W * W : W * W * W) : 2 * R * nd + 1;
  if (general) {
    in.taps = 0;
    for (int t = 0; t < ncoef; ++t) in.taps += cg[t] != 0.0;
  }
  in.useful_flops_per_point = 2.0 * in.taps;
  in.bytes_per_point = 2 * dtype_size(d.dtype);
  const int n = 16;
  const int KL = round_up(16 + 2 * R, 4);

  int path = d.path;
  in.time_block = 1;
  if (d.time_block > 1 && path != STENCIL_PATH_MFMA) path = STENCIL_PATH_GATHER;
  int tb_auto = 0;  // steps per launch the library chose (AUTO), 0 if none
  if (path == STENCIL_PATH_AUTO) {
    // Measured on MI355X: outer products on MFMA where the arithmetic
    // outgrows the memory traffic -- FP32 boxes of radius >= 3 (2D and 3D)
    // and 2D GENERAL line covers -- and the gather kernel elsewhere (stars and
    // small boxes stay HBM-bound, where the gather kernel ties or wins; the
    // FP64 matrix rate equals the FP64 vector rate).  2D extents whose column
    // count is not a multiple of 4 (no direct-to-LDS windows): outer products.
    const bool f32 = d.dtype == STENCIL_F32;
    if (nd == 3) {
      // Stars of radius 4 stay on the gather kernel: FP32 ahead by 4 % at
      // 512^3 and 3 % at 256^3, level at 384^3; FP64 (its rotating ring holds
      // two waves per SIMD) ahead by 17 % at 256^3, level at 512^3, 3 % behind
      // the hybrid outer products at 384^3.
      // GENERAL with few nonzero taps: the nonzero-tap gather beats the box
      // outer products up to 88 (r = 3) / 128 (r = 4) taps (256^3 FP32)
      static const int kSparse3DAuto[5] = {0, 0, 0, 88, 128};
      const bool few = general && in.taps <= kSparse3DAuto[R];
      path = f32 && box && R >= 3 && !few ? STENCIL_PATH_MFMA : STENCIL_PATH_GATHER;
      // Time blocking, two steps per launch, on k extents that take
      // direct-to-LDS lines, when every knob is left open; measured on MI355X
      // (zero halo) against the one-step gather: the whole-window form on
      // small grids (order 1 at 64^3 and below: 1.14-1.6x; FP32 stars 1.2x
      // at 128^3), the FP32 streaming form on planes of many (j, k) tiles
      // (FP32 7-point star from 32 tiles: 1.3x at 256^3, 1.8x at 320^3,
      // 1.86x at 384^3, 1.68x at 512^3; order-2 star from 48: 1.27x at
      // 320^3, 1.40x at 384^3, 1.32x at 512^3, losing at 256^3; 27-point box
      // from 96: 1.07x at 512^3, level at 384^3.  FP64 7-point star from 32:
      // 1.30x / 2.1x / 2.2x / 1.61x at 256^3 / 320^3 / 384^3 / 512^3;
      // 27-point box from 64: 1.54x at 384^3, 1.10x at 512^3, losing at 256^3)
      const int64_t pts3 = d.dims[0] * d.dims[1] * d.dims[2];
      const int64_t tiles3 = ceil_div(d.dims[1], kTJ) * ceil_div(d.dims[2], kTK);
      const bool small3 = R == 1 && (pts3 <= (int64_t(1) << 18) || (f32 && !box && pts3 <= (int64_t(1) << 21)));
      const int64_t stream_tiles = f32 ? (!box ? (R == 1 ? 32 : R == 2 ? 48 : 0) : (R == 1 ? 96 : 0))
                                       : (R == 1 ? (box ? 64 : 32) : 0);
      const bool stream3 = stream_tiles > 0 && tiles3 >= stream_tiles;
      if ((small3 || stream3) && !general && d.dims[2] % 4 == 0 && d.time_block == 0 &&
          d.lines == STENCIL_LINES_AUTO && d.block_n == 0 && d.chunk == 0) {
        path = STENCIL_PATH_GATHER;
        tb_auto = 2;
      }
    } else {
      // grids at most 64 columns wide (the paper's smallest Table 3 shapes):
      // outer products for stars and the FP64 9-point box, measured ahead there
      const bool dma_cols = d.dims[1] % 4 == 0;
      bool heavy = f32 && (general || (box && R >= 3));
      const bool narrow = d.dims[1] <= 64 && (!box || (!f32 && R == 1));
      if (general && f32 && dma_cols && d.dims[1] > 64) {
        // GENERAL: the gather against the line cover.  Time per point fitted
        // on MI355X (order 4, 8192^2 FP32), in units of 1e-16 s: 12290 + 403 n
        // for the nonzero-tap gather over n taps, 12910 + 1530 L for L lines,
        // the line term scaled by the band length (2r + 4) / 12 for other
        // orders.  Past kSparseMax taps the plan runs the all-tap gather,
        // whose time per point equals the nonzero-tap kernel's at that count
        // (the limit is their measured crossover), so n is capped there.
        int rr[9] = {0}, cc[9] = {0};
        const int L = general_cover(cg, R, d.block_n != 16, rr, cc);
        const int n_eff = std::min(in.taps, kSparseMax[0][R]);
        if (12 * 403 * n_eff < 12 * 620 + 1530 * L * (4 + 2 * R)) heavy = false;
      }
      path = dma_cols && !heavy && !narrow ? STENCIL_PATH_GATHER : STENCIL_PATH_MFMA;
      // Time blocking: on grids that take direct-to-LDS windows, the
      // time-blocked gather with the step count measured fastest on MI355X
      // (512^2, 2048^2 and 8192^2, periodic) beats every one-step plan.  On
      // narrow grids too (10 steps, alone: 32^2, 48^2, 32 x 128 and 64^2 take
      // 24-60 us against 50-108 us for the best one-step plan; batches of 64^2
      // grids run 1.6-2.1x faster), except the FP32 box of order 4, which
      // keeps the outer products up to 64 columns (69 vs 73-76 us).  FP32: 8 / 4 / 4 / 3 steps per launch for stars of order 1..4,
      // 8 / 4 / 4 / 2 for boxes (ahead of the outer products by 2-4 % at
      // order 3 and 7-10 % at order 4 on 8192^2, by 1.1-1.4x on 2048^2).
      // FP64: stars 8 / 4 / 2 / 2, boxes 8 / 4 and none from order 3 (their
      // 49 / 81 weights take 98 / 162 vector registers there).  Only when
      // every kernel knob is left to the library.
      static const int kAutoTimeBlock[2][2][5] = {{{0, 8, 4, 4, 3}, {0, 8, 4, 4, 2}},   // F32 star, box
                                                  {{0, 8, 4, 2, 2}, {0, 8, 4, 0, 0}}};  // F64 star, box
      const bool tb_cols = d.dims[1] > 64 || !(f32 && box && R == 4);
      if (!general && dma_cols && tb_cols && d.time_block == 0 && d.lines == STENCIL_LINES_AUTO &&
          d.block_n == 0 && d.chunk == 0 && d.reg_rows == 0 && d.tile_width == 0) {
        const int t = kAutoTimeBlock[f32 ? 0 : 1][box ? 1 : 0][R];
        if (t > 1) {
          path = STENCIL_PATH_GATHER;
          tb_auto = t;
        }
      }
    }
  }
  const bool split = path == STENCIL_PATH_MFMA_BF16X3 || path == STENCIL_PATH_MFMA_F16X3;
  rs->split16 = path == STENCIL_PATH_MFMA_F16X3 ? 1 : 0;
  int lines = d.lines;
  if (box) {
    lines = STENCIL_LINES_PARALLEL;
  } else if (lines == STENCIL_LINES_AUTO) {
    if (nd == 2) lines = R == 1 ? STENCIL_LINES_PARALLEL : STENCIL_LINES_ORTHOGONAL;
    // 3D: the hybrid cover on FP32/FP64 MFMA; the split paths keep the line
    // along k alone on MFMA (measured on MI355X at 384^3 and 512^3: the hybrid
    // split kernel ties it at r = 4 and trails it by 6 % at r = 1, its extra
    // hi/lo products costing more than the vector FMAs they replace)
    else lines = split ? STENCIL_LINES_PARALLEL : STENCIL_LINES_HYBRID;
  }

  KArgs& a = rs->args;
  std::memset(&a, 0, sizeof(a));
  a.d0 = d.dims[0];
  a.d1 = d.dims[1];
  a.d2 = nd == 3 ? d.dims[2] : 1;
  a.periodic = d.boundary == STENCIL_BC_PERIODIC ? 1 : 0;
  a.out_scale = 1.0f;
  a.lo_scale = 1.0f;

  // Dense coefficients in the arithmetic dtype (gather kernels, vector lines).
  rs->coef.assign((size_t)ncoef * dtype_size(d.dtype), 0);
  for (int t = 0; t < ncoef; ++t) {
    if (d.dtype == STENCIL_F64) put<double>(rs->coef, t, cg[t]);
    else put<float>(rs->coef, t, (float)cg[t]);
  }

  if (nd == 2) {
    // Column strips of kTile2D columns, each walked in chunks of `chunk` rows
    // (a multiple of the 64-row block), sized for >= ~2048 workgroups.
    // Column strips walked in row chunks; the kernel picker fixes the strip
    // width and row block at launch (it depends on the buffers' alignment).
    // Bound the item count of the narrowest strips and smallest chunks.
    const int64_t strips = ceil_div(d.dims[1], 64);
    if (strips * ceil_div(d.dims[0], 16) > (int64_t(1) << 31) - 1) return STENCIL_EUNSUPPORTED;
    if (d.chunk > (int64_t(1) << 30)) return STENCIL_EINVAL;
    rs->chunk_req = d.chunk;
    in.tile_rows = kTile2D;
    in.tile_cols = kTile2D;
    if (path == STENCIL_PATH_GATHER && (d.time_block > 1 || tb_auto > 1)) {
      rs->family = FAM_TB2D;
      rs->pick = find_tb2d(d.dtype, R, box);
      rs->pick_batch = find_tb2d_batch(d.dtype, R, box);
      rs->time_block = d.time_block > 1 ? d.time_block : tb_auto;
      rs->tb_auto = tb_auto > 1;
      in.time_block = rs->time_block;
      in.tile_rows = d.dtype == STENCIL_F64 ? 32 : 64;
      in.tile_cols = 64;
      in.executed_flops_per_point = 2.0 * in.taps;
      lines = STENCIL_LINES_AUTO;
    } else if (path == STENCIL_PATH_GATHER) {
      rs->family = FAM_GATHER2D;
      // GENERAL: the nonzero-tap gather (Section 3.5: weights left to vector
      // units) up to kSparseMax taps, the all-tap gather beyond
      // (grids that cannot take direct-to-LDS windows run every tap anyway)
      const bool dma_shape = d.dims[1] % 4 == 0 && !(d.dtype == STENCIL_F32 && d.dims[1] <= kTile2D);
      const bool sparse = general && dma_shape && in.taps <= kSparseMax[d.dtype == STENCIL_F64 ? 1 : 0][R];
      rs->pick = sparse ? find_sparse2d(d.dtype, R) : find_gather2d(d.dtype, R, box);
      in.executed_flops_per_point = 2.0 * (sparse || !general ? in.taps : W * W);
      if (sparse) {  // table of the nonzero taps
        const size_t es = dtype_size(d.dtype);
        rs->frag.assign(kSparseWeightOffset + (size_t)kSparseTapMax * es, 0);
        int nt = 0;
        for (int t = 0; t < ncoef; ++t) {
          if (cg[t] == 0.0) continue;
          put<int32_t>(rs->frag, 1 + nt, (int32_t)((t / W) << 8 | (t % W)));
          if (d.dtype == STENCIL_F64) put<double>(rs->frag, kSparseWeightOffset / 8 + nt, cg[t]);
          else put<float>(rs->frag, kSparseWeightOffset / 4 + nt, (float)cg[t]);
          ++nt;
        }
        put<int32_t>(rs->frag, 0, nt);
      }
      lines = STENCIL_LINES_AUTO;
    } else if (path == STENCIL_PATH_MFMA) {
      rs->family = FAM_MFMA2D;
      // GENERAL: a cover of the nonzero weights by lines (Section 3.5); when it
      // is every column (no lines along j) the box kernel does the same work.
      int crow[9] = {0}, ccol[9] = {0}, ncov = 0;
      bool cover = false;
      if (general) {
        ncov = general_cover(cg, R, d.dtype == STENCIL_F32 && d.block_n != 16, crow, ccol);
        for (int b = 0; b < W; ++b) cover |= crow[b] != 0 || ccol[b] == 0;
        if (d.dtype != STENCIL_F32 || d.block_n == 16) cover = true;
      }
      rs->variant = cover ? VAR_COVER
                          : (box ? VAR_BOX : (lines == STENCIL_LINES_PARALLEL ? VAR_STAR_PARALLEL : VAR_STAR_ORTHO));
      if (general) lines = STENCIL_LINES_AUTO;
      // FP32 box / parallel star: n = 4 blocks on 4x4x1 by default (less band
      // padding); block_n = 16 selects the 16x16x4 kernel.
      const bool b4_ok = d.dtype == STENCIL_F32 && (rs->variant == VAR_BOX || rs->variant == VAR_STAR_PARALLEL);
      if (d.block_n == 4 && !b4_ok && !cover) return STENCIL_EUNSUPPORTED;
      const bool b4 = b4_ok && d.block_n != 16;
      // register / workgroup tile of the n = 4 box kernel (library choice: 16 rows, 256 columns)
      const bool tiles_set = (d.reg_rows != 0 && d.reg_rows != 16) || (d.tile_width != 0 && d.tile_width != 256);
      if (tiles_set && !(b4 && rs->variant == VAR_BOX)) return STENCIL_EUNSUPPORTED;
      const int ui = d.reg_rows ? d.reg_rows / 4 : 4, wr = d.tile_width == 128 ? 2 : 1;
      if (b4 && rs->variant == VAR_BOX) {
        in.reg_rows = 4 * ui;
        in.tile_width = 256 / wr;
      }
      rs->pick = b4 ? find_mfma2d_b4(R, box, rs->variant == VAR_BOX ? ui : 4, rs->variant == VAR_BOX ? wr : 1)
                    : find_mfma2d(d.dtype, R, rs->variant);  // cover: set below
      if (d.time_block > 1) {
        // two steps per launch (validated above: FP32 box, n = 4, library tiles)
        if (!(b4 && rs->variant == VAR_BOX && ui == 4 && wr == 1)) return STENCIL_EUNSUPPORTED;
        rs->pick = find_tbm2d(R);
        rs->time_block = 2;
        in.time_block = 2;
      }
      std::vector<Line> col, row;
      const int fixed_r[3] = {R, R, 0};
      if (rs->variant == VAR_COVER) {
        // Lines along i (C^g columns) first, then lines along j (C^g rows, with
        // the cover's columns zeroed so each weight is counted once), padded
        // with zero lines to 2r+1 fragment slots.
        const int* rows = crow;
        const int* cols = ccol;
        const bool c4 = d.dtype == STENCIL_F32 && d.block_n != 16;  // n = 4 blocks (+16x16 for the fallback)
        int64_t code = 0;
        int k = 0;
        for (int b = 0; b < W; ++b)
          if (cols[b]) {
            const int fx[3] = {0, b, 0};
            col.push_back(line_of(cg, 2, R, 0, fx, false));
            code |= (int64_t)b << (5 * k++);
          }
        for (int a0 = 0; a0 < W; ++a0)
          if (rows[a0]) {
            Line w(W);
            for (int y = 0; y < W; ++y) w[y] = cols[y] ? 0.0 : cg[(size_t)a0 * W + y];
            col.push_back(w);
            code |= (int64_t)(16 | a0) << (5 * k++);
          }
        while ((int)col.size() < W) col.push_back(Line(W, 0.0));
        a.lcode0 = (int32_t)(code & ((int64_t(1) << 30) - 1));
        a.lcode1 = (int32_t)((code >> 30) | ((int64_t)ncov << 27));
        if (d.block_n == 4 && !c4) return STENCIL_EUNSUPPORTED;
        if (c4) rs->pick = find_mfma2d_b4c(R);
        in.block_n = c4 ? 4 : n;
        if (pack) {
          std::vector<uint8_t> f4;
          if (c4) {
            pack_mfma_b4(rs, R, col);
            f4.swap(rs->frag);
          }
          pack_mfma(rs, R, d.dtype, col, row);
          if (c4) rs->frag.insert(rs->frag.begin(), f4.begin(), f4.end());
        }
        in.mfma_lines = ncov;
        in.valu_lines = 0;
        in.k_rows = ncov * (c4 ? 4 + 2 * R : KL);
        in.rank1_per_block = (int64_t)ncov * (2 * R + in.block_n);
        in.executed_flops_per_point = 2.0 * in.k_rows;
        lines = STENCIL_LINES_AUTO;
        col.clear();
      }
      for (int b = 0; b < W; ++b) {
        if (rs->variant == VAR_COVER) break;
        if (rs->variant != VAR_BOX && b != R) continue;
        const int fx[3] = {0, b, 0};
        col.push_back(line_of(cg, 2, R, 0, fx, false));  // C^g column b
      }
      if (rs->variant == VAR_STAR_ORTHO) row.push_back(line_of(cg, 2, R, 1, fixed_r, true));  // C^g row r
      if (rs->variant != VAR_COVER) fill_2d_counts(rs, R, rs->variant, false);
      if (rs->variant == VAR_COVER) {
        // packed above
      } else if (b4) {
        if (pack) pack_mfma_b4(rs, R, col);
        else in.k_rows = (int)col.size() * (4 + 2 * R);
        in.block_n = 4;
        in.rank1_per_block = rs->variant == VAR_BOX ? (int64_t)W * (2 * R + 4) : (2 * R + 4) + (int64_t)2 * R * 4;
      } else {
        if (pack) pack_mfma(rs, R, d.dtype, col, row);
        else in.k_rows = (int)(col.size() + row.size()) * KL;
        in.block_n = n;
      }
      in.executed_flops_per_point = 2.0 * in.k_rows + 2.0 * in.valu_lines;
    } else {
      // Split precision: lines along j (C^g rows), star as a box with zero weights.
      rs->family = FAM_SPLIT2D;
      rs->pick = find_split2d(rs->split16, R, 0);
      lines = STENCIL_LINES_PARALLEL;
      std::vector<Line> row;
      for (int r0 = 0; r0 < W; ++r0) {
        const int fx[3] = {r0, 0, 0};
        row.push_back(line_of(cg, 2, R, 1, fx, false));
      }
      fill_2d_counts(rs, R, 0, true);
      if (pack) pack_split(rs, R, rs->split16, row);
      else in.k_rows = W * 32;
      a.out_scale = rs->out_scale;
      a.lo_scale = rs->lo_scale;
      in.block_n = n;
      in.executed_flops_per_point = 3.0 * 2.0 * in.k_rows;
    }
  } else {
    // 3D: workgroup tile kTJ x kTK in (j, k), a chunk of planes along i.
    const int64_t t0 = ceil_div(d.dims[1], kTJ), t1 = ceil_div(d.dims[2], kTK);
    const int64_t tiles = t0 * t1;
    // about 2048 work items, each at least 4r planes deep (the 2r warm-up
    // planes of a chunk are re-read, from HBM when the previous chunk's
    // workgroup read them long before); fewer, deeper items where a sweep on
    // 512^3 measured them faster: FP64 stars and 27-point box (larger windows,
    // fewer workgroups per CU) and low-order FP32 stars on the gather kernel
    int64_t items = 2048;
    if (d.dtype == STENCIL_F64 && (!box || R == 1)) items = (!box && R == 4) ? 256 : 512;
    else if (d.dtype == STENCIL_F32 && !box && R <= 3 && path == STENCIL_PATH_GATHER) items = R == 1 ? 512 : 1024;
    int64_t chunk = d.dims[0] * tiles / items;
    // boxes of radius >= 2 spend most of their time in arithmetic, which the
    // 2r warm-up planes repeat: deeper chunks while ~1024 items remain
    // (measured on 512^3: +5-10 % at 64 planes)
    if (box && R >= 2) chunk = std::max(chunk, std::min<int64_t>(64, d.dims[0] * tiles / 1024));
    if (chunk < 4 * R) chunk = 4 * R;
    if (d.chunk > 0) chunk = d.chunk;
    rs->chunk_req = d.chunk;  // 0: the kernel's picker may re-cut to one wave of resident workgroups
    if (chunk > d.dims[0]) chunk = d.dims[0];
    const int64_t nch = ceil_div(d.dims[0], chunk);
    if (tiles * nch > (int64_t(1) << 31) - 1 || tiles > (int64_t(1) << 30)) return STENCIL_EUNSUPPORTED;
    a.tiles0 = (int32_t)t0;
    a.tiles1 = (int32_t)t1;
    a.chunk = (int32_t)chunk;
    a.nchunks = (int32_t)nch;
    in.tile_rows = kTJ;
    in.tile_cols = kTK;
    const int tb3 = d.time_block > 1 ? d.time_block : tb_auto;
    if (path == STENCIL_PATH_GATHER && tb3 > 1) {
      rs->family = FAM_TB3D;
      rs->pick = find_tb3d(d.dtype, R, box);
      rs->pick_batch = find_tb3d_batch(d.dtype, R, box);
      rs->time_block = tb3;
      rs->tb_auto = d.time_block <= 1;
      in.time_block = tb3;
      in.executed_flops_per_point = 2.0 * in.taps;
      lines = STENCIL_LINES_AUTO;
    } else if (path == STENCIL_PATH_GATHER) {
      rs->family = FAM_GATHER3D;
      // GENERAL: the nonzero-tap gather up to the tap count where the all-tap
      // gather catches up (measured on MI355X; FP32 / FP64, orders 1..4)
      const bool sparse = general && in.taps <= kSparse3DMax[d.dtype == STENCIL_F64 ? 1 : 0][R];
      rs->pick = sparse ? find_sparse3d(d.dtype, R) : find_gather3d(d.dtype, R, box);
      in.executed_flops_per_point = 2.0 * (sparse || !general ? in.taps : W * W * W);
      if (sparse) {  // taps grouped by coefficient plane
        const size_t es = dtype_size(d.dtype);
        rs->frag.assign(kSparse3DWeightOffset + (size_t)kSparse3DTapMax * es, 0);
        int nt = 0;
        for (int ap = 0; ap < W; ++ap) {
          put<int32_t>(rs->frag, 1 + ap, nt);
          for (int t = ap * W * W; t < (ap + 1) * W * W; ++t) {
            if (cg[t] == 0.0) continue;
            const int rem = t - ap * W * W;
            put<int32_t>(rs->frag, kSparse3DCodeIndex + nt, (int32_t)((rem / W) << 8 | (rem % W)));
            if (d.dtype == STENCIL_F64) put<double>(rs->frag, kSparse3DWeightOffset / 8 + nt, cg[t]);
            else put<float>(rs->frag, kSparse3DWeightOffset / 4 + nt, (float)cg[t]);
            ++nt;
          }
        }
        put<int32_t>(rs->frag, 1 + W, nt);
        put<int32_t>(rs->frag, 0, nt);
      }
      lines = STENCIL_LINES_AUTO;
    } else if (path == STENCIL_PATH_MFMA) {
      if (!box && lines != STENCIL_LINES_HYBRID) return STENCIL_EUNSUPPORTED;
      rs->family = box ? FAM_MFMA3D_BOX : FAM_MFMA3D_STAR;
      rs->pick = find_mfma3d(d.dtype, R, box);
      std::vector<Line> col, row;
      if (box) {
        for (int ap = 0; ap < W; ++ap)
          for (int c = 0; c < W; ++c) {
            const int fx[3] = {ap, 0, c};
            col.push_back(line_of(cg, 3, R, 1, fx, false));  // CLS(a, *, c)
          }
        in.mfma_lines = W * W;
        in.valu_lines = 0;
        in.rank1_per_block = (int64_t)W * W * (2 * R + n);
      } else {
        const int fx[3] = {R, 0, R};
        col.push_back(line_of(cg, 3, R, 1, fx, false));  // CLS(r, *, r), centre included
        const int fk[3] = {R, R, 0};
        row.push_back(line_of(cg, 3, R, 2, fk, true));   // CLS(r, r, *), centre excluded
        in.mfma_lines = 2;
        in.valu_lines = 2 * R;
        in.rank1_per_block = 2 * (2 * R + n) + (int64_t)2 * R * n;  // Table 2, hybrid
      }
      // FP32 stars and boxes: n = 4 blocks by default (block_n = 16: the
      // 16x16x4 kernel)
      const bool b4 = d.dtype == STENCIL_F32 && d.block_n != 16;
      if (d.block_n == 4 && !b4) return STENCIL_EUNSUPPORTED;
      if (b4) {
        rs->pick = find_mfma3d_b4(R, box);
        std::vector<Line> lines4(col);
        lines4.insert(lines4.end(), row.begin(), row.end());
        if (pack) {
          if (box && R >= 2) pack_mfma_b4_compact(rs, R, lines4);
          else pack_mfma_b4(rs, R, lines4);
        }
        in.k_rows = (int)lines4.size() * (4 + 2 * R);
        in.block_n = 4;
        in.rank1_per_block = box ? (int64_t)W * W * (2 * R + 4) : 2 * (2 * R + 4) + (int64_t)2 * R * 4;
      } else {
        if (pack) pack_mfma(rs, R, d.dtype, col, row);
        else in.k_rows = (int)(col.size() + row.size()) * KL;
        in.block_n = n;
      }
      in.executed_flops_per_point = 2.0 * in.k_rows + 2.0 * in.valu_lines;
    } else {
      if (!box && lines != STENCIL_LINES_PARALLEL && lines != STENCIL_LINES_HYBRID) return STENCIL_EUNSUPPORTED;
      const bool hybrid = !box && lines == STENCIL_LINES_HYBRID;
      rs->family = box ? FAM_SPLIT3D_BOX : FAM_SPLIT3D_STAR;
      rs->pick = find_split3d(rs->split16, R, box, hybrid);
      std::vector<Line> row;
      if (box) {
        for (int ap = 0; ap < W; ++ap)
          for (int b = 0; b < W; ++b) {
            const int fx[3] = {ap, b, 0};
            row.push_back(line_of(cg, 3, R, 2, fx, false));  // CLS(a, b, *)
          }
        in.mfma_lines = W * W;
        in.valu_lines = 0;
        in.rank1_per_block = (int64_t)W * W * (2 * R + n);
      } else if (hybrid) {
        const int fk[3] = {R, R, 0};
        row.push_back(line_of(cg, 3, R, 2, fk, false));  // CLS(r, r, *), centre included (B operand)
        const int fj[3] = {R, 0, R};
        row.push_back(line_of(cg, 3, R, 1, fj, true));   // CLS(r, *, r), centre excluded (A operand)
        in.mfma_lines = 2;
        in.valu_lines = 2 * R;
        in.rank1_per_block = 2 * (2 * R + n) + (int64_t)2 * R * n;  // Table 2, hybrid
      } else {
        const int fk[3] = {R, R, 0};
        row.push_back(line_of(cg, 3, R, 2, fk, false));  // CLS(r, r, *), centre included
        in.mfma_lines = 1;
        in.valu_lines = 4 * R;
        in.rank1_per_block = (2 * R + n) + (int64_t)4 * R * n;  // Table 2, parallel
      }
      if (pack) pack_split(rs, R, rs->split16, row);
      else in.k_rows = (int)row.size() * 32;
      a.out_scale = rs->out_scale;
      a.lo_scale = rs->lo_scale;
      in.block_n = n;
      in.executed_flops_per_point = 3.0 * 2.0 * in.k_rows + 2.0 * in.valu_lines;
    }
  }
  in.path = path;
  in.lines = lines;
  if (((d.reg_rows != 0 && d.reg_rows != 16) || (d.tile_width != 0 && d.tile_width != 256)) && in.reg_rows == 0)
    return STENCIL_EUNSUPPORTED;  // the tile knobs belong to the n = 4 2D box kernel
  if (pack) in.operand_bytes = 256 + (int64_t)round_up((int)rs->coef.size(), 256) + (int64_t)round_up((int)rs->frag.size(), 256);
  if (!rs->pick) return STENCIL_EUNSUPPORTED;
  if (d.block_n != 0 && path != STENCIL_PATH_GATHER && d.block_n != in.block_n) return STENCIL_EUNSUPPORTED;
  return STENCIL_OK;
}

}  // namespace stencil
