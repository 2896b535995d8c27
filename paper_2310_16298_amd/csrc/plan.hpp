// Host-side plan: descriptor validation, coefficient line cover, banded
// operand construction and MFMA fragment packing, kernel selection.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/stencil.h"
#include "device_common.hpp"
#include "launch.hpp"

namespace stencil {

// Kernel families.
enum Family {
  FAM_GATHER2D = 0,
  FAM_MFMA2D = 1,      // outer-product form, grid dtype (f32/f64)
  FAM_SPLIT2D = 2,     // outer-product form, bf16/f16 hi/lo split operands
  FAM_GATHER3D = 3,
  FAM_MFMA3D_STAR = 4, // hybrid cover, Algorithm 1 plane order
  FAM_MFMA3D_BOX = 5,
  FAM_SPLIT3D_STAR = 6,
  FAM_SPLIT3D_BOX = 7,
  FAM_TB2D = 8,        // time-blocked gather
  FAM_TB3D = 9         // time-blocked 3D gather (r = 1)
};

// Everything the plan resolves on the host.
struct Resolved {
  stencil_plan_info_t info{};
  int family = 0;
  int variant = 0;          // kernel-specific (line option)
  int split16 = 0;          // 0 = bf16, 1 = f16 (split families)
  std::vector<double> cg;   // C^g after rounding to the grid dtype
  std::vector<uint8_t> frag;  // packed operand fragments (bytes)
  std::vector<uint8_t> coef;  // dense C^g in the arithmetic dtype (bytes)
  float out_scale = 1.0f, lo_scale = 1.0f;
  KArgs args{};             // everything but in/out
  int32_t chunk_req = 0;    // requested rows (2D) per work item, 0 = library choice
  int32_t time_block = 1;   // steps per launch
  bool tb_auto = false;     // time_block chosen by the library (AUTO): batches may time-block such plans
  Picker pick = nullptr;
  // The kernel of a time-blocked launch when the grid is one of many in a
  // batched launch (nullptr: pick).  A grid's own pick is sized for the grid
  // alone, where a small grid leaves most CUs idle; among many grids the
  // chip is full, and forms that buy occupancy with redundant work lose.
  Picker pick_batch = nullptr;
};

// Validate + resolve + pack (no device calls).  Returns a stencil status.
int resolve_plan(const stencil_desc_t* desc, Resolved* out, bool pack);

// Banded operand of a 2D coefficient line (see stencil_line_band).
double band_value(const double* cg2d, int R, int n, int axis, int index, int i, int j);

// Minimum axis-parallel line cover of a 2D C^g (Section 3.5); returns its size.
int line_cover(const double* cg2d, int R, int* rows_out, int* cols_out);

// Kernel lookups, one per family (defined next to the kernels).
Picker find_gather2d(int dtype, int R, bool box);
// Nonzero-tap gather of GENERAL 2D stencils.  Its table in the fragment
// buffer: int32 tap count at byte 0, int32 codes (row << 8 | column) from
// byte 4, weights in the arithmetic dtype from byte kSparseWeightOffset.
constexpr int kSparseTapMax = 81, kSparseWeightOffset = 512;
Picker find_sparse2d(int dtype, int R);
// 3D: int32 tap count at index 0, the first tap of each coefficient plane
// a = 0 .. 2r at index 1 + a (index 2r + 2: the count), int32 codes
// (j row << 8 | k column) from index kSparse3DCodeIndex, taps ordered by a,
// weights from byte kSparse3DWeightOffset; at most kSparse3DTapMax taps.
constexpr int kSparse3DTapMax = 128, kSparse3DCodeIndex = 16, kSparse3DWeightOffset = 1024;
Picker find_sparse3d(int dtype, int R);
Picker find_mfma2d(int dtype, int R, int variant);
Picker find_mfma2d_b4(int R, bool box, int ui = 4, int wr = 1);  // ui 4-row blocks per wave, wr rows of waves
Picker find_mfma2d_b4_tiles(int R, int ui, int wr);  // the box kernel's other register / workgroup tiles
Picker find_mfma2d_b4c(int R);  // line cover, n = 4 (FP32)
// Bytes of the n = 4 cover fragments that precede the 16x16 ones.
inline size_t cover_b4_frag_bytes(int R) { return (size_t)(2 * R + 1) * (4 + 2 * R) * 64 * sizeof(float); }
Picker find_split2d(int kind, int R, int variant);
Picker find_gather3d(int dtype, int R, bool box);
Picker find_mfma3d(int dtype, int R, bool box);
Picker find_mfma3d_b4(int R, bool box);  // FP32 n = 4 blocks: stars, 27-point box
Picker find_split3d(int kind, int R, bool box, bool hybrid);  // hybrid: stars, lines along j and k on MFMA
Picker find_tb2d(int dtype, int R, bool box);
Picker find_tb2d_batch(int dtype, int R, bool box);  // among many grids: FP64 tiles of full height
Picker find_tb3d(int dtype, int R, bool box);  // two steps per launch
Picker find_tb3d_batch(int dtype, int R, bool box);  // among many grids: the streaming form or none
Picker find_tbm2d(int R);  // FP32 2D box outer products, two steps per launch
bool tb3d_built(int dtype, int R, bool box);    // F32: stars r <= 4, the 27-point box; F64: r = 1
int tb2d_max_steps(int dtype, int R);  // largest time_block of the time-blocked kernel

hipError_t launch_error_norms(const void* a, int a_dtype, const double* ref, int64_t n, double* out,
                              hipStream_t s);
// n values of dtype spread over [-1, 1), a fixed function of (seed, index)
hipError_t launch_trial_fill(void* p, int dtype, int64_t n, uint64_t seed, hipStream_t s);

}  // namespace stencil
