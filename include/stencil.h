/*
 * stencil.h -- C ABI of the MI355X (gfx950) outer-product stencil library.
 *
 * The library computes Jacobi time steps of 2D/3D star and box stencils of
 * order (radius) r.  The problem statement follows "Stencil Matrixization"
 * (arXiv 2310.16298):
 *   - two arrays A (time t) and B (time t+1) that swap roles every step
 *     (Section 2.2);
 *   - a (2r+1)^d gather coefficient tensor C^g (Section 3.2, Eq. (1)-(2)),
 *     B[x] = sum_o C^g[o + r] * A[x + o];
 *   - stencils classified by dimension, shape (star/box) and order
 *     (Section 1; star = box with the off-axis weights zero, Section 3.3);
 *   - C-style storage, rightmost index contiguous (Section 4.1 footnote).
 *
 * Two computation paths sit behind one plan:
 *   GATHER   -- the plain gather-form vector kernel of Eq. (1) (baseline);
 *   MFMA*    -- the scatter-mode outer-product form of Eq. (3)-(12): each
 *               coefficient line (Eq. (9)) becomes a banded operand tile, and
 *               the rank-1 updates of Eq. (12) are issued as matrix-core
 *               (MFMA) products band x input-tile into an output tile held in
 *               registers (Section 3.2-3.3, Section 4, Algorithm 1).
 *
 * Conventions for every entry point:
 *   - Every function returns a stencil_status_t; no C++ exception crosses
 *     the ABI.  Negative values are errors.
 *   - Grid buffers are device pointers owned by the caller: contiguous,
 *     unpadded, C order, dims slowest to fastest, element type = plan dtype.
 *   - Streams are hipStream_t handles passed as void*; NULL means the
 *     default (null) stream of the current device.
 *   - Entry points that take a stream only enqueue work on it: they do not
 *     synchronise and do not allocate device memory, so they can be captured
 *     into a HIP graph (see stencil_run_steps for its own graph cache).
 *     Kernel faults surface at the caller's next synchronisation.
 *   - A plan belongs to the device that was current when it was created and
 *     must be used with that device current.  A plan is immutable after
 *     creation; concurrent applies of one plan on different streams are safe
 *     as long as their buffers do not overlap.
 */
#ifndef PAPER_2310_16298_STENCIL_H
#define PAPER_2310_16298_STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STENCIL_OK = 0,
  STENCIL_EINVAL = -1,       /* bad argument: null pointer, ndim, radius, dims, star with off-axis weight, non-finite coefficient */
  STENCIL_EUNSUPPORTED = -2, /* valid request whose combination is not built (e.g. split precision on FP64 grids) */
  STENCIL_ENOMEM = -3,       /* device or host allocation failed */
  STENCIL_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
  STENCIL_EALIAS = -5,       /* input and output buffers are the same */
  STENCIL_EINTERNAL = -6,    /* unexpected internal error */
  STENCIL_ETOOBIG = -7       /* the plan's operands exceed the static scratch buffer of
                                stencil_run_steps_noalloc (STENCIL_NOALLOC_SCRATCH_BYTES) */
} stencil_status_t;

/* STAR: only on-axis weights may be nonzero (2rd+1 taps); BOX: any weights,
 * all (2r+1)^d taps computed; GENERAL: any weights, 2D outer-product plans
 * cover the nonzero weights with a minimum set of axis-parallel coefficient
 * lines (Section 3.5, see stencil_line_cover) -- at most 2r+1 lines of either
 * direction, a weight on a column line and a row line being carried by the
 * column line only (on FP32 n = 4 blocks, where a line along j costs about
 * 1.5 lines along i, the nonzero columns alone are used when they are not
 * dearer); the 2D GATHER path computes only the nonzero weights (a tap list
 * in the plan) when there are at most 3 / 10 / 27 / 43 of them (FP32, order
 * 1 / 2 / 3 / 4; FP64 5 / 10 / 27 / 31: where the all-tap gather catches up
 * on MI355X), every tap otherwise; the 3D GATHER path likewise up to 5 / 44 /
 * 128 / 128 nonzero taps (FP32; FP64 3 / 40 / 128 / 128); other paths treat
 * GENERAL as BOX.  The line option (lines) must be
 * AUTO for GENERAL. */
typedef enum { STENCIL_STAR = 0, STENCIL_BOX = 1, STENCIL_GENERAL = 2 } stencil_shape_t;

/* Boundary rule (the paper states none):
 *   ZERO     -- every grid point is updated; values outside the grid read as 0;
 *   PERIODIC -- indices wrap modulo each extent. */
typedef enum { STENCIL_BC_ZERO = 0, STENCIL_BC_PERIODIC = 1 } stencil_boundary_t;

/* Element type of the grids (and of the arithmetic for GATHER/MFMA). */
typedef enum { STENCIL_F32 = 0, STENCIL_F64 = 1 } stencil_dtype_t;

typedef enum {
  STENCIL_PATH_AUTO = 0,        /* library picks, from measurements on MI355X: MFMA for F32 boxes of
                                   order >= 3 (2D and 3D; 3D GENERAL stencils with at most 88 / 128
                                   nonzero taps at order 3 / 4 take GATHER), F64 3D stars of order
                                   4 and 2D GENERAL
                                   stencils (FP32 grids wider than 64 columns: the line cover or
                                   the nonzero-tap gather, whichever a cost fitted on MI355X
                                   prefers -- 12290 + 403 n per point for n nonzero taps (n capped
                                   at the nonzero-tap limit of the GENERAL gather, past which the
                                   all-tap gather runs at about that cost) against
                                   12910 + 1530 L (2r+4)/12 for L lines), GATHER otherwise; 2D
                                   grids whose column extent is not
                                   a multiple of 4, or at most 64 (stars, the F64 9-point box),
                                   take MFMA;
                                   stencil_plan_info reports the choice */
  STENCIL_PATH_GATHER = 1,      /* gather-form vector kernel, Eq. (1) */
  STENCIL_PATH_MFMA = 2,        /* outer-product form on MFMA in the grid dtype (FP32 or FP64) */
  STENCIL_PATH_MFMA_BF16X3 = 3, /* outer-product form, BF16 hi/lo split operands (3 products), FP32 accumulate; F32 grids
                                  (2D stars and boxes, 3D stars and boxes r = 1..4) */
  STENCIL_PATH_MFMA_F16X3 = 4   /* outer-product form, FP16 hi/lo split operands (3 products), FP32 accumulate; F32 grids */
} stencil_path_t;

/* Coefficient line cover for star stencils (Tables 1 and 2).
 *   PARALLEL   -- lines along one axis only (2D: CLS(*,j); 3D: CLS(i,*,k), i=r or k=r);
 *   ORTHOGONAL -- one line per axis through the centre (2D only here);
 *   HYBRID     -- 3D: CLS(i,*,r) for all i plus CLS(r,r,*).
 * Box stencils always use PARALLEL. */
typedef enum {
  STENCIL_LINES_AUTO = 0,
  STENCIL_LINES_PARALLEL = 1,
  STENCIL_LINES_ORTHOGONAL = 2,
  STENCIL_LINES_HYBRID = 3
} stencil_lines_t;

typedef struct {
  int32_t ndim;         /* 2 or 3 (1D stencils have no outer-product form, Section 3.1) */
  int32_t radius;       /* order r, 1..4 */
  int64_t dims[3];      /* extents, slowest to fastest; dims[2] ignored when ndim == 2 */
  int32_t shape;        /* stencil_shape_t */
  int32_t boundary;     /* stencil_boundary_t */
  int32_t dtype;        /* stencil_dtype_t */
  int32_t path;         /* stencil_path_t */
  int32_t lines;        /* stencil_lines_t */
  int32_t block_n;      /* edge n of the MFMA output block: 0 = library choice; 4 selects
                           v_mfma_f32_4x4x1_16b blocks (F32 only: 2D boxes, parallel-line and
                           GENERAL covers; 3D stars and boxes; the default there), 16 the 16x16
                           instructions (F64, 2D orthogonal stars, 3D boxes up to order 2); any
                           other resolved block edge: EUNSUPPORTED; ignored by the GATHER path */
  int32_t chunk;        /* output rows (2D) or i-planes (3D) per workgroup work item: 0 = library
                           choice (on the 3D GATHER path a grid that fits the LDS with its halo,
                           8^3 or 16^3 say, is then one work item computed whole by one
                           workgroup); rounded up to the kernel's row block and clipped to the
                           extent */
  int32_t time_block;   /* steps fused per launch (time blocking; the temporal reuse Section 6
                           leaves to future work): 1 = one step per launch; T > 1: each launch
                           advances T steps on overlapped tiles held in LDS (halo r*T), cutting HBM
                           traffic per point-step about T-fold.  Built for 2D grids on the GATHER
                           path (AUTO resolves to it), and T = 2 on the MFMA path for F32 BOX grids
                           whose column extent is a multiple of 4 with block_n, reg_rows and
                           tile_width left at 0 / 4 / 16 / 256 (n = 4 outer products at both levels;
                           its launches need 16-byte aligned buffers, else stencil_run_steps returns
                           EINVAL); on the GATHER path the halo r*T rounded up to a multiple of 4 is
                           at most 12 for F32 and 8 for F64 (r = 1: T <= 12 / 8; r = 2: 6 / 4;
                           r = 3: 4 / 2; r = 4: 3 / 2), and for 3D r = 1 STAR / BOX grids and
                           F32 STAR grids of r = 2..4 whose last extent is a multiple of 4
                           (T = 2; its launches need 16-byte
                           aligned buffers, else stencil_run_steps returns EINVAL); else
                           EUNSUPPORTED.  0 = library choice:
                           one step per launch, except that path AUTO on 2D STAR / BOX grids
                           whose column extent is a multiple of 4 (the F32 order-4 box: and
                           more than 64), with
                           lines, block_n, chunk, reg_rows and tile_width all 0, takes the
                           time-blocked gather with T measured fastest on MI355X (r = 1..4,
                           F32 stars 8 / 4 / 4 / 3, boxes 8 / 4 / 4 / 2; F64 stars 8 / 4 / 2 /
                           2, boxes 8 / 4 / - / -), and AUTO on 3D grids whose last extent is a
                           multiple of 4 takes T = 2 for r = 1 STAR / BOX grids of at most 64^3
                           points (F32 stars: 128^3) and for planes of many 32 x 64 (j, k) tiles:
                           at least 32 (r = 1 STARs), 48 (F32 r = 2 STAR), 64 (F64 r = 1 BOX) or
                           96 (F32 r = 1 BOX) (stencil_plan_info reports it).  stencil_apply is
                           always one step */
  int32_t reg_rows;     /* register tile of the 2D FP32 outer products on n = 4 blocks (box stencils,
                           MFMA path; the i unrolling of Section 4.2): output rows per wave, 8 / 16 / 32
                           (two, four or eight 4-row accumulator blocks), 0 = library choice (16) */
  int32_t tile_width;   /* workgroup tile of the same kernel: columns per strip, 256 (four waves side by
                           side) or 128 (two rows of two waves), 0 = library choice (256).  Non-default
                           reg_rows / tile_width on any other plan: EUNSUPPORTED; grids whose column
                           extent is not a multiple of 4 run the tiled kernel, which ignores both */
  const double* coeffs; /* host pointer to (2r+1)^ndim gather coefficients C^g,
                           C order, index o + r for offset o; copied by the call.
                           For an F32 plan they are rounded to float first. */
} stencil_desc_t;

typedef struct {
  int32_t path;          /* resolved stencil_path_t */
  int32_t lines;         /* resolved stencil_lines_t */
  int32_t ndim, radius, shape, boundary, dtype;
  int32_t taps;          /* nonzero-capable taps: (2r+1)^d box, 2rd+1 star (Section 3.4) */
  int32_t tile_rows;     /* output tile of one workgroup: rows (2D) or j-rows (3D) */
  int32_t tile_cols;     /* ... contiguous columns */
  int32_t block_n;       /* edge n of one MFMA output block (4 or 16); 0 for GATHER */
  int32_t mfma_lines;    /* coefficient lines issued on the matrix cores */
  int32_t valu_lines;    /* single-weight lines issued as vector FMAs */
  int32_t k_rows;        /* rank-1 updates per n x n block as issued, incl. MFMA K padding */
  int64_t rank1_per_block;       /* outer products per n x n block of the cover, Section 3.4 / Tables 1-2 */
  double useful_flops_per_point; /* 2 * taps */
  double executed_flops_per_point; /* flops the matrix+vector units execute per output point */
  int32_t bytes_per_point;       /* algorithmic HBM bytes per point-step: read + write of one element */
  int32_t time_block;            /* steps fused per launch (1 = none) */
  int32_t pad0;
  int64_t operand_bytes;         /* device bytes of the plan's operands: band fragments, dense C^g
                                    and a 256-byte zero line, each rounded up to 256 bytes */
  int32_t reg_rows;              /* output rows per wave of the n = 4 2D outer products (0: other kernels) */
  int32_t tile_width;            /* their workgroup tile width in columns (0: other kernels) */
} stencil_plan_info_t;

typedef struct stencil_plan_s* stencil_plan_t;

/* Version string of the library (static storage). */
const char* stencil_version(void);

/* Human-readable text for a status (static storage; never NULL). */
const char* stencil_status_string(stencil_status_t s);

/* Host-only: validate a descriptor without touching any device.
 * Returns STENCIL_OK, STENCIL_EINVAL or STENCIL_EUNSUPPORTED. */
stencil_status_t stencil_desc_check(const stencil_desc_t* desc);

/* Host-only: resolve the plan choices (path, line cover, tile, operation
 * counts) that stencil_plan would make, without touching any device. */
stencil_status_t stencil_plan_describe(const stencil_desc_t* desc, stencil_plan_info_t* info);

/* Host-only: the banded coefficient operand of one 2D coefficient line for an
 * output block of edge n (Section 3.2, Eq. (9)-(12); Section 3.3, Eq. (14)).
 *   axis 0 (a line along i, CLS(*, index) in the paper's naming, index = the
 *     C^g column; Eq. (9)): out is n x (n+2r), row-major;
 *     out[p*(n+2r) + x] = weight with which input row x of the block's
 *     halo'd input (row 0 = block row 0 minus r) reaches output row p;
 *     that is C^g[x-p][index] when 0 <= x-p <= 2r, else 0.  The input segment
 *     multiplied by it is shifted by index - r columns from the output.
 *   axis 1 (a line along j, CLS(index, *); Eq. (14)): out is (n+2r) x n;
 *     out[y*n + q] = C^g[index][y-q] when 0 <= y-q <= 2r, else 0: the weight
 *     with which input column y of the halo'd block reaches output column q,
 *     the input rows being shifted by index - r from the output.
 * coeffs: host (2r+1)x(2r+1) C^g, C order.  out: host, caller-allocated.
 * Returns STENCIL_EINVAL for null pointers, radius outside 1..4, n < 1 or
 * axis outside {0, 1}. */
stencil_status_t stencil_line_band(const double* coeffs, int32_t radius, int32_t n, int32_t axis,
                                   int32_t index, double* out);

/* Host-only: a minimum set of axis-parallel coefficient lines covering every
 * nonzero weight of a 2D C^g (Section 3.5).  The nonzeros are the edges of a
 * bipartite graph between row indices and column indices; a minimum vertex
 * cover (König's theorem: its size equals a maximum matching's) gives the
 * lines: row i in the cover is the line CLS(i, *) along j, column j the line
 * CLS(*, j) along i.
 * coeffs: host (2r+1)x(2r+1) C^g, C order.  rows_out, cols_out: host arrays of
 * 2r+1 int32, set to 1 for lines in the cover and 0 otherwise.  *count (may be
 * NULL) receives the number of lines.  Returns STENCIL_EINVAL for null
 * pointers or radius outside 1..4. */
stencil_status_t stencil_line_cover(const double* coeffs, int32_t radius, int32_t* rows_out, int32_t* cols_out,
                                    int32_t* count);

/* Create a plan on the current device: validates the descriptor, builds the
 * line cover and the banded operand fragments in MFMA lane order, and copies
 * them to the device (the only allocation the library makes).  The caller
 * may free desc->coeffs afterwards.  On error *out is set to NULL. */
stencil_status_t stencil_plan(const stencil_desc_t* desc, stencil_plan_t* out);

/* Report the resolved choices and operation counts of a plan. */
stencil_status_t stencil_plan_info(stencil_plan_t plan, stencil_plan_info_t* info);

/* Release a plan and its device memory.  NULL is accepted.  The caller must
 * ensure no enqueued work still uses the plan (e.g. synchronise first). */
stencil_status_t stencil_plan_destroy(stencil_plan_t plan);

/* One Jacobi step out = S(in) on `stream` (Section 2.2), also for a
 * time-blocked plan (one launch of one step).  in and out are
 * device buffers of the plan's dims and dtype and must not overlap
 * (in == out returns STENCIL_EALIAS). */
stencil_status_t stencil_apply(stencil_plan_t plan, const void* in, void* out, void* stream);

/* `steps` Jacobi steps with two buffers used alternately: step t reads
 * buf[t % 2] and writes buf[(t+1) % 2], starting from the state in buf0
 * (Section 2.2).  *result_index (may be NULL) receives the index of the
 * buffer holding the final state: steps % 2, or for a time-blocked plan
 * (stencil_plan_info's time_block T > 1, asked for or chosen by the library)
 * the parity of its launch count ceil(steps / T) -- each launch advances up
 * to T steps from one buffer into the other.  steps == 0
 * enqueues nothing.  Negative steps: EINVAL; overlapping buffers: EALIAS.
 * Launch mode: a run of at most 4 launches is enqueued kernel by kernel (a
 * graph replay costs more than that many direct launches).  Longer runs with
 * steps <= 4096, when `stream` is not being captured by the caller, are
 * recorded once into a HIP graph, cached in the plan per (buf0, buf1, steps)
 * (four entries, least recently used replaced), and replayed with one graph
 * launch; the first call for a key instantiates the graph (host-side work,
 * no device synchronisation).  While the caller is capturing `stream`, or
 * with the environment variable STENCIL_NO_GRAPH=1, the kernels are enqueued
 * one by one. */
stencil_status_t stencil_run_steps(stencil_plan_t plan, void* buf0, void* buf1, int64_t steps,
                                   void* stream, int32_t* result_index);

/* For callers that cannot allocate device memory -- tight serving loops,
 * harnesses that forbid hipMalloc -- the steps of stencil_run_steps without a
 * plan object: nothing is allocated on the device.  The descriptor is resolved
 * on the host as stencil_plan would (ordinary host memory only), its operands
 * (plan_info.operand_bytes: band fragments, dense C^g, the zero line) are
 * written into a static device array of STENCIL_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends (written by
 * small fill kernels that carry the bytes in their arguments: no host
 * staging, no memset), and the plan's kernels then run from it, one launch
 * per step (or per time block), eagerly on `stream`.
 * buf0 / buf1 / steps / result_index: as stencil_run_steps (the state starts
 * in buf0; *result_index receives the buffer of the final state).
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * operands: calls whose work overlaps in time on one GPU (other streams, or
 * the same stream from several threads) race and must be serialised by the
 * caller; calls in order on one stream are safe.
 * Errors: as stencil_desc_check (EINVAL / EUNSUPPORTED), EINVAL for null
 * buffers or negative steps, EALIAS for overlapping buffers, ETOOBIG when
 * operand_bytes exceeds STENCIL_NOALLOC_SCRATCH_BYTES (checked before any
 * device call), EUNSUPPORTED while `stream` is being captured (the upload is
 * not meant for graphs), EHIP for a failed device call. */
#define STENCIL_NOALLOC_SCRATCH_BYTES 32768
stencil_status_t stencil_run_steps_noalloc(const stencil_desc_t* desc, void* buf0, void* buf1, int64_t steps,
                                           void* stream, int32_t* result_index);

/* ---------------------------------------------------------------- batches
 * Many grids of uneven sizes (each with its own plan: dims, radius, shape,
 * coefficients, boundary) advanced by the same number of Jacobi steps with one
 * launch per kernel and step instead of one per grid: small grids (the
 * paper's 64^2..512^2 and 8^3..64^3 cases, Section 5) leave most of the GPU
 * idle one at a time.  Grids whose plans resolve to the same kernel form a
 * group; a group's launch is persistent -- at most (resident workgroups per
 * CU) x (CUs) workgroups loop over the (grid, tile) work items of all its
 * grids.  Grids whose plans the library time-blocked (stencil_plan_info's
 * time_block T > 1 with the descriptor's time_block 0) advance up to T steps
 * per launch, on kernels picked for a grid among many: 2D FP64 grids keep
 * tiles of full height (32 rows) however small, and 3D grids too small for
 * the streaming form (whose own plans take the whole-window form) run one
 * step per launch.  Grids sharing the T-step kernel form a class, whose run of
 * `steps` steps is the fewest launches of at most T steps (as even as
 * possible) whose count has the parity of `steps`, each launch size its own
 * group (one step: the plans' one-step kernel).  Plain groups (steps
 * launches each) and classes run concurrently on streams forked from the
 * caller's stream and joined back into it; multi-step runs are replayed from
 * a captured HIP graph.  Every grid ends in its buffer steps % 2, with the
 * result of its plan's stencil_run_steps bit for bit. */
typedef struct stencil_batch_s* stencil_batch_t;

/* Create a batch on the current device.  plans[i] (device = current device)
 * advances the grid held in buffers buf0[i] / buf1[i] (device pointers of
 * plans[i]'s dims and dtype).  Allocates the device work table (one
 * allocation) and count-1 streams at most.  The plans and buffers must outlive
 * the batch; the plans may be shared between batches.  Errors: EINVAL (null
 * pointers, count < 1, a plan of another device), EALIAS (any two of the
 * 2 x count buffers overlap), EUNSUPPORTED (more than 2^31-1 work items in
 * one group, or a plan whose descriptor asked for a time block > 1), ENOMEM,
 * EHIP.  A library-chosen time block whose buffers do not take the
 * time-blocked kernels (alignment) runs one step per launch.  On error *out
 * is NULL. */
stencil_status_t stencil_batch_create(const stencil_plan_t* plans, void* const* buf0, void* const* buf1,
                                      int32_t count, stencil_batch_t* out);

/* `steps` Jacobi steps of every grid of the batch, enqueued on `stream`: step
 * t reads buf[t % 2] and writes buf[(t+1) % 2] of each grid, starting from
 * buf0 (Section 2.2).  *result_index (may be NULL) receives steps % 2.  Calls
 * on one batch must not overlap in time (they share its buffers). */
stencil_status_t stencil_batch_run_steps(stencil_batch_t batch, int64_t steps, void* stream,
                                         int32_t* result_index);

/* Number of kernel groups (a time-blocked class counts one per launch size),
 * and total work items and persistent workgroups over all groups (any pointer
 * may be NULL). */
stencil_status_t stencil_batch_info(stencil_batch_t batch, int32_t* groups, int64_t* items, int64_t* blocks);

/* Release a batch (NULL accepted); enqueued work must have completed. */
stencil_status_t stencil_batch_destroy(stencil_batch_t batch);

/* ---------------------------------------------------------------- serving
 * A serving loop with continuous batching.  Requests -- a descriptor, an
 * input and an output grid buffer, a step count -- wait in a FIFO.  Each call
 * of stencil_server_tick
 *   1. admits requests from the head of the queue while their device
 *      footprint (two grids plus operand fragments, coefficients and a zero
 *      line, each rounded up to 256 bytes) fits the server's arena and, if
 *      max_active > 0, while fewer than max_active are resident;
 *   2. advances every resident request with persistent batched launches, k
 *      per kernel group (the kernels of stencil_batch_run_steps; requests
 *      admitted at different ticks advance together): k is chosen from an
 *      estimate of each group's cost per step (HBM bytes and executed flops
 *      of its plans) so that the costliest group does one step and cheaper
 *      groups up to 64 in about the same time; a request takes part in the
 *      first min(k, steps left) launches of its group;
 *   3. copies each request that has done its steps to its output buffer and
 *      releases its arena block.
 * The arena is one device allocation made at creation, with a first-fit
 * allocator; ticks make no device allocation or free (hipFree would
 * synchronise the device), except that the two work tables (pinned host and
 * device) grow when more requests are resident than ever before.  All work
 * runs on the server's own stream (stencil_server_stream), in order.  A
 * request's result equals the result of a plan of the same descriptor run
 * alone (same kernel, same arithmetic).  Not thread-safe: one thread drives a
 * server.  Time-blocked descriptors (time_block > 1) are rejected
 * (EUNSUPPORTED); a time block the library chose (time_block 0) is run one
 * step per launch, with the same arithmetic. */
typedef struct stencil_server_s* stencil_server_t;

typedef struct {
  int64_t arena_bytes;         /* device memory for resident requests (>= 256) */
  int32_t max_active;          /* 0 = limited by the arena only */
  int32_t max_inflight_ticks;  /* ticks enqueued ahead of the GPU before tick() waits; 0 = 4 */
} stencil_server_config_t;

typedef struct {
  int64_t tick;                /* ticks so far */
  int64_t arena_in_use;        /* bytes of the arena held by resident requests */
  int32_t active;              /* resident requests after this tick */
  int32_t queued;              /* waiting requests */
  int32_t groups;              /* kernel groups launched this tick */
  int32_t retired;             /* requests whose results were enqueued this tick */
} stencil_server_stats_t;

/* Create a server on the current device (allocates the arena, 64 pinned
 * staging buffers of 64 KiB and a stream).  Errors: EINVAL, ENOMEM, EHIP. */
stencil_status_t stencil_server_create(const stencil_server_config_t* config, stencil_server_t* out);

/* The server's stream (hipStream_t): work the caller enqueues on it before a
 * submit is ordered before that request's admission (e.g. writing its input). */
stencil_status_t stencil_server_stream(stencil_server_t server, void** stream);

/* Queue a request: `steps` Jacobi steps of the grid in `input` (device, the
 * descriptor's dims and dtype) written to `output` (device, same size, not
 * overlapping input).  The descriptor is resolved and its coefficients copied
 * now; input must stay valid and unchanged, and output valid, until
 * stencil_server_poll reports the request.  *id (may be NULL) receives its id
 * (1, 2, ... in submission order).  Errors: EINVAL (null arguments, negative
 * steps, anything stencil_desc_check rejects), EALIAS, EUNSUPPORTED
 * (time-blocked descriptor), ENOMEM (footprint larger than the arena). */
stencil_status_t stencil_server_submit(stencil_server_t server, const stencil_desc_t* desc, const void* input,
                                       void* output, int64_t steps, int64_t* id);

/* One tick (see above); stats (may be NULL) receives the server's counters.
 * Blocks only to keep at most max_inflight_ticks ticks in flight. */
stencil_status_t stencil_server_tick(stencil_server_t server, stencil_server_stats_t* stats);

/* Ids of requests whose results are complete in their output buffers, in
 * completion order; at most `capacity` (whole ticks at a time), *count
 * receives the number written.  Non-blocking. */
stencil_status_t stencil_server_poll(stencil_server_t server, int64_t* ids, int32_t capacity, int32_t* count);

/* Withdraw request `id` (a caller's time-out, a client gone).  A request
 * still queued leaves at once: the server never touched its buffers.  A
 * resident one gets no further launch and its output buffer is never
 * written; its arena block is free for later admissions (which are enqueued
 * behind the work already on the server's stream), and that already
 * enqueued work may still read its input until the server's stream passes
 * this point (synchronise stencil_server_stream before reusing the input).
 * A cancelled request is never reported by stencil_server_poll; the other
 * requests' results are unchanged.  Errors: EINVAL (null server, an id that
 * was never submitted, has finished -- its completion was enqueued -- or was
 * cancelled already). */
stencil_status_t stencil_server_cancel(stencil_server_t server, int64_t id);

/* Wait for the server's stream and release everything (NULL accepted);
 * requests not yet finished are dropped. */
stencil_status_t stencil_server_destroy(stencil_server_t server);

/* -------------------------------------------------------------- autotuner
 * Measures candidate plans of one descriptor on the current device and
 * returns the fastest (Section 5 compares line options and unrolling per
 * stencil and size; this search does the same on MI355X).  Candidates, in two
 * rounds:
 *   1. path x line cover x MFMA block edge, the chunk left to the library:
 *      paths GATHER and MFMA when desc->path is AUTO (plus BF16x3 / FP16x3 for
 *      F32 grids with STENCIL_TUNE_ALLOW_SPLIT: lower precision, see
 *      stencil_path_t), line covers PARALLEL / ORTHOGONAL / HYBRID for stars
 *      when desc->lines is AUTO, block edges 4 and 16 for MFMA when
 *      desc->block_n is 0 -- combinations stencil_desc_check rejects are
 *      skipped;
 *   2. when the winner is a 2D FP32 box on n = 4 MFMA blocks and reg_rows /
 *      tile_width are 0: register tiles of 8 / 16 / 32 rows per wave x
 *      workgroup tiles of 128 / 256 columns (the unrolling study of Section
 *      4.2, Fig. 4);
 *   3. path AUTO or GATHER, time_block 0: time blocks T = 2..12 (3D: T = 2)
 *      (those stencil_desc_check accepts) on the gather path;
 *   4. for the winner (unless time-blocked), chunk lengths 16..1024 rows (2D)
 *      or 8..128 planes (3D) when desc->chunk is 0.
 * Fields of desc other than 0 / AUTO are kept fixed.
 * Timing: two scratch grids of desc's size (allocated here, freed before
 * returning) on `stream`, which must not be under capture; per candidate one
 * warm-up run and the best of three timed runs of 24..64 steps (about 2e8
 * point-steps), each run from the same seeded state of values in [-1, 1)
 * (refilled before the run, outside the timed region: zero operands let the
 * matrix cores and vector ALUs hold a higher clock than real data does).
 * best: receives desc with the chosen path, lines, block_n, chunk,
 *   time_block, reg_rows and tile_width (coeffs pointer unchanged).  ms_per_step (may be NULL): the
 *   winner's time per step.
 * cache_path (may be NULL): a text file, one line per tuned request
 *   ("<key> -> path=.. lines=.. block_n=.. chunk=.. time_block=.. reg_rows=..
 *   tile_width=.. ms=.."),
 *   keyed by ndim,
 *   shape, radius, dtype, boundary, dims and the requested knobs (the
 *   coefficient values do not change the timing).  A hit returns the stored
 *   choice without measuring (unless STENCIL_TUNE_FORCE); a new result is
 *   appended.  An unreadable or unwritable file is treated as empty.
 * results / capacity / count (results may be NULL when capacity is 0): every
 *   measured candidate in order, at most `capacity` written; *count (may be
 *   NULL) receives the number measured (0 on a cache hit).
 * Errors: EINVAL (null desc/best, unknown flags, capacity < 0 or results NULL
 * with capacity > 0, and anything stencil_desc_check rejects), EUNSUPPORTED
 * (no candidate is built), ENOMEM, EHIP. */
#define STENCIL_TUNE_ALLOW_SPLIT 1
#define STENCIL_TUNE_FORCE 2

typedef struct {
  int32_t path, lines, block_n, chunk, time_block, reg_rows, tile_width;
  int32_t status;       /* stencil_status_t of the candidate */
  double ms_per_step;   /* best timed run; negative if the candidate failed */
} stencil_tune_result_t;

stencil_status_t stencil_autotune(const stencil_desc_t* desc, const char* cache_path, int32_t flags,
                                  stencil_desc_t* best, double* ms_per_step, void* stream,
                                  stencil_tune_result_t* results, int32_t capacity, int32_t* count);

/* Error norms of a state against a reference, for the drift check of
 * mixed-precision runs.  a: device array of n elements of a_dtype
 * (stencil_dtype_t); ref: device FP64 array of n elements.  out: device
 * array of 3 doubles, overwritten with
 *   out[0] = sum (a - ref)^2,  out[1] = sum ref^2,  out[2] = max |a - ref|
 * (out[2] is +infinity when an element of a or ref is NaN, as out[0] is NaN).
 * Enqueued on `stream`; the sums are accumulated with atomics, so their last
 * bits may vary between calls. */
stencil_status_t stencil_error_norms(const void* a, int32_t a_dtype, const double* ref, int64_t n,
                                     double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2310_16298_STENCIL_H */
