/*
 * dvmat.h -- C ABI of libdvmat: the dose-deposition-coefficient (DDC) products
 * of column-generation VMAT optimisation on one AMD Instinct MI355X (gfx950).
 *
 * Method: Tian et al., "Multi-GPU implementation of a VMAT treatment plan
 * optimization algorithm", arXiv:1503.01721.  Section 2.1 defines the model
 * (objective Eq. 1, price Eqs. 3-4, aperture DDC Eq. 5, master problem Eq. 6,
 * Barzilai-Borwein steps Eqs. 7-8 with the bound rules Eqs. 9-10); Section
 * 2.2.2 describes the GPU steps (price by CSR SpMV of D^T, row-wise aperture
 * selection, the four master-problem steps).
 *
 * Conventions for every call
 * --------------------------
 * - Return value: DVMAT_OK (0) or a negative dvmat_status; the message of the
 *   last failure on the calling thread is dvmat_last_error() (never NULL).
 *   Nothing throws, aborts or exits across this interface.
 * - O(1) argument checks run before anything is enqueued; O(nnz) index and
 *   finiteness checks run once, in dvmat_ddc_create.
 * - Pointers documented "device" are device memory owned by the caller; the
 *   library never allocates device memory.  Every handle that needs device
 *   state keeps it in a caller-provided workspace whose size is queried first.
 * - "stream" is a hipStream_t passed as void* (NULL = the null stream).  Hot
 *   calls only enqueue work on it and return; results are valid after the
 *   stream's work completes.  Calls that use one handle and overlap in time on
 *   different streams race on that handle's scratch; serialise them.
 * - Vectors with several right-hand sides (nrhs in 1..8) are row-major
 *   [n][nrhs]: element (i, k) at i*nrhs + k.
 * - Indices: voxel i in [0, n_vox), beamlet j in [0, n_bl); with a control-
 *   point geometry, beamlet j = (k*n_rows + r)*n_cols + c for control point k,
 *   MLC leaf row r and beamlet c along the row.
 */
#ifndef DVMAT_H
#define DVMAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dvmat_status;
#define DVMAT_OK        0
#define DVMAT_E_ARG    (-1)   /* bad argument: null pointer, size, dtype, non-finite value */
#define DVMAT_E_SHAPE  (-2)   /* inconsistent sizes (geometry, nrhs, workspace layout)     */
#define DVMAT_E_INDEX  (-3)   /* COO row/column index out of range                          */
#define DVMAT_E_NOMEM  (-4)   /* workspace smaller than the size query, or host alloc fail  */
#define DVMAT_E_HIP    (-5)   /* a HIP runtime call failed                                  */
#define DVMAT_E_STATE  (-6)   /* call out of order (unbound handle, occupied control point) */

/* storage type of the DDC values; accumulation is always FP32 */
#define DVMAT_F32   0
#define DVMAT_F16   1   /* IEEE half, value/s_j with s_j = max_i |D_ij| kept in FP32 */
#define DVMAT_BF16  2   /* bfloat16, same per-beamlet scale                           */

typedef void* dvmat_stream;

const char* dvmat_last_error(void);
/* library version, e.g. 0x000100 for 0.1.0 */
int32_t dvmat_version(void);

/* ------------------------------------------------------------------------
 * DDC matrix D (voxels x beamlets).
 *
 * The paper keeps D as COO on the host (Sec. 2.2.2) and D^T as CSR on the
 * GPU for the price product Pi = D^T g (Eq. 3).  Here both orientations live
 * in one GPU's memory: CSR of D ("dose matrix", rows = voxels) for z = D x,
 * and CSR of D^T ("price matrix", rows = beamlets) for p = D^T g.  Row
 * pointers are int64 (more than 2^31 non-zeros fit), column indices int32,
 * every (block) row is padded with explicit zeros to a multiple of 4 entries
 * so that rows start on 16-byte boundaries.
 * ---------------------------------------------------------------------- */
typedef struct dvmat_ddc_s* dvmat_ddc;

typedef struct {
    int64_t n_vox, n_bl, nnz;            /* nnz after summing duplicate pairs   */
    int64_t nnz_pad_dose, nnz_pad_price; /* stored entries incl. row padding     */
    int64_t n_blocks_dose, n_blocks_price; /* row blocks (work units)            */
    int64_t nonempty_rows_dose, nonempty_rows_price;
    int32_t storage;                     /* DVMAT_F32 / F16 / BF16               */
    int32_t value_bytes;                 /* 4 or 2                               */
    size_t workspace_bytes;              /* device bytes needed by dvmat_ddc_bind */
    int32_t dose_kernel, dose_workgroups;   /* launch shape in use: kernel 0 = row, 1 = stream, 2 = pipe */
    int32_t price_kernel, price_workgroups;
    float dose_tuned_ms, price_tuned_ms;    /* autotuner's best times (0 before tuning) */
    int32_t dose_block_rows, price_block_rows;  /* rows sharing one column index (build option) */
    int32_t dose_row_order, price_row_order;    /* row order of the layout (build option) */
    int32_t dose_layout, price_layout;          /* 0 = CSR, 1 = panels, 2 = sliced panels (as built) */
    int64_t dose_panels, price_panels;          /* panels (layouts 1 and 2), else 0         */
    int64_t dose_panel_cols, price_panel_cols;  /* largest column list of a panel           */
    int64_t dose_panel_cols_total, price_panel_cols_total; /* sum of the panels' column lists */
    int64_t dose_panel_parts, price_panel_parts;  /* workgroup tasks: runs of a panel's units */
    int32_t dose_slice_lanes, price_slice_lanes;  /* lanes per row of the sliced layout, else 0 */
} dvmat_ddc_info_t;

/* Build options of the device layout.  block_rows B in {1, 2, 4} (0: the
 * default for the layout and storage): B
 * consecutive rows form a block row that stores the union of their columns
 * once, with B values per column (zeros where a row lacks it), so one index
 * load and one gather of the input vector serve B rows.  Neighbouring voxels
 * see almost the same beamlets (the dose matrix gains most); neighbouring
 * beamlets overlap less.  Defaults depend on the storage type (below).
 * interleave (0/1, default 1): store the entries of each 256-entry chunk of a
 * block row interleaved so that each gather instruction of a wave covers
 * consecutive columns.  unit_entries: stored values per work unit (0: 2048
 * for CSR, 8192 when an orientation uses panels).
 * row_order: 0 = natural; 1 = rows stored in order of their first column
 * (empty rows last), so rows that read the same part of the input vector run
 * together (for the price matrix: beamlets covering the same slab of voxels,
 * from every angle); outputs are still written in natural order.
 *
 * layout: 0 = CSR, every product gathers the input vector from global memory;
 * 1 = panels: rows are grouped into panels, each with the sorted list of the
 * distinct columns its rows touch (at most panel_cols of them); the stored
 * column index is the position in that list (16 bits), and a product first
 * copies the panel's slice of the input vector into the compute unit's local
 * memory (LDS), then gathers from there.  Rows of neighbouring voxels (or of
 * neighbouring beamlets at neighbouring angles) touch few distinct columns, so
 * each staged value serves many products.  grid: the rows as a 3-D grid,
 * fastest axis first (voxels: nx, ny, nz; beamlets: columns, MLC rows,
 * control points), product equal to the row count; tile: the sub-grid of rows
 * that forms one panel (a tile with more distinct columns than panel_cols is
 * split along the row order).  A zero grid keeps the natural row order and
 * cuts panels greedily.  With block rows, tile[0] must be a multiple of B.
 * If a single block row has more than panel_cols distinct columns the
 * orientation is built as CSR (dvmat_ddc_info reports the layout built).
 * part_entries: a workgroup takes one part of a panel at a time, a run of
 * the panel's work units holding up to this many stored values (each part
 * stages the whole panel slice), so large panels are shared out.
 *
 * layout 2 = sliced panels: the panels of layout 1 (one row per block row),
 * each cut into parts of whole lines of rows (a line: the first extent of the
 * tile, or one row without a grid) holding up to part_entries stored values;
 * the rows of each part are sorted by length, longest first, and cut into
 * slices of 64 / W rows (W = dose_slice_lanes or price_slice_lanes); a wave
 * streams a slice with W lanes per row, all rows advancing together, 16
 * bytes of values per lane and step (4 entries at FP32, 8 at 16 bits), so
 * short rows pay neither a reduction over the whole wave nor a partial step
 * each.  Rows shorter than their slice's longest are padded
 * with zeros to its step count.  Rows without entries form slices of up to
 * 64 rows with no steps.  A slice is the work unit (n_blocks counts slices).
 * W in {4, 8, 16}; 0 chooses W from the orientation's mean non-empty row
 * length (the W whose slices take closest to 32 steps for such a row: more
 * lanes per row for longer rows); layout 2 needs block_rows 1 (0 resolves to
 * 1).  dvmat_ddc_info reports the lanes built. */
typedef struct {
    int32_t dose_block_rows;
    int32_t price_block_rows;
    int32_t interleave;
    int32_t unit_entries;
    int32_t dose_row_order;
    int32_t price_row_order;
    int32_t dose_layout, price_layout;
    int32_t dose_grid[3], price_grid[3];
    int32_t dose_tile[3], price_tile[3];
    int32_t panel_cols;
    int32_t part_entries;
    int32_t dose_slice_lanes, price_slice_lanes;
} dvmat_build_opts;

/* Fill opts with the defaults for a storage type (DVMAT_F32/F16/BF16): block
 * rows 0, which create resolves to the fastest measured for the layout (CSR:
 * dose B = 2 at 4-byte and 4 at 2-byte values, price B = 1 and 2; panels:
 * dose B = 1 and 2, price B = 1), price rows in first-column order, layout
 * CSR with zero grids (a caller that knows the voxel and beamlet grids sets
 * layout 1, the grids and tiles), panel_cols 12288, part_entries 131072.
 * Environment variables DVMAT_DOSE_B, DVMAT_PRICE_B, DVMAT_INTERLEAVE,
 * DVMAT_BLOCK_NNZ, DVMAT_DOSE_ORDER, DVMAT_PRICE_ORDER, DVMAT_PANEL_COLS and
 * DVMAT_PART_ENTRIES override single fields (DVMAT_SPMV_KIND and DVMAT_SPMV_WG
 * the launch shape a new handle starts with).  DVMAT_E_ARG for an unknown
 * storage. */
dvmat_status dvmat_ddc_default_opts(int32_t storage, dvmat_build_opts* opts);

/* Validate host COO (row = voxel, col = beamlet, val; length nnz; read during
 * the call only), sum duplicate pairs, build both CSR orientations, row blocks
 * and (F16/BF16) the quantised values with per-beamlet scales, staged in host
 * memory owned by the handle.  nnz may be 0.  Errors: DVMAT_E_ARG (null
 * pointer with nnz > 0, sizes < 1 or >= 2^31, unknown storage, non-finite
 * value), DVMAT_E_INDEX (index out of range), DVMAT_E_NOMEM (host memory). */
dvmat_status dvmat_ddc_create(int64_t n_vox, int64_t n_bl, int64_t nnz,
                              const int32_t* row_vox, const int32_t* col_bl,
                              const float* val, int32_t storage, dvmat_ddc* out);
/* As dvmat_ddc_create with explicit build options (NULL = defaults);
 * DVMAT_E_ARG for options out of range. */
dvmat_status dvmat_ddc_create_ex(int64_t n_vox, int64_t n_bl, int64_t nnz,
                                 const int32_t* row_vox, const int32_t* col_bl,
                                 const float* val, int32_t storage,
                                 const dvmat_build_opts* opts, dvmat_ddc* out);
/* Sizes and counts; valid right after create. */
dvmat_status dvmat_ddc_info(dvmat_ddc ddc, dvmat_ddc_info_t* info);

/* Copy one array of an orientation's device layout as built on the host
 * (between create and bind; DVMAT_E_STATE after bind), for inspection.
 * orientation 0 = dose, 1 = price; which: 0 = block-row pointers (int64),
 * 1 = column indices (int32 for CSR, uint16 panel-local for panels), 2 =
 * values (storage type, B per position), 3 = work units (int32 first block
 * rows), 4 = row at each stored position (int32; empty for natural order),
 * 5 = panel column lists (int32), 6 = panel offsets into them (int64), 7 =
 * first work unit of each panel (int32), 8 = first work unit of each part
 * (int32), 9 = panel of each part (int32).  Sliced panels (layout 2): 0 =
 * first entry of each slice (int64), 3 = first row position of each slice,
 * 7 and 8 count slices.  *size receives the array's byte size; dst (host, may
 * be NULL to query) must hold cap >= *size bytes. */
dvmat_status dvmat_ddc_layout_array(dvmat_ddc ddc, int32_t orientation, int32_t which, void* dst, size_t cap,
                                    size_t* size);
/* Copy the staged matrices into the caller's device workspace (>= info.
 * workspace_bytes, 256-byte aligned), synchronise the stream and release the
 * host staging.  Binding once is allowed; DVMAT_E_STATE on a second bind,
 * DVMAT_E_NOMEM if bytes is too small, DVMAT_E_ARG if misaligned. */
dvmat_status dvmat_ddc_bind(dvmat_ddc ddc, void* d_workspace, size_t bytes, dvmat_stream stream);
/* Frees host memory only (the workspace stays the caller's). NULL is a no-op. */
void dvmat_ddc_destroy(dvmat_ddc ddc);

/* ------------------------------------------------------------------------
 * Objective (Eq. 1): F(z) = sum_i w+_i max(0, z_i - T_i)^2 + w-_i max(0, T_i - z_i)^2
 * with per-voxel (T, w+, w-) looked up from a structure id, the small
 * replicated per-voxel parameters of Sec. 2.2.2.  w+ is the over-dose weight
 * (Eq. 1 and the sentence after it).
 * ---------------------------------------------------------------------- */
typedef struct dvmat_obj_s* dvmat_obj;

/* Device bytes needed by dvmat_obj_create for n_struct structures. */
dvmat_status dvmat_obj_workspace_size(int32_t n_struct, size_t* bytes);
/* d_struct_id: device uint8[n_vox], kept by reference (caller keeps it alive);
 * table: host float[n_struct][3] of (T, w+, w-), copied into the workspace.
 * n_struct in 1..256; ids >= n_struct read an all-zero row (no objective).
 * Enqueues the table copy on stream. */
dvmat_status dvmat_obj_create(int64_t n_vox, int32_t n_struct, const uint8_t* d_struct_id,
                              const float* table, void* d_workspace, size_t bytes,
                              dvmat_stream stream, dvmat_obj* out);
void dvmat_obj_destroy(dvmat_obj obj);

/* Standalone objective and gradient of an externally supplied dose.
 * z: device [n_vox][nrhs]; g: device [n_vox][nrhs] = dF/dz (nullable);
 * F: device float[nrhs] (nullable).  Eqs. (1) and (4) (g of Eq. 4 is -dF/dz). */
dvmat_status dvmat_objective(dvmat_obj obj, const float* z, int32_t nrhs, float* g, float* F,
                             dvmat_stream stream);

/* ------------------------------------------------------------------------
 * Hot products.
 * ---------------------------------------------------------------------- */

/* Dose z = D x: the dose update of the master problem (Sec. 2.2.2 step 4;
 * z = sum_k DA(A_k) y_k of Sec. 2.1 written per beamlet) and, for x the
 * indicator of an aperture, the aperture DDC vector DA of Eq. (5).
 * x: device [n_bl][nrhs]; z: device [n_vox][nrhs]; nrhs in 1..8.
 * With obj != NULL the objective epilogue also writes g = dF/dz (if g != NULL)
 * and F[nrhs] (if F != NULL), fused into the same pass over D. */
dvmat_status dvmat_dose(dvmat_ddc ddc, const float* x, int32_t nrhs, float* z,
                        dvmat_obj obj, float* g, float* F, dvmat_stream stream);

/* Price p = D^T g (Eq. 3 with g = dF/dz; the paper's price is pi = -p).
 * g: device [n_vox][nrhs]; p: device [n_bl][nrhs]; nrhs in 1..8. */
dvmat_status dvmat_price(dvmat_ddc ddc, const float* g, int32_t nrhs, float* p,
                         dvmat_stream stream);

/* Autotuner: times every candidate launch shape (block kernel "row",
 * "stream" or "pipe" x workgroup count) of the plain dose and of the price on the
 * caller's vectors (x: device float[n_bl], z: float[n_vox], g: float[n_vox],
 * p: float[n_bl], contents of z and p are overwritten), reps timed launches
 * each after one warm-up, and keeps the fastest per orientation for all later
 * calls on this handle.  Synchronises the stream.  Results are the same for
 * every shape (each shape's reductions have a fixed order). */
dvmat_status dvmat_ddc_autotune(dvmat_ddc ddc, const float* x, float* z, const float* g, float* p,
                                int32_t reps, dvmat_stream stream);
/* As dvmat_ddc_autotune, with the products timed as the column-generation
 * loop runs them: the dose with obj's objective epilogue (writing z, g = dF/dz
 * and F) and the price of that g, nrhs right-hand sides.  x: device
 * float[n_bl][nrhs]; z, g: float[n_vox][nrhs]; F: float[nrhs]; p:
 * float[n_bl][nrhs] (z, g, F, p are overwritten). */
dvmat_status dvmat_ddc_autotune_obj(dvmat_ddc ddc, dvmat_obj obj, const float* x, int32_t nrhs, float* z, float* g,
                                    float* F, float* p, int32_t reps, dvmat_stream stream);
/* Set the launch shape by hand: orientation 0 = dose, 1 = price; kind 0 =
 * row (one block row at a time), 1 = stream (a unit's entries as one range;
 * one row per block row only), 2 = pipe (row, with the next step's loads
 * issued before the current step's gathers, across block rows); workgroups
 * in [8, 8192] (rounded to a multiple of 8). */
dvmat_status dvmat_ddc_set_kernel(dvmat_ddc ddc, int32_t orientation, int32_t kind, int32_t workgroups);

/* Curvature of F along a fluence direction, for the first step length of a
 * master-problem solve: curv = sum_i w_i(z_ref) (D x_dir)_i^2 with w_i = w+
 * where z_ref_i > T_i, w- where z_ref_i < T_i, 0 where equal.  x_dir: device
 * float[n_bl]; z_ref: device float[n_vox]; d_out: device float[n_vox]
 * receives D x_dir (nullable); curv: device double[1]. */
dvmat_status dvmat_dose_curvature(dvmat_ddc ddc, const float* x_dir, dvmat_obj obj,
                                  const float* z_ref, float* d_out, double* curv,
                                  dvmat_stream stream);

/* ------------------------------------------------------------------------
 * Aperture selection (pricing problem, second step; Sec. 2.1 and 2.2.2
 * without the interdigitation constraint): per unoccupied control point and
 * MLC leaf row, the opening [L, R) with the smallest sum of p (the paper
 * maximises pi = -p); the aperture price is the sum over rows; the best
 * control point has the smallest price.  Openings are half-open beamlet
 * intervals, the closed row is (0, 0) with sum 0; ties: smaller sum, then
 * shorter, then smaller L; between control points the lower index.
 * ---------------------------------------------------------------------- */
typedef struct { int32_t n_cp, n_rows, n_cols; } dvmat_geom;

/* p: device float[n_cp*n_rows*n_cols]; occupied: device uint8[n_cp] (nonzero =
 * occupied, nullable = none); leaf_window: device int32[n_cp][n_rows][4]
 * (Lmin, Lmax, Rmin, Rmax; nullable = no limits): an opening [L, R) is
 * allowed iff Lmin <= L <= Lmax and Rmin <= R <= Rmax, a closed row parks at
 * the smallest position allowed to both leaves (Sec. 2.1: candidates must be
 * deliverable after the apertures at occupied neighbouring control points;
 * see dvmat_leaf_windows); a control point with a row that has no allowed
 * opening is infeasible (price +inf).  L, R: device int32[n_cp][n_rows]
 * (occupied and infeasible control points get 0, 0); cp_price: device
 * float[n_cp] (+inf if occupied or infeasible); best: device int32[1] = the
 * chosen control point, or -1 when no control point has a price < 0 (the
 * column generation stops, Sec. 2.1); best_price: device float[1] (the
 * smallest price, +inf if none is feasible).  Limits: n_cols <= 1024 and
 * n_rows*(n_cols+1) <= 16384 (one control point's prices are staged in
 * 64 KiB of LDS). */
dvmat_status dvmat_aperture_select(dvmat_geom geom, const float* p, const uint8_t* occupied,
                                   const int32_t* leaf_window, int32_t* L, int32_t* R, float* cp_price,
                                   int32_t* best, float* best_price, dvmat_stream stream);

/* Aperture selection under the interdigitation constraint of Sec. 2.2.2,
 * L_r <= min(R_{r-1}, R_{r+1}): adjacent rows need L_r <= R_{r+1} and
 * L_{r+1} <= R_r, so the rows are coupled; a closed row may park at any
 * position p (L = R = p, sum 0).  Exact minimum over all feasible apertures
 * by dynamic programming over the rows (state = one row's opening); ties go to
 * the smallest state index, states ordered by L then R.  Leaf windows and
 * outputs as dvmat_aperture_select.  n_cols <= 96 (the row DP works in LDS); d_workspace: device memory of
 * dvmat_aperture_select_ws_size bytes (per-row state values for backtracking). */
dvmat_status dvmat_aperture_select_ws_size(dvmat_geom geom, size_t* bytes);

/* Leaf windows from the apertures at occupied control points (Sec. 2.1):
 * occupied device uint8[n_cp]; L, R device int32[n_cp][n_rows], the openings
 * of the aperture at each occupied control point (other entries are not
 * read); travel: the largest leaf movement between adjacent control points,
 * in beamlets (a reading: the paper bounds it through gantry speed and leaf
 * speed, parameters given in references it cites; dvmat_machine_leaf_travel
 * derives it from a machine model).  Writes leaf_window
 * device int32[n_cp][n_rows][4]: for each row, each leaf within travel of
 * its position at the occupied neighbours k-1 and k+1, intersected with
 * [0, n_cols]. */
dvmat_status dvmat_leaf_windows(dvmat_geom geom, const uint8_t* occupied, const int32_t* L, const int32_t* R,
                                int32_t travel, int32_t* leaf_window, dvmat_stream stream);
dvmat_status dvmat_aperture_select_interdigitated(dvmat_geom geom, const float* p, const uint8_t* occupied,
                                                  const int32_t* leaf_window, int32_t* L, int32_t* R,
                                                  float* cp_price,
                                                  int32_t* best, float* best_price,
                                                  void* d_workspace, size_t bytes, dvmat_stream stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * selection as dvmat_aperture_select_interdigitated, same arguments and
 * results bit for bit, without the workspace.  The per-row state values live
 * in a library-owned static device array of 32 MiB (DVMAT_SELECT_SCRATCH_BYTES)
 * that each GPU the library runs on holds until the process ends; its device
 * address is looked up on the first call on each device (the device current
 * on the calling thread, which must be the stream's).  No call allocates.
 * DVMAT_E_NOMEM when dvmat_aperture_select_ws_size exceeds the array (e.g. the
 * 180 x 40 x 40 geometry needs 24.8 MB; 96 columns allow 1,764 rows in all);
 * DVMAT_E_SHAPE / DVMAT_E_ARG as the workspace form.  Every call on one GPU
 * shares the array, which keeps the last call's values: each call writes
 * every value it reads, but calls that overlap in time on one GPU (other
 * streams, other threads) race on it; serialise them. */
#define DVMAT_SELECT_SCRATCH_BYTES (32u << 20)
dvmat_status dvmat_aperture_select_interdigitated_noalloc(dvmat_geom geom, const float* p, const uint8_t* occupied,
                                                          const int32_t* leaf_window, int32_t* L, int32_t* R,
                                                          float* cp_price, int32_t* best, float* best_price,
                                                          dvmat_stream stream);

/* ------------------------------------------------------------------------
 * Machine constraints of Eq. (2) and the rate boxes they give the master
 * problem, Eq. (6): y_k in [R^L / S^U_k, R^U / S^L_k].  The paper takes the
 * parameter values from references it cites; here they are inputs.
 * Readings: s_k is the gantry speed on the arc from control point k to k+1,
 * so the leaf motion from A_k to A_{k+1} (d = the largest position change of
 * any leaf, in beamlet widths, closed rows' leaves where the selection placed
 * them) bounds s_k <= leaf_speed * gantry_step / d when both points hold
 * apertures (no bound for d = 0); S^U_k is the largest speed at k of any
 * profile within [S^L, S^U] that meets those bounds and |s_k - s_{k+1}| <=
 * speed_change along the whole arc; S^L_k = S^L.
 * ---------------------------------------------------------------------- */
typedef struct {
    float gantry_step;   /* angle between consecutive control points, > 0          */
    float speed_min;     /* S^L >= 0 (0: no upper rate bound)                      */
    float speed_max;     /* S^U > 0, >= S^L; may be +inf                            */
    float speed_change;  /* largest |s_k - s_{k+1}|, >= 0; may be +inf              */
    float rate_min;      /* R^L >= 0, finite                                        */
    float rate_max;      /* R^U >= R^L; may be +inf                                 */
    float leaf_speed;    /* leaf speed in beamlet widths per unit time, > 0; may be +inf */
} dvmat_machine;

/* Leaf travel for dvmat_leaf_windows (host, no GPU work): a candidate must be
 * reachable from the apertures at occupied neighbours even at the slowest
 * gantry speed, travel = floor(leaf_speed * gantry_step / speed_min) capped at
 * n_cols (n_cols when speed_min = 0 or leaf_speed = +inf).  With it every
 * S^U_k >= S^L and every box is non-empty.  DVMAT_E_ARG for a machine out of
 * range. */
dvmat_status dvmat_machine_leaf_travel(const dvmat_machine* m, int32_t n_cols, int32_t* travel);
/* S^U_k and the box of every control point.  m: host pointer (read during the
 * call); occupied device uint8[n_cp]; L, R device int32[n_cp][n_rows] (rows of
 * unoccupied points are not read); speed_hi, lo, hi: device float[n_cp]
 * (lo = rate_min / S^U_k, hi = rate_max / speed_min or +inf).  n_cp <= 8192;
 * one workgroup, O(n_cp^2) work.  DVMAT_E_ARG / DVMAT_E_SHAPE on bad input. */
dvmat_status dvmat_machine_boxes(dvmat_geom geom, const dvmat_machine* m, const uint8_t* occupied, const int32_t* L,
                                 const int32_t* R, float* speed_hi, float* lo, float* hi, dvmat_stream stream);

/* ------------------------------------------------------------------------
 * Master problem (Eq. 6) by Barzilai-Borwein steps (Eqs. 7-8, alternating)
 * with the subspace bound rules (Eqs. 9-10), state kept on the device.
 *
 * One solve: dvmat_bb_begin, optionally dvmat_bb_direction +
 * dvmat_dose_curvature for the first step length, then per iteration
 * dvmat_bb_step -> dvmat_dose (with objective) -> dvmat_price.
 * Readings (the paper is silent): step length at the first iteration of a
 * solve = <Gt,Gt>/(2 curv) (Cauchy step), later BB1 = <s,s>/<s,q> on odd and
 * BB2 = <s,q>/<q,q> on even iterations, used as step along -Gt (Eqs. 7-8 are
 * written with the negative gradient); if <s,q> <= 0 or the ratio is not
 * finite and positive the previous length is reused (flag FALLBACK).
 * Stopping: |F_{t-5} - F_t| <= eps_f |F_t|, max|y_t - y_{t-1}| <= eps_step
 * max(1, max|y_t|), all masked gradient components zero, or max_iter steps;
 * a threshold of 0 switches its test off.
 * Once stopped, further steps leave y unchanged (the caller may keep a fixed
 * number of steps).  Inner products are FP64, y and alpha FP32.
 * ---------------------------------------------------------------------- */
typedef struct dvmat_bb_s* dvmat_bb;

typedef struct {
    int32_t max_iter;    /* steps per solve (>= 1)             */
    float   eps_f;       /* relative F change over five steps  */
    float   eps_step;    /* step size relative to max(1,|y|)   */
} dvmat_bb_params;

#define DVMAT_BB_REL_F      1u
#define DVMAT_BB_SMALL_STEP 2u
#define DVMAT_BB_MAX_ITER   4u
#define DVMAT_BB_FALLBACK   8u
#define DVMAT_BB_CONVERGED 16u
#define DVMAT_BB_NONFINITE 32u

dvmat_status dvmat_bb_workspace_size(dvmat_geom geom, int32_t max_apertures, size_t* bytes);
/* Initialises an empty aperture set in the caller's device workspace. */
dvmat_status dvmat_bb_create(dvmat_geom geom, int32_t max_apertures, dvmat_bb_params params,
                             void* d_workspace, size_t bytes, dvmat_stream stream, dvmat_bb* out);
void dvmat_bb_destroy(dvmat_bb bb);
/* Host-side count of apertures (-1 for a NULL handle). */
int32_t dvmat_bb_count(dvmat_bb bb);
/* Device uint8[n_cp] inside the workspace, 1 where a control point holds an
 * aperture; maintained by dvmat_bb_add_aperture, suitable as the occupied
 * argument of dvmat_aperture_select (the "unoccupied control points" of Sec. 2.1). */
dvmat_status dvmat_bb_occupancy(dvmat_bb bb, const uint8_t** d_occupied);
/* Add the aperture chosen at control point cp (host value, e.g. read back
 * from dvmat_aperture_select's best): d_L, d_R device int32[n_rows] openings
 * (e.g. L + cp*n_rows), box [lo, hi] (hi may be +inf), initial rate
 * y0 (clamped to the box).  DVMAT_E_STATE if cp is occupied or the set is full. */
dvmat_status dvmat_bb_add_aperture(dvmat_bb bb, int32_t cp, const int32_t* d_L, const int32_t* d_R,
                                   float lo, float hi, float y0, dvmat_stream stream);
/* Replace the box of every aperture (the rate bounds of Eq. 6) by that of its
 * control point: lo_cp, hi_cp device float[n_cp] (e.g. from
 * dvmat_machine_boxes, which moves them as apertures are added); each rate is
 * clipped into its new box (into hi_cp where lo_cp > hi_cp).  Values are not
 * checked on the host: NaN boxes are the caller's error. */
dvmat_status dvmat_bb_set_boxes(dvmat_bb bb, const float* lo_cp, const float* hi_cp, dvmat_stream stream);
/* Start a master-problem solve (iteration counter, flags and F history reset). */
dvmat_status dvmat_bb_begin(dvmat_bb bb, dvmat_stream stream);
/* From the price p = D^T dF/dz at the current rates: the gradient in the
 * aperture domain G_k = sum_{j in A_k} p_j, masked by Eqs. (9)-(10), expanded
 * to beamlets: x_dir_j = Gt_k for j in A_k, else 0.  x_dir: device float[n_bl]. */
dvmat_status dvmat_bb_direction(dvmat_bb bb, const float* p, float* x_dir, dvmat_stream stream);
/* One iteration: p = D^T dF/dz and F at the current rates (device), curv from
 * dvmat_dose_curvature (device double[1], used on the first iteration of a
 * solve; NULL = fall back to max|y|/max|Gt|); writes the new beamlet fluence
 * x_next = B y (device float[n_bl]) and the solve's flags (device uint32[1],
 * nullable). */
dvmat_status dvmat_bb_step(dvmat_bb bb, const float* p, const float* F, const double* curv,
                           float* x_next, uint32_t* flags, dvmat_stream stream);
/* Device pointers into the workspace: the current rates y (float[count]) and
 * the masked gradient of the last dvmat_bb_direction/step (float[count]);
 * valid while the handle lives, contents change with each call. */
dvmat_status dvmat_bb_state(dvmat_bb bb, const float** y, const float** gt);
/* As dvmat_bb_direction and dvmat_bb_step, but with the gradient in the
 * aperture domain supplied by the caller: G device float[count] = dF/dy_k
 * (e.g. from automatic differentiation of F(D B y)); nothing is gathered.
 * x_next of dvmat_bb_step_g may be NULL: no beamlet fluence is written (the
 * DA form forms the dose from its aperture columns, not from x). */
dvmat_status dvmat_bb_direction_g(dvmat_bb bb, const float* G, float* x_dir, dvmat_stream stream);
dvmat_status dvmat_bb_step_g(dvmat_bb bb, const float* G, const float* F, const double* curv,
                             float* x_next, uint32_t* flags, dvmat_stream stream);
/* x = B y for the current rates (device float[n_bl]). */
dvmat_status dvmat_bb_expand(dvmat_bb bb, float* x, dvmat_stream stream);
/* Copy the current rates to device float[count]. */
dvmat_status dvmat_bb_get_y(dvmat_bb bb, float* y, dvmat_stream stream);

/* ------------------------------------------------------------------------
 * Batched products over many plans in one launch: the row blocks of every
 * plan form one work list that a single persistent grid walks, so plans of
 * very different sizes share the GPU without a launch per plan.  (The paper
 * suggests lending idle GPUs to another plan, Sec. 4; here the plans share
 * one GPU.)  All plans must be bound and share a storage type, the block
 * rows and, per orientation, the layout (and, for sliced panels, the lanes
 * per row: build such plans with explicit lanes, since lanes left at 0 follow
 * each plan's row lengths); n <= 64.  With panels the work list
 * is the plans' panel parts, each staging its panel's slice of the input
 * vectors in LDS (a sliced plan's slices run as in the single-plan product);
 * right-hand sides beyond what LDS holds go in chunks, one launch each (plans
 * built with panel_cols <= 3584 take 4 right-hand sides per launch).
 * ---------------------------------------------------------------------- */
typedef struct dvmat_batch_s* dvmat_batch;

dvmat_status dvmat_batch_workspace_size(int32_t n, size_t* bytes);
/* Records the plans' device layouts in the workspace (the ddc handles and
 * their workspaces must outlive the batch).  Synchronises the stream. */
dvmat_status dvmat_batch_create(const dvmat_ddc* ddcs, int32_t n, void* d_workspace, size_t bytes,
                                dvmat_stream stream, dvmat_batch* out);
void dvmat_batch_destroy(dvmat_batch batch);
/* z_i = D_i x_i for every plan i in one launch.  xs, zs: host arrays of n
 * device pointers ([n_bl_i][nrhs] and [n_vox_i][nrhs]); nrhs in {1,2,4,8}.
 * The pointers are passed by value as kernel arguments, so a captured graph
 * replays with the same buffers. */
dvmat_status dvmat_batch_dose(dvmat_batch batch, const float* const* xs, int32_t nrhs, float* const* zs,
                              dvmat_stream stream);
/* p_i = D_i^T g_i for every plan i in one launch (layout as above). */
dvmat_status dvmat_batch_price(dvmat_batch batch, const float* const* gs, int32_t nrhs, float* const* ps,
                               dvmat_stream stream);
/* Autotuner of the two batched launches (as dvmat_ddc_autotune; overwrites zs, ps). */
dvmat_status dvmat_batch_autotune(dvmat_batch batch, const float* const* xs, float* const* zs,
                                  const float* const* gs, float* const* ps, int32_t nrhs, int32_t reps,
                                  dvmat_stream stream);
/* Launch shape by hand (as dvmat_ddc_set_kernel). */
dvmat_status dvmat_batch_set_kernel(dvmat_batch batch, int32_t orientation, int32_t kind, int32_t workgroups);
/* Total work units (CSR) or panel parts of the dose and price work lists; cfg (nullable) receives
 * {dose kernel, dose workgroups, price kernel, price workgroups}. */
dvmat_status dvmat_batch_info(dvmat_batch batch, int64_t* dose_blocks, int64_t* price_blocks, int32_t* cfg);

/* ------------------------------------------------------------------------
 * Aperture maps for an explicit aperture list (no BB state): the fluence of
 * the chosen apertures, x_j = y_k for beamlet j in aperture A_k (z = D x is
 * then sum_k DA(A_k) y_k, Sec. 2.1 with Eq. 5), and its adjoint, the gradient
 * in the aperture domain G_k = sum_{j in A_k} p_j (step 1 of the master
 * problem, Sec. 2.2.2).  cps: device int32[m] distinct control points;
 * L, R: device int32[m][n_rows] openings [L, R); y, G: device float[m];
 * x, p: device float[n_cp*n_rows*n_cols].  expand writes every beamlet (0
 * outside the apertures).
 * ---------------------------------------------------------------------- */
dvmat_status dvmat_aperture_expand(dvmat_geom geom, int32_t m, const int32_t* cps, const int32_t* L,
                                   const int32_t* R, const float* y, float* x, dvmat_stream stream);
dvmat_status dvmat_aperture_gather(dvmat_geom geom, int32_t m, const int32_t* cps, const int32_t* L,
                                   const int32_t* R, const float* p, float* G, dvmat_stream stream);

/* ------------------------------------------------------------------------
 * DA-form master problem (Eq. 6 as written in the paper): the dose vector of
 * each chosen aperture, DA(A_k) = sum_{j in A_k} D_:j (Eq. 5), is formed once
 * on the device as a dense column; z = sum_k DA_k y_k and the gradient in the
 * aperture domain G_k = <DA_k, dF/dz> then need only the m columns, not the
 * whole matrix (Sec. 2.2.2 forms DA on the CPU; here one dose product of the
 * aperture's indicator fluence does it on the GPU).
 * ---------------------------------------------------------------------- */
typedef struct dvmat_da_s* dvmat_da;

dvmat_status dvmat_da_workspace_size(int64_t n_vox, int32_t max_apertures, size_t* bytes);
dvmat_status dvmat_da_create(int64_t n_vox, int32_t max_apertures, void* d_workspace, size_t bytes,
                             dvmat_da* out);
void dvmat_da_destroy(dvmat_da da);
int32_t dvmat_da_count(dvmat_da da);
/* Keep only the rows of the objective's support in the columns: the voxels
 * whose structure has a non-zero weight (w+ or w-), the only ones F and
 * G = dF/dy depend on (dF/dz is zero elsewhere).  Call before the first
 * dvmat_da_append (DVMAT_E_STATE after); obj must have n_vox voxels.  Once
 * restricted, dvmat_da_eval writes z and dF/dz only at support voxels, leaving
 * the caller's other entries unchanged (dF/dz is zero there; the dose there is
 * not formed), and dvmat_da_column returns columns of *n_rows entries in the
 * support's voxel order.  *n_rows (nullable) receives the support's size
 * (n_vox if no voxel is weighted: nothing is restricted).  Set-up work: one
 * workgroup scans the voxels, then the call synchronises the stream. */
dvmat_status dvmat_da_set_support(dvmat_da da, dvmat_obj obj, int64_t* n_rows, dvmat_stream stream);
/* Append DA = D x_ind for the next aperture: x_ind device float[n_bl], the
 * aperture's indicator fluence (e.g. dvmat_aperture_expand with rate 1).
 * DVMAT_E_STATE when max_apertures columns exist. */
dvmat_status dvmat_da_append(dvmat_da da, dvmat_ddc ddc, const float* x_ind, dvmat_stream stream);
/* y: device float[count]; z, g (nullable): device float[n_vox] receive the dose
 * and dF/dz; G: device float[count] = dF/dy; F (nullable): device float[1]. */
dvmat_status dvmat_da_eval(dvmat_da da, dvmat_obj obj, const float* y, float* z, float* g, float* G,
                           float* F, dvmat_stream stream);
/* One Barzilai-Borwein iteration of the DA-form master problem in one launch
 * (the four steps of Sec. 2.2.2 on the aperture columns; Eqs. 7-10): G = dF/dy
 * and F at the current rates of bb (as dvmat_da_eval, without z and dF/dz),
 * then the step of dvmat_bb_step_g(bb, G, F, curv, NULL, flags), taken by the
 * launch's last workgroup.  The result equals those two calls bit for bit.
 * bb holds the apertures of the da columns, in the same order (DVMAT_E_STATE
 * if the counts differ).  G: device float[>= count] and F: device float[1]
 * receive the values at the rates before the step; curv, flags as
 * dvmat_bb_step_g.  Calls on one da handle must not overlap in time. */
dvmat_status dvmat_da_bb_step(dvmat_da da, dvmat_bb bb, dvmat_obj obj, float* G, float* F, const double* curv,
                              uint32_t* flags, dvmat_stream stream);
/* curv = sum_i w_i(z_ref) (sum_k DA_k dir_k)_i^2 (weights as dvmat_dose_curvature);
 * dir: device float[count]; curv: device double[1]. */
dvmat_status dvmat_da_curvature(dvmat_da da, dvmat_obj obj, const float* dir, const float* z_ref,
                                double* curv, dvmat_stream stream);
/* Device pointer of column k (float[n_vox], or float[n_rows] of the support). */
dvmat_status dvmat_da_column(dvmat_da da, int32_t k, const float** col);

#ifdef __cplusplus
}
#endif
#endif /* DVMAT_H */
