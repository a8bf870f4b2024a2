// Internal definitions shared by the libdvmat translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "dvmat.h"

namespace dvmat {

// Row padding of both CSR orientations (entries); rows start 16-byte aligned.
constexpr int kRowPad = 4;
// Device sub-buffer alignment inside caller workspaces.
constexpr size_t kAlign = 256;
// Workgroups of the SpMV launches are a multiple of the XCD count so that the
// hardware's round-robin workgroup -> XCD dispatch gives each XCD an equal
// share; each XCD then walks a contiguous range of row blocks.
constexpr int kNumXcd = 8;
constexpr int kWaveSize = 64;
constexpr int kSpmvThreads = 256;                 // 4 waves per workgroup
constexpr int kMaxSpmvWorkgroups = 8192;          // partial-sum slots in the objective workspace
constexpr int kMaxRhs = 8;
// Row blocks hold at most this many rows (the stream kernel stages them in LDS).
constexpr int kBlockRowsMax = 64;
// Plans per batched launch (their vector pointers travel as kernel arguments).
constexpr int kMaxBatch = 64;
// Sliced panels: lanes per row (a slice holds 64 / W rows).
inline bool slice_lanes_ok(int w) { return w == 4 || w == 8 || w == 16; }

// Launch shape of one SpMV orientation: block kernel (Kind below) and
// workgroup count.
struct KernelCfg {
    int kind;
    int workgroups;
};
KernelCfg initial_kernel_cfg();

// Block kernels: row, stream and pipe read the CSR layout, panel the panel layout.
enum Kind { KIND_ROW = 0, KIND_STREAM = 1, KIND_PIPE = 2, KIND_PANEL = 3 };

dvmat_status set_error(dvmat_status code, const char* fmt, ...);
dvmat_status check_hip(hipError_t e, const char* what);

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// One orientation (CSR or panels) inside the device workspace.
struct CsrDev {
    int64_t n_rows = 0;                // rows of the orientation (voxels or beamlets)
    int B = 1;                         // rows per block row
    int64_t nnz_pad = 0;
    int64_t n_blocks = 0;
    int64_t nonempty = 0;
    const int64_t* rowptr = nullptr;   // [n_block_rows + 1], in block entries
    const int32_t* col = nullptr;      // [block entries]
    const void* val = nullptr;         // [block entries * B] of value_bytes
    const int32_t* blocks = nullptr;   // [n_blocks + 1] first block row of each work unit
    const int32_t* perm = nullptr;     // [n_rows] row stored at each position, or nullptr (natural order)
    int perm_runs = 0;                 // every block row's rows are consecutive natural rows
    // panel layout (layout 1): col is unused, col16 holds panel-local columns
    int layout = 0;
    int64_t n_panels = 0;
    int64_t max_panel_cols = 0;
    const uint16_t* col16 = nullptr;   // [block entries] position in the panel's column list
    const int32_t* ulist = nullptr;    // concatenated sorted column lists of the panels
    const int64_t* panel_u = nullptr;  // [n_panels + 1] offsets into ulist
    const int32_t* panel_units = nullptr;  // [n_panels + 1] first work unit of each panel
    int64_t n_parts = 0;
    const int32_t* part_units = nullptr;   // [n_parts + 1] first work unit of each part
    const int32_t* part_panel = nullptr;   // [n_parts] panel of each part
    // sliced panels (layout 2): rowptr and blocks index slices, W lanes per row
    int slice_lanes = 0;
};

// Host staging of one orientation before bind.
struct CsrHost {
    int64_t n_rows = 0;
    int B = 1;
    int64_t n_brows = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<uint8_t> val;          // value_bytes per value, B values per block entry
    std::vector<int32_t> blocks;
    std::vector<int32_t> perm;         // empty: natural row order
    int perm_runs = 0;
    int64_t nonempty = 0;
    int layout = 0;
    std::vector<uint16_t> col16;
    std::vector<int32_t> ulist;
    std::vector<int64_t> panel_u;
    std::vector<int32_t> panel_units;
    std::vector<int32_t> part_units, part_panel;
    int64_t max_panel_cols = 0;
    int slice_lanes = 0;
    int slice_entries = 0;
};

}  // namespace dvmat

struct dvmat_ddc_s {
    int64_t n_vox = 0, n_bl = 0, nnz = 0;
    int32_t storage = DVMAT_F32;
    int32_t value_bytes = 4;
    bool bound = false;
    dvmat::CsrHost host_dose, host_price;
    std::vector<float> host_scale;     // per-beamlet scale (16-bit storage)
    dvmat::CsrDev dose, price;
    const float* scale = nullptr;      // device [n_bl] (16-bit storage)
    float* xs = nullptr;               // device [n_bl * kMaxRhs] scaled-x scratch (16-bit)
    size_t ws_bytes = 0;
    dvmat::KernelCfg dose_cfg{0, 2048}, price_cfg{0, 2048};
    dvmat_build_opts opts{};
    float dose_tuned_ms = 0.0f, price_tuned_ms = 0.0f;
    // workspace layout offsets
    size_t off_dose_rowptr = 0, off_dose_col = 0, off_dose_val = 0, off_dose_blocks = 0, off_dose_perm = 0;
    size_t off_price_rowptr = 0, off_price_col = 0, off_price_val = 0, off_price_blocks = 0, off_price_perm = 0;
    size_t off_dose_ulist = 0, off_dose_panel_u = 0, off_dose_panel_units = 0;
    size_t off_price_ulist = 0, off_price_panel_u = 0, off_price_panel_units = 0;
    size_t off_dose_part_units = 0, off_dose_part_panel = 0, off_price_part_units = 0, off_price_part_panel = 0;
    size_t off_scale = 0, off_xs = 0;
    int64_t dose_panel_cols_total = 0, price_panel_cols_total = 0;
};

struct dvmat_obj_s {
    int64_t n_vox = 0;
    int32_t n_struct = 0;
    const uint8_t* sid = nullptr;      // device [n_vox]
    float* table = nullptr;            // device [256][4] (T, w+, w-, 0)
    float* partial = nullptr;          // device [kMaxSpmvWorkgroups * kMaxRhs]
    double* partial_d = nullptr;       // device [kMaxSpmvWorkgroups]
};

// Launch helpers implemented in spmv.hip, used by other units.
namespace dvmat {
dvmat_status launch_expand_scale(const dvmat_ddc_s* d, const float* x, int nrhs, hipStream_t s);
}
