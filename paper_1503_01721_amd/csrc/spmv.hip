// Dose z = D x and price p = D^T g on gfx950, the objective epilogue, the
// batched multi-plan launch and the kernel autotuner.
//
// Both products are CSR row-times-vector kernels over the orientation that
// makes the output a row: CSR(D) for the dose (rows = voxels, the dose update
// of the master problem, Sec. 2.2.2, and Eq. 5 for aperture indicators) and
// CSR(D^T) for the price (rows = beamlets, Eq. 3; the paper assigns one warp
// per beamlet row, Sec. 2.2.2).  The path is HBM-bound (2 flop per 8 bytes of
// matrix at FP32), so no matrix cores are used.
//
// Work units: rows are grouped on the host into blocks of consecutive rows
// with a bounded number of stored entries (and at most kBlockRowsMax rows).
// One wave64 processes one block at a time.  Three block kernels over CSR (the
// panel layout has its own kernel, spmv_panel.hip, with the same arithmetic):
//  - "row": block row by block row; each lane streams 4 consecutive block
//    entries per step, two steps in flight (16-byte non-temporal value and
//    column loads, so the matrix stream does not evict the gathered vector
//    from L2), gathers x[col], FP32 accumulation, a fixed-order DPP reduction
//    across the wave; small blocks leave each row's sums in the lane of that
//    row and every lane finishes its own row;
//  - "stream": the block's entries as one contiguous range, 256 per step with
//    the next step's loads in flight, a segmented reduction across the wave,
//    per-row sums in LDS, lane i finishes row i;
//  - "pipe": the row kernel's arithmetic with the loads of the next step
//    (possibly the next block row's first) issued before the current step's
//    gathers.
// The grid is a multiple of the 8 XCDs; workgroup w runs on XCD w % 8 and each
// XCD owns a contiguous range of blocks, so the waves sharing one L2 touch
// neighbouring rows.  Every reduction has a fixed order: results are bitwise
// reproducible run to run.
#include "spmv_device.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <new>

namespace dvmat {

// Eight waves per SIMD (at most 64 VGPRs): the loads in flight, not the
// registers per wave, set the throughput of these kernels.
template <int KIND, int ST, int NRHS, int EPI, int B>
__global__ __launch_bounds__(kSpmvThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void spmv_kernel(SpmvParams P) {
    constexpr int kWaves = kSpmvThreads / kWaveSize;
    const WaveSlot w = wave_slot();
    const int64_t b0 = P.n_blocks * w.xcd / kNumXcd;
    const int64_t b1 = P.n_blocks * (w.xcd + 1) / kNumXcd;
    float fpart[NRHS];
#pragma unroll
    for (int h = 0; h < NRHS; ++h) fpart[h] = 0.0f;
    double cpart = 0.0;
    __shared__ f32x4 s_tab[(EPI == EPI_OBJ || EPI == EPI_CURV) ? 256 : 1];
    if constexpr (EPI == EPI_OBJ || EPI == EPI_CURV) {
        static_assert(kSpmvThreads == 256, "one table row per thread");
        s_tab[threadIdx.x] = reinterpret_cast<const f32x4*>(P.table)[threadIdx.x];
        __syncthreads();
    }
    // the unit's first and last block row; the next unit's are loaded while
    // this one runs (lanes 0 and 1)
    int64_t b = b0 + w.lw;
    int bnd = b < b1 ? P.blocks[b + (w.lane & 1)] : 0;
    __shared__ float s_acc[(KIND == KIND_STREAM && B == 1) ? kWaves : 1][kBlockRowsMax * NRHS];
    __shared__ int s_rel[(KIND == KIND_STREAM && B == 1) ? kWaves : 1][kBlockRowsMax + 1];
    for (; b < b1; b += w.waves_per_xcd) {
        const int r0 = __builtin_amdgcn_readlane(bnd, 0);
        const int r1 = __builtin_amdgcn_readlane(bnd, 1);
        const int64_t bn = b + w.waves_per_xcd;
        if (bn < b1) bnd = P.blocks[bn + (w.lane & 1)];
        if constexpr (KIND == KIND_PIPE)
            block_pipe<ST, NRHS, EPI, false, B>(P, r0, r1, w.lane, s_tab, fpart, cpart);
        else if constexpr (KIND == KIND_ROW || B != 1)
            block_rows<ST, NRHS, EPI, false, B>(P, r0, r1, w.lane, s_tab, fpart, cpart);
        else
            block_stream<ST, NRHS, EPI, false>(P, r0, r1, w.lane, s_acc[w.wid], s_rel[w.wid], s_tab, fpart, cpart);
    }
    workgroup_partials<NRHS, EPI>(P, w.lane, w.wid, fpart, cpart);
}

// ---- batched launch over many plans ----------------------------------------

template <int KIND, int ST, int NRHS, int EPI, bool SCALE_X, int BR>
__global__ __launch_bounds__(kSpmvThreads) void spmv_batch_kernel(BatchParams B) {
    constexpr int kWaves = kSpmvThreads / kWaveSize;
    const WaveSlot w = wave_slot();
    const int64_t b0 = B.total_blocks * w.xcd / kNumXcd;
    const int64_t b1 = B.total_blocks * (w.xcd + 1) / kNumXcd;
    float fpart[NRHS];
#pragma unroll
    for (int h = 0; h < NRHS; ++h) fpart[h] = 0.0f;
    double cpart = 0.0;
    __shared__ float s_acc[kWaves][(KIND == KIND_STREAM ? kBlockRowsMax : 1) * NRHS];
    __shared__ int s_rel[kWaves][(KIND == KIND_STREAM ? kBlockRowsMax + 1 : 1)];
    static_assert(EPI == EPI_PLAIN || EPI == EPI_SCALE, "the batched launch has no objective epilogue");
    int p = 0;
    for (int64_t b = b0 + w.lw; b < b1; b += w.waves_per_xcd) {
        while (p + 1 < B.n_plans && B.plans[p + 1].block_base <= b) ++p;   // b only grows
        const PlanDev& pd = B.plans[p];
        const int r0 = pd.blocks[b - pd.block_base];
        const int r1 = pd.blocks[b - pd.block_base + 1];
        SpmvParams P{};
        P.n_rows = pd.n_rows;
        P.perm = pd.perm;
        P.rowptr = pd.rowptr;
        P.col = pd.col;
        P.val = pd.val;
        P.blocks = pd.blocks;
        P.n_blocks = pd.n_blocks;
        P.x = B.x[p];
        P.y = B.y[p];
        P.row_scale = pd.scale;
        P.x_scale = pd.scale;
        P.ld = NRHS;
        if constexpr (KIND == KIND_ROW || BR != 1)
            block_rows<ST, NRHS, EPI, SCALE_X, BR>(P, r0, r1, w.lane, nullptr, fpart, cpart);
        else
            block_stream<ST, NRHS, EPI, SCALE_X>(P, r0, r1, w.lane, s_acc[w.wid], s_rel[w.wid], nullptr, fpart,
                                                 cpart);
    }
}

// ---- small kernels -----------------------------------------------------------

// Sum of per-workgroup partials in a fixed order (FP64), one workgroup.
__global__ __launch_bounds__(256) void finalize_f_kernel(const float* partial, int nwg, int nrhs, float* F) {
    __shared__ double s[256];
    for (int h = 0; h < nrhs; ++h) {
        double a = 0.0;
        for (int i = threadIdx.x; i < nwg; i += 256) a += (double)partial[(int64_t)i * nrhs + h];
        s[threadIdx.x] = a;
        __syncthreads();
        for (int o = 128; o >= 1; o >>= 1) {
            if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) F[h] = (float)s[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void finalize_d_kernel(const double* partial, int nwg, double* out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < nwg; i += 256) a += partial[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// Standalone objective over an external dose (grid-stride, fixed grid).
__global__ __launch_bounds__(256) void objective_kernel(const float* z, int64_t n, int nrhs, const uint8_t* sid,
                                                        const float* table, float* g, float* partial) {
    __shared__ float s[256 * kMaxRhs];
    float acc[kMaxRhs];
    for (int h = 0; h < kMaxRhs; ++h) acc[h] = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int st = sid[i];
        const float T = table[st * 4 + 0], wo = table[st * 4 + 1], wu = table[st * 4 + 2];
        for (int h = 0; h < nrhs; ++h) {
            const float zz = z[i * nrhs + h];
            const float over = fmaxf(zz - T, 0.0f), under = fmaxf(T - zz, 0.0f);
            if (g) g[i * nrhs + h] = 2.0f * wo * over - 2.0f * wu * under;
            acc[h] += wo * over * over + wu * under * under;
        }
    }
    for (int h = 0; h < nrhs; ++h) s[h * 256 + threadIdx.x] = acc[h];
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int h = 0; h < nrhs; ++h) s[h * 256 + threadIdx.x] += s[h * 256 + threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int h = 0; h < nrhs; ++h) partial[(int64_t)blockIdx.x * nrhs + h] = s[h * 256];
}

// xs_j = s_j * x_j (16-bit storage keeps D_ij / s_j; the scale moves onto x).
__global__ __launch_bounds__(256) void scale_x_kernel(const float* x, const float* scale, int64_t n_bl, int nrhs,
                                                      float* xs) {
    const int64_t n = n_bl * nrhs;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        xs[i] = x[i] * scale[i / nrhs];
}

// ---- launch plumbing ---------------------------------------------------------

static int clamp_workgroups(int want, int64_t n_blocks) {
    const int64_t need = (n_blocks + 3) / 4;
    int64_t w = std::min<int64_t>(want, need);
    w = (w + kNumXcd - 1) / kNumXcd * kNumXcd;
    w = std::max<int64_t>(kNumXcd, std::min<int64_t>(w, kMaxSpmvWorkgroups));
    return (int)w;
}

// Default launch shape; the autotuner overrides it per matrix orientation.
static KernelCfg default_cfg() {
    KernelCfg c{KIND_ROW, 2048};
    if (const char* s = std::getenv("DVMAT_SPMV_KIND")) c.kind = s[0] == 's' ? KIND_STREAM : s[0] == 'p' ? KIND_PIPE : KIND_ROW;
    if (const char* s = std::getenv("DVMAT_SPMV_WG")) c.workgroups = std::max(8, std::atoi(s));
    return c;
}

template <int KIND, int ST, int EPI, int B>
static void launch_nrhs(const SpmvParams& P, int nrhs, int nwg, hipStream_t s) {
    dim3 grid(nwg), block(kSpmvThreads);
    switch (nrhs) {
#define DVMAT_CASE(N) \
    case N: hipLaunchKernelGGL((spmv_kernel<KIND, ST, N, EPI, B>), grid, block, 0, s, P); break;
        DVMAT_CASE(1) DVMAT_CASE(2) DVMAT_CASE(3) DVMAT_CASE(4)
        DVMAT_CASE(5) DVMAT_CASE(6) DVMAT_CASE(7) DVMAT_CASE(8)
#undef DVMAT_CASE
        default: break;
    }
}

template <int ST, int EPI>
static void launch_st(const KernelCfg& cfg, int B, const SpmvParams& P, int nrhs, int nwg, hipStream_t s) {
    if (cfg.kind == KIND_PIPE) {
        if (B == 4) launch_nrhs<KIND_PIPE, ST, EPI, 4>(P, nrhs, nwg, s);
        else if (B == 2) launch_nrhs<KIND_PIPE, ST, EPI, 2>(P, nrhs, nwg, s);
        else launch_nrhs<KIND_PIPE, ST, EPI, 1>(P, nrhs, nwg, s);
    } else if (B == 4) launch_nrhs<KIND_ROW, ST, EPI, 4>(P, nrhs, nwg, s);
    else if (B == 2) launch_nrhs<KIND_ROW, ST, EPI, 2>(P, nrhs, nwg, s);
    else if (cfg.kind == KIND_STREAM) launch_nrhs<KIND_STREAM, ST, EPI, 1>(P, nrhs, nwg, s);
    else launch_nrhs<KIND_ROW, ST, EPI, 1>(P, nrhs, nwg, s);
}

template <int EPI>
static void launch_spmv(const KernelCfg& cfg, int storage, int B, const SpmvParams& P0, int nrhs, hipStream_t s) {
    const int nwg = clamp_workgroups(cfg.workgroups, P0.n_blocks);
    SpmvParams P = P0;
    P.ld = nrhs;
    if (storage == DVMAT_F32) launch_st<DVMAT_F32, EPI>(cfg, B, P, nrhs, nwg, s);
    else if (storage == DVMAT_F16) launch_st<DVMAT_F16, EPI>(cfg, B, P, nrhs, nwg, s);
    else launch_st<DVMAT_BF16, EPI>(cfg, B, P, nrhs, nwg, s);
}

// Curvature only needs one right-hand side.
template <int ST>
static void launch_curv_st(const KernelCfg& cfg, int B, const SpmvParams& P, int nwg, hipStream_t s) {
    dim3 grid(nwg), block(kSpmvThreads);
    if (cfg.kind == KIND_PIPE) {
        if (B == 4) hipLaunchKernelGGL((spmv_kernel<KIND_PIPE, ST, 1, EPI_CURV, 4>), grid, block, 0, s, P);
        else if (B == 2) hipLaunchKernelGGL((spmv_kernel<KIND_PIPE, ST, 1, EPI_CURV, 2>), grid, block, 0, s, P);
        else hipLaunchKernelGGL((spmv_kernel<KIND_PIPE, ST, 1, EPI_CURV, 1>), grid, block, 0, s, P);
    } else if (B == 4) hipLaunchKernelGGL((spmv_kernel<KIND_ROW, ST, 1, EPI_CURV, 4>), grid, block, 0, s, P);
    else if (B == 2) hipLaunchKernelGGL((spmv_kernel<KIND_ROW, ST, 1, EPI_CURV, 2>), grid, block, 0, s, P);
    else if (cfg.kind == KIND_STREAM) hipLaunchKernelGGL((spmv_kernel<KIND_STREAM, ST, 1, EPI_CURV, 1>), grid, block, 0, s, P);
    else hipLaunchKernelGGL((spmv_kernel<KIND_ROW, ST, 1, EPI_CURV, 1>), grid, block, 0, s, P);
}

static void launch_curv(const KernelCfg& cfg, int storage, int B, const SpmvParams& P0, hipStream_t s) {
    const int nwg = clamp_workgroups(cfg.workgroups, P0.n_blocks);
    SpmvParams P = P0;
    P.ld = 1;
    if (storage == DVMAT_F32) launch_curv_st<DVMAT_F32>(cfg, B, P, nwg, s);
    else if (storage == DVMAT_F16) launch_curv_st<DVMAT_F16>(cfg, B, P, nwg, s);
    else launch_curv_st<DVMAT_BF16>(cfg, B, P, nwg, s);
}

static int elementwise_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

static dvmat_status check_ddc(const dvmat_ddc_s* d, const char* fn) {
    if (!d) return set_error(DVMAT_E_ARG, "%s: ddc is NULL", fn);
    if (!d->bound) return set_error(DVMAT_E_STATE, "%s: ddc not bound to a device workspace", fn);
    return DVMAT_OK;
}

static SpmvParams orientation_params(const CsrDev& c) {
    SpmvParams P{};
    P.n_rows = c.n_rows;
    P.perm = c.perm;
    P.perm_runs = c.perm_runs;
    P.rowptr = c.rowptr;
    P.col = c.col;
    P.val = c.val;
    P.blocks = c.blocks;
    P.n_blocks = c.n_blocks;
    return P;
}

// One product over an orientation in its layout: the panel kernel, or a CSR
// kernel of the configured kind.  nwg: workgroups launched (partial sums).
template <int EPI>
static dvmat_status run_orientation(const dvmat_ddc_s* d, const CsrDev& c, const KernelCfg& cfg, SpmvParams P,
                                    const float* x, int nrhs, hipStream_t s, int* nwg) {
    // the price's long beamlet rows gain 2 % from XCD-contiguous parts; the dose lost 2 % with them
    if (c.layout >= 1) return launch_panel<EPI>(cfg, d->storage, c, P, x, nrhs, s, nwg, &c == &d->price);
    P.x = x;
    *nwg = clamp_workgroups(cfg.workgroups, P.n_blocks);
    if constexpr (EPI == EPI_CURV) launch_curv(cfg, d->storage, c.B, P, s);
    else launch_spmv<EPI>(cfg, d->storage, c.B, P, nrhs, s);
    return check_hip(hipGetLastError(), "sparse product launch");
}

// The dose input: x itself, or s_j x_j for 16-bit storage (values hold D_ij / s_j).
static const float* dose_input(dvmat_ddc_s* d, const float* x, int nrhs, hipStream_t s) {
    if (d->storage == DVMAT_F32) return x;
    hipLaunchKernelGGL(scale_x_kernel, dim3(elementwise_grid(d->n_bl * nrhs)), dim3(256), 0, s, x, d->scale, d->n_bl,
                       nrhs, d->xs);
    return d->xs;
}

// Plain dose (no objective), used by the public call and the autotuner.
static dvmat_status dose_plain(dvmat_ddc_s* d, const KernelCfg& cfg, const float* x, int nrhs, float* z, hipStream_t s) {
    const float* xin = dose_input(d, x, nrhs, s);
    SpmvParams P = orientation_params(d->dose);
    P.y = z;
    int nwg = 0;
    return run_orientation<EPI_PLAIN>(d, d->dose, cfg, P, xin, nrhs, s, &nwg);
}

// Dose with the objective epilogue: z, dF/dz (g, nullable) and F (nullable).
static dvmat_status dose_obj(dvmat_ddc_s* d, const KernelCfg& cfg, const float* x, int nrhs, float* z,
                             const dvmat_obj_s* obj, float* g, float* F, hipStream_t s) {
    const float* xin = dose_input(d, x, nrhs, s);
    SpmvParams P = orientation_params(d->dose);
    P.y = z;
    P.sid = obj->sid;
    P.table = obj->table;
    P.g = g;
    P.partial = obj->partial;
    int nwg = 0;
    dvmat_status st = run_orientation<EPI_OBJ>(d, d->dose, cfg, P, xin, nrhs, s, &nwg);
    if (st) return st;
    if (F) hipLaunchKernelGGL(finalize_f_kernel, dim3(1), dim3(256), 0, s, obj->partial, nwg, nrhs, F);
    return check_hip(hipGetLastError(), "dose launch");
}

static dvmat_status price_any(dvmat_ddc_s* d, const KernelCfg& cfg, const float* g, int nrhs, float* p, hipStream_t s) {
    SpmvParams P = orientation_params(d->price);
    P.y = p;
    P.row_scale = d->scale;
    int nwg = 0;
    if (d->storage == DVMAT_F32) return run_orientation<EPI_PLAIN>(d, d->price, cfg, P, g, nrhs, s, &nwg);
    return run_orientation<EPI_SCALE>(d, d->price, cfg, P, g, nrhs, s, &nwg);
}

}  // namespace dvmat

struct dvmat_batch_s {
    int32_t n = 0;
    int32_t storage = DVMAT_F32;
    std::vector<int64_t> n_vox, n_bl;
    dvmat::PlanDev* dose_plans = nullptr;    // device
    dvmat::PlanDev* price_plans = nullptr;   // device
    int64_t dose_blocks = 0, price_blocks = 0;    // work units (CSR) or parts (panels) of all plans
    dvmat::KernelCfg dose_cfg{}, price_cfg{};
    int dose_B = 1, price_B = 1;
    int dose_layout = 0, price_layout = 0;
    int dose_W = 0, price_W = 0;                   // lanes per row of sliced panels
    int64_t dose_max_cols = 0, price_max_cols = 0; // largest panel column list over the plans
};

namespace dvmat {

template <int KIND, int ST, int EPI, bool SCALE_X, int BR>
static void launch_batch_nrhs(const BatchParams& B, int nrhs, int nwg, hipStream_t s) {
    dim3 grid(nwg), block(kSpmvThreads);
    switch (nrhs) {
#define DVMAT_CASE(N) \
    case N: hipLaunchKernelGGL((spmv_batch_kernel<KIND, ST, N, EPI, SCALE_X, BR>), grid, block, 0, s, B); break;
        DVMAT_CASE(1) DVMAT_CASE(2) DVMAT_CASE(4) DVMAT_CASE(8)
#undef DVMAT_CASE
        default: break;
    }
}

template <int ST, int EPI, bool SCALE_X>
static void launch_batch_st(int kind, int BR, const BatchParams& B, int nrhs, int nwg, hipStream_t s) {
    if (BR == 4) launch_batch_nrhs<KIND_ROW, ST, EPI, SCALE_X, 4>(B, nrhs, nwg, s);
    else if (BR == 2) launch_batch_nrhs<KIND_ROW, ST, EPI, SCALE_X, 2>(B, nrhs, nwg, s);
    else if (kind == KIND_STREAM) launch_batch_nrhs<KIND_STREAM, ST, EPI, SCALE_X, 1>(B, nrhs, nwg, s);
    else launch_batch_nrhs<KIND_ROW, ST, EPI, SCALE_X, 1>(B, nrhs, nwg, s);
}

// dose: plain epilogue, 16-bit scale applied to each gathered entry;
// price: 16-bit scale applied per output row.
template <bool DOSE>
static void launch_batch(const dvmat_batch_s* bt, const KernelCfg& cfg, const BatchParams& B, int nrhs,
                         hipStream_t s) {
    const int nwg = clamp_workgroups(cfg.workgroups, B.total_blocks);
    const int st = bt->storage;
    const int BR = DOSE ? bt->dose_B : bt->price_B;
    if (st == DVMAT_F32) launch_batch_st<DVMAT_F32, EPI_PLAIN, false>(cfg.kind, BR, B, nrhs, nwg, s);
    else if (st == DVMAT_F16) {
        if (DOSE) launch_batch_st<DVMAT_F16, EPI_PLAIN, true>(cfg.kind, BR, B, nrhs, nwg, s);
        else launch_batch_st<DVMAT_F16, EPI_SCALE, false>(cfg.kind, BR, B, nrhs, nwg, s);
    } else {
        if (DOSE) launch_batch_st<DVMAT_BF16, EPI_PLAIN, true>(cfg.kind, BR, B, nrhs, nwg, s);
        else launch_batch_st<DVMAT_BF16, EPI_SCALE, false>(cfg.kind, BR, B, nrhs, nwg, s);
    }
}

static dvmat_status batch_call(dvmat_batch_s* bt, bool dose, const KernelCfg& cfg, const float* const* in,
                               int32_t nrhs, float* const* out, hipStream_t s, const char* fn) {
    if (!bt || !in || !out) return set_error(DVMAT_E_ARG, "%s: NULL argument", fn);
    if (nrhs != 1 && nrhs != 2 && nrhs != 4 && nrhs != 8)
        return set_error(DVMAT_E_ARG, "%s: nrhs=%d not in {1,2,4,8}", fn, nrhs);
    BatchParams B{};
    B.plans = dose ? bt->dose_plans : bt->price_plans;
    B.n_plans = bt->n;
    B.total_blocks = dose ? bt->dose_blocks : bt->price_blocks;
    for (int i = 0; i < bt->n; ++i) {
        if (!in[i] || !out[i]) return set_error(DVMAT_E_ARG, "%s: NULL vector for plan %d", fn, i);
        B.x[i] = in[i];
        B.y[i] = out[i];
    }
    const int layout = dose ? bt->dose_layout : bt->price_layout;
    const int Bk = layout == 2 ? -(dose ? bt->dose_W : bt->price_W) : (dose ? bt->dose_B : bt->price_B);
    if (layout >= 1)
        return launch_batch_panel(bt->storage, Bk,
                                  !dose && bt->storage != DVMAT_F32, dose && bt->storage != DVMAT_F32,
                                  dose ? bt->dose_max_cols : bt->price_max_cols, B, nrhs, cfg.workgroups, s);
    if (dose) launch_batch<true>(bt, cfg, B, nrhs, s);
    else launch_batch<false>(bt, cfg, B, nrhs, s);
    return check_hip(hipGetLastError(), fn);
}

// ---- autotuner ---------------------------------------------------------------

static const int kTuneWorkgroups[] = {1024, 2048, 4096, 8192};

template <class Run>
static dvmat_status time_config(Run&& run, int reps, hipStream_t s, float* ms_out) {
    hipEvent_t a, b;
    dvmat_status st = check_hip(hipEventCreate(&a), "autotune event");
    if (st) return st;
    if ((st = check_hip(hipEventCreate(&b), "autotune event"))) { (void)hipEventDestroy(a); return st; }
    st = run();                                              // warm-up
    if (!st) st = check_hip(hipEventRecord(a, s), "autotune record");
    for (int i = 0; i < reps && !st; ++i) st = run();
    if (!st) st = check_hip(hipEventRecord(b, s), "autotune record");
    if (!st) st = check_hip(hipEventSynchronize(b), "autotune sync");
    float ms = 0.0f;
    if (!st) st = check_hip(hipEventElapsedTime(&ms, a, b), "autotune elapsed");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms_out = ms / std::max(reps, 1);
    return st;
}

template <class RunCfg>
static dvmat_status tune(RunCfg&& run_cfg, int reps, hipStream_t s, KernelCfg* best, float* best_ms, int B,
                         bool with_pipe = true, bool panel = false) {
    *best_ms = INFINITY;
    for (int kind : {KIND_ROW, KIND_STREAM, KIND_PIPE, KIND_PANEL})
        for (int wg : kTuneWorkgroups) {
            if (panel != (kind == KIND_PANEL)) continue;
            if ((kind == KIND_STREAM && B != 1) || (kind == KIND_PIPE && !with_pipe)) continue;
            KernelCfg c{kind, wg};
            float ms = 0.0f;
            dvmat_status st = time_config([&] { return run_cfg(c); }, reps, s, &ms);
            if (st) return st;
            if (std::getenv("DVMAT_AUTOTUNE_VERBOSE"))
                fprintf(stderr, "[dvmat autotune] kernel=%s workgroups=%d %.4f ms\n",
                        kind == KIND_ROW ? "row" : kind == KIND_STREAM ? "stream" : kind == KIND_PIPE ? "pipe" : "panel",
                        wg, ms);
            if (ms < *best_ms) { *best_ms = ms; *best = c; }
        }
    return DVMAT_OK;
}

}  // namespace dvmat

using namespace dvmat;

extern "C" {

dvmat_status dvmat_obj_workspace_size(int32_t n_struct, size_t* bytes) {
    if (!bytes) return set_error(DVMAT_E_ARG, "dvmat_obj_workspace_size: bytes is NULL");
    if (n_struct < 1 || n_struct > 256)
        return set_error(DVMAT_E_ARG, "dvmat_obj_workspace_size: n_struct=%d not in 1..256", n_struct);
    *bytes = align_up(256 * 4 * sizeof(float)) + align_up((size_t)kMaxSpmvWorkgroups * kMaxRhs * sizeof(float)) +
             align_up((size_t)kMaxSpmvWorkgroups * sizeof(double));
    return DVMAT_OK;
}

dvmat_status dvmat_obj_create(int64_t n_vox, int32_t n_struct, const uint8_t* d_sid, const float* table,
                              void* ws, size_t bytes, dvmat_stream stream, dvmat_obj* out) {
    if (!out) return set_error(DVMAT_E_ARG, "dvmat_obj_create: out is NULL");
    *out = nullptr;
    size_t need = 0;
    dvmat_status st = dvmat_obj_workspace_size(n_struct, &need);
    if (st) return st;
    if (n_vox < 1) return set_error(DVMAT_E_ARG, "dvmat_obj_create: n_vox < 1");
    if (!d_sid || !table || !ws) return set_error(DVMAT_E_ARG, "dvmat_obj_create: NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return set_error(DVMAT_E_ARG, "dvmat_obj_create: workspace misaligned");
    if (bytes < need) return set_error(DVMAT_E_NOMEM, "dvmat_obj_create: workspace %zu < %zu bytes", bytes, need);
    for (int i = 0; i < n_struct * 3; ++i)
        if (!std::isfinite(table[i])) return set_error(DVMAT_E_ARG, "dvmat_obj_create: non-finite table entry %d", i);
    dvmat_obj_s* o = new (std::nothrow) dvmat_obj_s();
    if (!o) return set_error(DVMAT_E_NOMEM, "dvmat_obj_create: host allocation failed");
    char* base = static_cast<char*>(ws);
    o->n_vox = n_vox;
    o->n_struct = n_struct;
    o->sid = d_sid;
    o->table = reinterpret_cast<float*>(base);
    o->partial = reinterpret_cast<float*>(base + align_up(256 * 4 * sizeof(float)));
    o->partial_d = reinterpret_cast<double*>(base + align_up(256 * 4 * sizeof(float)) +
                                             align_up((size_t)kMaxSpmvWorkgroups * kMaxRhs * sizeof(float)));
    // padded 4-wide table; rows past n_struct are zero (no objective)
    std::vector<float> host_tab(256 * 4, 0.0f);
    for (int s = 0; s < n_struct; ++s)
        for (int c = 0; c < 3; ++c) host_tab[s * 4 + c] = table[s * 3 + c];
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    st = check_hip(hipMemcpyAsync(o->table, host_tab.data(), host_tab.size() * sizeof(float), hipMemcpyHostToDevice, hs),
                   "dvmat_obj_create: table copy");
    if (st == DVMAT_OK) st = check_hip(hipStreamSynchronize(hs), "dvmat_obj_create: synchronize");
    if (st) { delete o; return st; }
    *out = o;
    return DVMAT_OK;
}

void dvmat_obj_destroy(dvmat_obj o) { delete o; }

dvmat_status dvmat_objective(dvmat_obj o, const float* z, int32_t nrhs, float* g, float* F, dvmat_stream stream) {
    if (!o || !z) return set_error(DVMAT_E_ARG, "dvmat_objective: NULL argument");
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(DVMAT_E_ARG, "dvmat_objective: nrhs=%d not in 1..8", nrhs);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int grid = std::min(elementwise_grid(o->n_vox), 1024);
    hipLaunchKernelGGL(objective_kernel, dim3(grid), dim3(256), 0, s, z, o->n_vox, nrhs, o->sid, o->table, g,
                       o->partial);
    if (F) hipLaunchKernelGGL(finalize_f_kernel, dim3(1), dim3(256), 0, s, o->partial, grid, nrhs, F);
    return check_hip(hipGetLastError(), "dvmat_objective launch");
}

dvmat_status dvmat_dose(dvmat_ddc d, const float* x, int32_t nrhs, float* z, dvmat_obj obj, float* g, float* F,
                        dvmat_stream stream) {
    dvmat_status st = check_ddc(d, "dvmat_dose");
    if (st) return st;
    if (!x || !z) return set_error(DVMAT_E_ARG, "dvmat_dose: x and z must be non-NULL");
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(DVMAT_E_ARG, "dvmat_dose: nrhs=%d not in 1..8", nrhs);
    if (obj && obj->n_vox != d->n_vox)
        return set_error(DVMAT_E_SHAPE, "dvmat_dose: objective has %lld voxels, matrix %lld",
                         (long long)obj->n_vox, (long long)d->n_vox);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!obj) return dose_plain(d, d->dose_cfg, x, nrhs, z, s);
    return dose_obj(d, d->dose_cfg, x, nrhs, z, obj, g, F, s);
}

dvmat_status dvmat_price(dvmat_ddc d, const float* g, int32_t nrhs, float* p, dvmat_stream stream) {
    dvmat_status st = check_ddc(d, "dvmat_price");
    if (st) return st;
    if (!g || !p) return set_error(DVMAT_E_ARG, "dvmat_price: g and p must be non-NULL");
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(DVMAT_E_ARG, "dvmat_price: nrhs=%d not in 1..8", nrhs);
    return price_any(d, d->price_cfg, g, nrhs, p, reinterpret_cast<hipStream_t>(stream));
}

dvmat_status dvmat_dose_curvature(dvmat_ddc d, const float* x_dir, dvmat_obj obj, const float* z_ref, float* d_out,
                                  double* curv, dvmat_stream stream) {
    dvmat_status st = check_ddc(d, "dvmat_dose_curvature");
    if (st) return st;
    if (!x_dir || !obj || !z_ref || !curv) return set_error(DVMAT_E_ARG, "dvmat_dose_curvature: NULL argument");
    if (obj->n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_dose_curvature: voxel count mismatch");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float* xin = dose_input(d, x_dir, 1, s);
    SpmvParams P = orientation_params(d->dose);
    P.y = d_out;
    P.sid = obj->sid;
    P.table = obj->table;
    P.zref = z_ref;
    P.partial_d = obj->partial_d;
    int nwg = 0;
    st = run_orientation<EPI_CURV>(d, d->dose, d->dose_cfg, P, xin, 1, s, &nwg);
    if (st) return st;
    hipLaunchKernelGGL(finalize_d_kernel, dim3(1), dim3(256), 0, s, obj->partial_d, nwg, curv);
    return check_hip(hipGetLastError(), "dvmat_dose_curvature launch");
}

dvmat_status dvmat_ddc_autotune(dvmat_ddc d, const float* x, float* z, const float* g, float* p, int32_t reps,
                                dvmat_stream stream) {
    dvmat_status st = check_ddc(d, "dvmat_ddc_autotune");
    if (st) return st;
    if (!x || !z || !g || !p) return set_error(DVMAT_E_ARG, "dvmat_ddc_autotune: NULL argument");
    if (reps < 1) return set_error(DVMAT_E_ARG, "dvmat_ddc_autotune: reps < 1");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KernelCfg best{};
    float ms = 0.0f;
    st = tune([&](const KernelCfg& c) { return dose_plain(d, c, x, 1, z, s); }, reps, s, &best, &ms, d->dose.B, true,
              d->dose.layout >= 1);
    if (st) return st;
    d->dose_cfg = best;
    d->dose_tuned_ms = ms;
    st = tune([&](const KernelCfg& c) { return price_any(d, c, g, 1, p, s); }, reps, s, &best, &ms, d->price.B, true,
              d->price.layout >= 1);
    if (st) return st;
    d->price_cfg = best;
    d->price_tuned_ms = ms;
    return DVMAT_OK;
}

dvmat_status dvmat_ddc_autotune_obj(dvmat_ddc d, dvmat_obj obj, const float* x, int32_t nrhs, float* z, float* g,
                                    float* F, float* p, int32_t reps, dvmat_stream stream) {
    dvmat_status st = check_ddc(d, "dvmat_ddc_autotune_obj");
    if (st) return st;
    if (!obj || !x || !z || !g || !F || !p) return set_error(DVMAT_E_ARG, "dvmat_ddc_autotune_obj: NULL argument");
    if (obj->n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_ddc_autotune_obj: voxel count mismatch");
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(DVMAT_E_ARG, "dvmat_ddc_autotune_obj: nrhs=%d not in 1..8", nrhs);
    if (reps < 1) return set_error(DVMAT_E_ARG, "dvmat_ddc_autotune_obj: reps < 1");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KernelCfg best{};
    float ms = 0.0f;
    st = tune([&](const KernelCfg& c) { return dose_obj(d, c, x, nrhs, z, obj, g, F, s); }, reps, s, &best, &ms,
              d->dose.B, true, d->dose.layout >= 1);
    if (st) return st;
    d->dose_cfg = best;
    d->dose_tuned_ms = ms;
    // the price of the gradient the dose just wrote, as the loop runs it
    st = tune([&](const KernelCfg& c) { return price_any(d, c, g, nrhs, p, s); }, reps, s, &best, &ms, d->price.B,
              true, d->price.layout >= 1);
    if (st) return st;
    d->price_cfg = best;
    d->price_tuned_ms = ms;
    return DVMAT_OK;
}

dvmat_status dvmat_ddc_set_kernel(dvmat_ddc d, int32_t orientation, int32_t kind, int32_t workgroups) {
    if (!d) return set_error(DVMAT_E_ARG, "dvmat_ddc_set_kernel: NULL handle");
    if (kind != KIND_ROW && kind != KIND_STREAM && kind != KIND_PIPE && kind != KIND_PANEL)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_set_kernel: kind %d", kind);
    if (workgroups < kNumXcd || workgroups > kMaxSpmvWorkgroups)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_set_kernel: workgroups %d not in [8, 8192]", workgroups);
    KernelCfg c{kind, workgroups};
    if (orientation != 0 && orientation != 1)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_set_kernel: orientation %d", orientation);
    if (kind == KIND_STREAM && (orientation == 0 ? d->dose.B : d->price.B) != 1)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_set_kernel: the stream kernel needs one row per block row");
    if ((kind == KIND_PANEL) != ((orientation == 0 ? d->dose.layout : d->price.layout) >= 1))
        return set_error(DVMAT_E_ARG, "dvmat_ddc_set_kernel: kind 3 (panel) goes with the panel layout and only there");
    if (orientation == 0) d->dose_cfg = c;
    else d->price_cfg = c;
    return DVMAT_OK;
}

// ---- batched plans -------------------------------------------------------------

dvmat_status dvmat_batch_workspace_size(int32_t n, size_t* bytes) {
    if (!bytes) return set_error(DVMAT_E_ARG, "dvmat_batch_workspace_size: bytes is NULL");
    if (n < 1 || n > kMaxBatch) return set_error(DVMAT_E_ARG, "dvmat_batch_workspace_size: n=%d not in 1..%d", n, kMaxBatch);
    *bytes = 2 * align_up((size_t)n * sizeof(PlanDev));
    return DVMAT_OK;
}

dvmat_status dvmat_batch_create(const dvmat_ddc* ddcs, int32_t n, void* ws, size_t bytes, dvmat_stream stream,
                                dvmat_batch* out) {
    if (!out) return set_error(DVMAT_E_ARG, "dvmat_batch_create: out is NULL");
    *out = nullptr;
    size_t need = 0;
    dvmat_status st = dvmat_batch_workspace_size(n, &need);
    if (st) return st;
    if (!ddcs || !ws) return set_error(DVMAT_E_ARG, "dvmat_batch_create: NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return set_error(DVMAT_E_ARG, "dvmat_batch_create: workspace misaligned");
    if (bytes < need) return set_error(DVMAT_E_NOMEM, "dvmat_batch_create: workspace %zu < %zu bytes", bytes, need);
    std::vector<PlanDev> dp(n), pp(n);
    int64_t bd = 0, bp = 0, max_cols_d = 0, max_cols_p = 0;
    for (int i = 0; i < n; ++i) {
        const dvmat_ddc_s* d = ddcs[i];
        if ((st = check_ddc(d, "dvmat_batch_create"))) return st;
        if (d->storage != ddcs[0]->storage)
            return set_error(DVMAT_E_ARG, "dvmat_batch_create: plan %d has a different storage type", i);
        if (d->dose.B != ddcs[0]->dose.B || d->price.B != ddcs[0]->price.B)
            return set_error(DVMAT_E_ARG, "dvmat_batch_create: plan %d has a different block-row layout", i);
        if (d->dose.layout != ddcs[0]->dose.layout || d->price.layout != ddcs[0]->price.layout)
            return set_error(DVMAT_E_ARG, "dvmat_batch_create: plan %d has a different layout (CSR / panels)", i);
        if ((d->dose.layout == 2 && d->dose.slice_lanes != ddcs[0]->dose.slice_lanes) ||
            (d->price.layout == 2 && d->price.slice_lanes != ddcs[0]->price.slice_lanes))
            return set_error(DVMAT_E_ARG, "dvmat_batch_create: plan %d has different lanes per row of its slices", i);
        auto plan = [](const CsrDev& c, const float* scale, int64_t base) {
            PlanDev q{};
            q.rowptr = c.rowptr;
            q.col = c.col;
            q.val = c.val;
            q.blocks = c.blocks;
            q.scale = scale;
            q.perm = c.perm;
            q.perm_runs = c.perm_runs;
            q.n_rows = c.n_rows;
            q.block_base = base;
            q.n_blocks = c.layout >= 1 ? c.n_parts : c.n_blocks;
            q.col16 = c.col16;
            q.ulist = c.ulist;
            q.panel_u = c.panel_u;
            q.part_units = c.part_units;
            q.part_panel = c.part_panel;
            return q;
        };
        dp[i] = plan(d->dose, d->scale, bd);
        pp[i] = plan(d->price, d->scale, bp);
        bd += dp[i].n_blocks;
        bp += pp[i].n_blocks;
        max_cols_d = std::max<int64_t>(max_cols_d, d->dose.max_panel_cols);
        max_cols_p = std::max<int64_t>(max_cols_p, d->price.max_panel_cols);
    }
    dvmat_batch_s* bt = new (std::nothrow) dvmat_batch_s();
    if (!bt) return set_error(DVMAT_E_NOMEM, "dvmat_batch_create: host allocation failed");
    char* base = static_cast<char*>(ws);
    bt->n = n;
    bt->storage = ddcs[0]->storage;
    bt->dose_B = ddcs[0]->dose.B;
    bt->price_B = ddcs[0]->price.B;
    bt->dose_plans = reinterpret_cast<PlanDev*>(base);
    bt->price_plans = reinterpret_cast<PlanDev*>(base + align_up((size_t)n * sizeof(PlanDev)));
    bt->dose_blocks = bd;
    bt->price_blocks = bp;
    bt->dose_layout = ddcs[0]->dose.layout;
    bt->price_layout = ddcs[0]->price.layout;
    bt->dose_W = ddcs[0]->dose.slice_lanes;
    bt->price_W = ddcs[0]->price.slice_lanes;
    bt->dose_max_cols = max_cols_d;
    bt->price_max_cols = max_cols_p;
    bt->dose_cfg = default_cfg();
    bt->price_cfg = default_cfg();
    if (bt->dose_layout >= 1) bt->dose_cfg.kind = KIND_PANEL;
    if (bt->price_layout >= 1) bt->price_cfg.kind = KIND_PANEL;
    for (int i = 0; i < n; ++i) {
        bt->n_vox.push_back(ddcs[i]->n_vox);
        bt->n_bl.push_back(ddcs[i]->n_bl);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = check_hip(hipMemcpyAsync(bt->dose_plans, dp.data(), n * sizeof(PlanDev), hipMemcpyHostToDevice, s),
                   "dvmat_batch_create: copy");
    if (!st) st = check_hip(hipMemcpyAsync(bt->price_plans, pp.data(), n * sizeof(PlanDev), hipMemcpyHostToDevice, s),
                            "dvmat_batch_create: copy");
    if (!st) st = check_hip(hipStreamSynchronize(s), "dvmat_batch_create: synchronize");
    if (st) { delete bt; return st; }
    *out = bt;
    return DVMAT_OK;
}

void dvmat_batch_destroy(dvmat_batch b) { delete b; }

dvmat_status dvmat_batch_dose(dvmat_batch b, const float* const* xs, int32_t nrhs, float* const* zs,
                              dvmat_stream stream) {
    return batch_call(b, true, b ? b->dose_cfg : KernelCfg{}, xs, nrhs, zs, reinterpret_cast<hipStream_t>(stream),
                      "dvmat_batch_dose");
}

dvmat_status dvmat_batch_price(dvmat_batch b, const float* const* gs, int32_t nrhs, float* const* ps,
                               dvmat_stream stream) {
    return batch_call(b, false, b ? b->price_cfg : KernelCfg{}, gs, nrhs, ps, reinterpret_cast<hipStream_t>(stream),
                      "dvmat_batch_price");
}

dvmat_status dvmat_batch_autotune(dvmat_batch b, const float* const* xs, float* const* zs, const float* const* gs,
                                  float* const* ps, int32_t nrhs, int32_t reps, dvmat_stream stream) {
    if (!b || !xs || !zs || !gs || !ps) return set_error(DVMAT_E_ARG, "dvmat_batch_autotune: NULL argument");
    if (reps < 1) return set_error(DVMAT_E_ARG, "dvmat_batch_autotune: reps < 1");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    KernelCfg best{};
    float ms = 0.0f;
    dvmat_status st = tune([&](const KernelCfg& c) { return batch_call(b, true, c, xs, nrhs, zs, s, "dvmat_batch_autotune"); },
                           reps, s, &best, &ms, b->dose_B, false, b->dose_layout >= 1);
    if (st) return st;
    b->dose_cfg = best;
    st = tune([&](const KernelCfg& c) { return batch_call(b, false, c, gs, nrhs, ps, s, "dvmat_batch_autotune"); },
              reps, s, &best, &ms, b->price_B, false, b->price_layout >= 1);
    if (st) return st;
    b->price_cfg = best;
    return DVMAT_OK;
}

dvmat_status dvmat_batch_set_kernel(dvmat_batch b, int32_t orientation, int32_t kind, int32_t workgroups) {
    if (!b) return set_error(DVMAT_E_ARG, "dvmat_batch_set_kernel: NULL handle");
    if (kind != KIND_ROW && kind != KIND_STREAM && kind != KIND_PANEL)
        return set_error(DVMAT_E_ARG, "dvmat_batch_set_kernel: kind %d", kind);
    if (workgroups < kNumXcd || workgroups > kMaxSpmvWorkgroups)
        return set_error(DVMAT_E_ARG, "dvmat_batch_set_kernel: workgroups %d not in [8, 8192]", workgroups);
    if (orientation == 0 || orientation == 1) {
        const int layout = orientation == 0 ? b->dose_layout : b->price_layout;
        if ((kind == KIND_PANEL) != (layout >= 1))
            return set_error(DVMAT_E_ARG, "dvmat_batch_set_kernel: kind 3 (panel) goes with the panel layout and only there");
        if (kind == KIND_STREAM && (orientation == 0 ? b->dose_B : b->price_B) != 1)
            return set_error(DVMAT_E_ARG, "dvmat_batch_set_kernel: the stream kernel needs one row per block row");
    }
    KernelCfg c{kind, workgroups};
    if (orientation == 0) b->dose_cfg = c;
    else if (orientation == 1) b->price_cfg = c;
    else return set_error(DVMAT_E_ARG, "dvmat_batch_set_kernel: orientation %d", orientation);
    return DVMAT_OK;
}

dvmat_status dvmat_batch_info(dvmat_batch b, int64_t* dose_blocks, int64_t* price_blocks, int32_t* cfg) {
    if (!b) return set_error(DVMAT_E_ARG, "dvmat_batch_info: NULL handle");
    if (dose_blocks) *dose_blocks = b->dose_blocks;
    if (price_blocks) *price_blocks = b->price_blocks;
    if (cfg) {
        cfg[0] = b->dose_cfg.kind;
        cfg[1] = b->dose_cfg.workgroups;
        cfg[2] = b->price_cfg.kind;
        cfg[3] = b->price_cfg.workgroups;
    }
    return DVMAT_OK;
}

}  // extern "C"

namespace dvmat {
KernelCfg initial_kernel_cfg() { return default_cfg(); }
}  // namespace dvmat
