// Sparse products on the panel layout.
//
// The rows of one orientation are grouped into panels (a tile of the voxel
// grid for the dose; neighbouring beamlets at neighbouring gantry angles for
// the price).  Each panel lists the distinct columns its rows touch, and the
// stored column indices are positions in that list (16 bits).  A workgroup
// takes one part of a panel at a time (a run of its work units, so that large
// panels are shared out): it copies the panel's slice of the input vector
// into LDS (the sorted list read coalesced, several entries in flight per
// thread), then its eight waves run
// the block-row arithmetic of the CSR row kernel with gathers served by LDS.
// The gathers thus leave the L1/L2 request path, which bounds the CSR kernels:
// there a gathered value costs a cache-line request of its own, here a staged
// value serves tens of products (Sec. 2.2.2 gives the products; this layout is
// the GPU mapping of them).
//
// Right-hand sides beyond what LDS holds are processed in chunks, each chunk
// one launch over the matrix.
#include "spmv_device.hpp"

#include <algorithm>
#include <type_traits>

namespace dvmat {

struct PanelParams {
    const float* x;             // input vector, ldx values per column (chunk offset applied)
    int64_t ldx;
    const uint16_t* col16;
    const int32_t* ulist;
    const int64_t* panel_u;
    const int32_t* part_units;
    const int32_t* part_panel;
    int64_t n_parts;
    int xcd_runs;               // 1: each XCD takes a contiguous eighth of the parts
};

// Eight waves share one LDS slice.  Slices up to 36 KB (the widest dose
// panel of the full-scale single-arc workload has 9,114 columns under the
// default 12,288-column budget, 8,192 under the tuned one) let four
// workgroups fill a CU's 160 KB of LDS and all of its 32 wave slots.
constexpr int kPanelThreads = 512;

// Copy a panel's slice of the input into LDS: xs[i*R + h] = x[list[i]*ldx + h]
// (times scale[list[i]] when SCALE).  Each thread issues kDepth list loads,
// then kDepth gathers, then the LDS writes, so a slice of several thousand
// columns costs a few dependent round trips to memory instead of one per 512
// columns.  Indexes past the list's end are clamped to its last entry (loads
// stay in bounds, their values are not written).
template <int R, bool SCALE, int NT = kPanelThreads>
__device__ __forceinline__ void stage_slice(float* xs, const int32_t* __restrict__ list, int nu,
                                            const float* __restrict__ x, int64_t ldx,
                                            const float* __restrict__ scale) {
    constexpr int kDepth = R <= 2 ? 8 : 4;
    for (int i0 = threadIdx.x; i0 < nu; i0 += kDepth * NT) {
        int32_t j[kDepth];
#pragma unroll
        for (int u = 0; u < kDepth; ++u) j[u] = list[min(i0 + u * NT, nu - 1)];
        float v[kDepth][R];
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
            const float sc = SCALE ? scale[j[u]] : 1.0f;
#pragma unroll
            for (int h = 0; h < R; ++h) v[u][h] = x[(int64_t)j[u] * ldx + h] * sc;
        }
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
            const int i = i0 + u * NT;
            if (i < nu) {
#pragma unroll
                for (int h = 0; h < R; ++h) xs[i * R + h] = v[u][h];
            }
        }
    }
}

template <int ST, int R, int EPI, int B>
__global__ __launch_bounds__(kPanelThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void spmv_panel_kernel(
    SpmvParams P, PanelParams Q) {
    constexpr int kWaves = kPanelThreads / kWaveSize;
    extern __shared__ float xs[];
    __shared__ f32x4 s_tab[(EPI == EPI_OBJ || EPI == EPI_CURV) ? 256 : 1];
    if constexpr (EPI == EPI_OBJ || EPI == EPI_CURV) {
        if (threadIdx.x < 256) s_tab[threadIdx.x] = reinterpret_cast<const f32x4*>(P.table)[threadIdx.x];
    }
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    // four steps in flight for the long rows of D^T (a beamlet reaches well
    // over a thousand voxels); the dose's shorter voxel rows ran slower with
    // the larger loop body
    constexpr bool kDeep = EPI == EPI_PLAIN || EPI == EPI_SCALE;
    float fpart[R];
#pragma unroll
    for (int h = 0; h < R; ++h) fpart[h] = 0.0f;
    double cpart = 0.0;
    // with xcd_runs, workgroup b (dispatched to XCD b % 8) walks that XCD's
    // contiguous eighth of the parts: neighbouring panels share input columns
    // in its L2
    const int xcd = Q.xcd_runs ? (int)(blockIdx.x % kNumXcd) : 0;
    const int64_t stride = Q.xcd_runs ? gridDim.x / kNumXcd : gridDim.x;
    const int64_t t_end = Q.xcd_runs ? Q.n_parts * (xcd + 1) / kNumXcd : Q.n_parts;
    const int64_t t_begin = Q.xcd_runs ? Q.n_parts * xcd / kNumXcd + blockIdx.x / kNumXcd : blockIdx.x;
    for (int64_t t = t_begin; t < t_end; t += stride) {
        const int p = Q.part_panel[t];
        const int64_t u0 = Q.panel_u[p];
        const int nu = (int)(Q.panel_u[p + 1] - u0);
        __syncthreads();                              // the previous panel's gathers are done
        stage_slice<R, false>(xs, Q.ulist + u0, nu, Q.x, Q.ldx, nullptr);
        __syncthreads();
        const int q0 = Q.part_units[t], q1 = Q.part_units[t + 1];
        for (int q = q0 + wid; q < q1; q += kWaves)
            block_rows<ST, R, EPI, false, B, true, kDeep>(P, P.blocks[q], P.blocks[q + 1], lane, s_tab, fpart, cpart, xs,
                                                   Q.col16);
    }
    workgroup_partials_n<R, EPI, kWaves>(P, lane, wid, fpart, cpart);
}

// ---- sliced panels (layout 2) ------------------------------------------------
//
// A slice holds up to 64 / W rows of one panel, sorted by length; the wave's
// lanes i*W .. i*W + W-1 share row i and all rows advance together, E
// entries per lane and step (one 16-byte value load: 4 entries at FP32 with
// an 8-byte index load, 8 at 16 bits with a 16-byte one), four steps in flight
// (two for several right-hand sides, the curvature and bfloat16, whose
// registers would not hold four).  The step count is the slice's (uniform), so
// the loop has no per-lane exit and no partial step per row; the W lanes of a
// row are summed by DPP permutes at the end (two to four per slice instead of
// a whole-wave reduction per row).  Lanes past the slice's rows re-read an
// active lane's entries (same cache lines, no extra traffic) and store
// nothing.  Rows without entries come in slices with no steps: one lane per
// row writes its epilogue from zero sums.

// Sum over the W lanes of each row group, every lane of the group receiving it.
template <int W>
__device__ __forceinline__ float group_sum(float v) {
    static_assert(W == 1 || W == 2 || W == 4 || W == 8 || W == 16, "lanes per row");
    if constexpr (W >= 2) v = dpp_step<0xB1>(v);    // quad_perm [1,0,3,2]
    if constexpr (W >= 4) v = dpp_step<0x4E>(v);    // quad_perm [2,3,0,1]
    if constexpr (W >= 8) v = dpp_step<0x141>(v);   // row_half_mirror
    if constexpr (W >= 16) v = dpp_step<0x140>(v);  // row_mirror
    return v;
}

// A slice's first row position, row count, first entry and stored entries.
struct SliceDesc {
    int p0, nr, len;
    int64_t base;
};

__device__ __forceinline__ int64_t readlane64(int64_t v, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), j);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The epilogue inputs of a row whose natural index is known.
template <int EPI>
__device__ __forceinline__ EpiRow epi_load_nat(const SpmvParams& P, int64_t n) {
    EpiRow e{0, 0.0f, 1.0f};
    if constexpr (EPI == EPI_OBJ || EPI == EPI_CURV) e.sid = P.sid[n];
    if constexpr (EPI == EPI_CURV) e.zr = P.zref[n];
    if constexpr (EPI == EPI_SCALE) e.rs = P.row_scale[n];
    return e;
}

// Entries per lane and step: 16 bytes of values (4 at FP32, 8 at 16 bits).
template <int ST>
constexpr int slice_entries() { return ST == DVMAT_F32 ? 4 : 8; }

// One lane's entries of one step as loaded: 16 bytes of values (4 FP32 or 8
// 16-bit codes) and their panel-local columns (8 or 16 bytes); unpacked only
// when the products are formed, so that four steps in flight fit the
// registers.
typedef unsigned int u32x2v __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

template <int ST>
struct SliceStep {
    u32x4v v;
    typename std::conditional<ST == DVMAT_F32, u32x2v, u32x4v>::type c;
};

template <int ST>
__device__ __forceinline__ void slice_step_loads(const SpmvParams& P, const uint16_t* col16, int64_t k,
                                                 SliceStep<ST>& s) {
    constexpr int E = slice_entries<ST>();
    s.v = __builtin_nontemporal_load(reinterpret_cast<const u32x4v*>(P.val) + k / E);
    s.c = __builtin_nontemporal_load(reinterpret_cast<const decltype(s.c)*>(col16) + k / E);
}

template <int ST>
__device__ __forceinline__ void slice_step_zero(SliceStep<ST>& s) {
    s.v = u32x4v{0u, 0u, 0u, 0u};
}

__device__ __forceinline__ i32x4 unpack_cols(unsigned a, unsigned b) {
    return i32x4{(int)(a & 0xffffu), (int)(a >> 16), (int)(b & 0xffffu), (int)(b >> 16)};
}

template <int ST>
__device__ __forceinline__ f32x4 unpack_vals(unsigned a, unsigned b) {
    if constexpr (ST == DVMAT_F16) {
        typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
        const f16x2 x = __builtin_bit_cast(f16x2, a), y = __builtin_bit_cast(f16x2, b);
        return f32x4{(float)x.x, (float)x.y, (float)y.x, (float)y.y};
    } else {
        return f32x4{__uint_as_float(a << 16), __uint_as_float(a & 0xffff0000u), __uint_as_float(b << 16),
                     __uint_as_float(b & 0xffff0000u)};
    }
}

template <int ST, int R>
__device__ __forceinline__ void slice_step_fma(float (&acc)[1][R], const SpmvParams& P, const float* xs,
                                               const SliceStep<ST>& s) {
    if constexpr (ST == DVMAT_F32) {
        const f32x4 V[1] = {__builtin_bit_cast(f32x4, s.v)};
        fma4_blocked<R, 1, false>(acc, P, xs, V, unpack_cols(s.c.x, s.c.y));
    } else {
        const f32x4 V0[1] = {unpack_vals<ST>(s.v.x, s.v.y)};
        const f32x4 V1[1] = {unpack_vals<ST>(s.v.z, s.v.w)};
        fma4_blocked<R, 1, false>(acc, P, xs, V0, unpack_cols(s.c.x, s.c.y));
        fma4_blocked<R, 1, false>(acc, P, xs, V1, unpack_cols(s.c.z, s.c.w));
    }
}

template <int ST, int R, int EPI, int W>
__device__ __forceinline__ void slice_rows(const SpmvParams& P, const SliceDesc& d, int lane, const f32x4* tab,
                                           float (&fpart)[R], double& cpart, const float* xs,
                                           const uint16_t* col16) {
    // sliced panels always carry the row permutation (rows sorted by length)
    if (d.len == 0) {
        if (lane < d.nr) {
            const int64_t n = P.perm[d.p0 + lane];
            const EpiRow e = epi_load_nat<EPI>(P, n);
            float acc[R];
#pragma unroll
            for (int h = 0; h < R; ++h) acc[h] = 0.0f;
            row_epilogue<R, EPI>(P, n, e, tab, acc, fpart, cpart);
        }
        return;
    }
    const int i = lane / W;
    const bool act = i < d.nr;
    const int64_t nat = P.perm[d.p0 + (act ? i : 0)];
    constexpr int E = slice_entries<ST>();
    const int stride = d.nr * W * E;                   // entries per step
    const int S = d.len / stride;                      // >= 1
    const int64_t k0 = d.base + E * (act ? lane : lane % (d.nr * W));
    float acc[1][R];
#pragma unroll
    for (int h = 0; h < R; ++h) acc[0][h] = 0.0f;
    // steps in flight: four for one right-hand side, two where four would
    // not fit the registers (several right-hand sides, the curvature,
    // bfloat16's unpacking)
    constexpr int D = (R == 1 && EPI != EPI_CURV && ST != DVMAT_BF16) ? 4 : 2;
    // the first D steps without branches: steps past the slice's end re-read
    // its last step (lines already on their way) and count zero
    {
        SliceStep<ST> st[D];
#pragma unroll
        for (int j = 0; j < D; ++j) slice_step_loads<ST>(P, col16, k0 + (int64_t)min(j, S - 1) * stride, st[j]);
#pragma unroll
        for (int j = 1; j < D; ++j)
            if (j >= S) slice_step_zero<ST>(st[j]);
#pragma unroll
        for (int j = 0; j < D; ++j) slice_step_fma<ST, R>(acc, P, xs, st[j]);
    }
    // the epilogue inputs: the natural row arrived with the first steps, and
    // this load's latency hides behind the next steps'
    const EpiRow e = epi_load_nat<EPI>(P, nat);
    int64_t k = k0 + (int64_t)D * stride;
    int t = D;
    for (; t + D <= S; t += D) {
        SliceStep<ST> st[D];
#pragma unroll
        for (int j = 0; j < D; ++j) slice_step_loads<ST>(P, col16, k + j * stride, st[j]);
#pragma unroll
        for (int j = 0; j < D; ++j) slice_step_fma<ST, R>(acc, P, xs, st[j]);
        k += (int64_t)D * stride;
    }
    if (t < S) {
        // the last steps (fewer than D), loads issued together
        const int rem = S - t;
        SliceStep<ST> st[D - 1];
        slice_step_loads<ST>(P, col16, k, st[0]);
#pragma unroll
        for (int j = 1; j < D - 1; ++j)
            if (rem > j) slice_step_loads<ST>(P, col16, k + j * stride, st[j]);
        slice_step_fma<ST, R>(acc, P, xs, st[0]);
#pragma unroll
        for (int j = 1; j < D - 1; ++j)
            if (rem > j) slice_step_fma<ST, R>(acc, P, xs, st[j]);
    }
    float sum[R];
#pragma unroll
    for (int h = 0; h < R; ++h) sum[h] = group_sum<W>(acc[0][h]);
    if (act && lane % W == 0) row_epilogue<R, EPI>(P, nat, e, tab, sum, fpart, cpart);
}

// A part of sliced panels after its staging: the part's slices in a fixed
// order: a part's slices are sorted longest first, and wave w takes slice w
// of each round of NW, in reverse order every second round, so that each
// wave's share of a part comes out about even.  The descriptors of a wave's
// next 64 slices are read one per lane (SliceLanes; the caller reads the
// first 64 before the staging), so a slice starts without a round trip for
// them.
struct SliceLanes {
    int p0 = 0, p1 = 0;
    int64_t b0 = 0, b1 = 0;
};

template <int NW>
__device__ __forceinline__ int slice_of(int q0, int r, int wid) {
    return q0 + r * NW + ((r & 1) ? NW - 1 - wid : wid);
}

template <int NW>
__device__ __forceinline__ SliceLanes slice_lanes(const SpmvParams& P, int q0, int q1, int wid, int lane, int rb) {
    SliceLanes l;
    const int qj = slice_of<NW>(q0, rb + lane, wid);
    if (qj < q1) {
        l.p0 = P.blocks[qj];
        l.p1 = P.blocks[qj + 1];
        l.b0 = P.rowptr[qj];
        l.b1 = P.rowptr[qj + 1];
    }
    return l;
}

template <int ST, int R, int EPI, int W, int NW>
__device__ __forceinline__ void slice_part(const SpmvParams& P, const uint16_t* col16, int q0, int q1, int wid,
                                           int lane, SliceLanes dl, const f32x4* tab, float (&fpart)[R],
                                           double& cpart, const float* xs) {
    for (int rb = 0; slice_of<NW>(q0, rb, wid) < q1; rb += kWaveSize) {
        if (rb > 0) dl = slice_lanes<NW>(P, q0, q1, wid, lane, rb);
        for (int j = 0; j < kWaveSize && slice_of<NW>(q0, rb + j, wid) < q1; ++j) {
            SliceDesc d;
            d.p0 = __builtin_amdgcn_readlane(dl.p0, j);
            d.nr = __builtin_amdgcn_readlane(dl.p1, j) - d.p0;
            const int64_t b0 = readlane64(dl.b0, j);
            d.base = b0;
            d.len = (int)(readlane64(dl.b1, j) - b0);
            slice_rows<ST, R, EPI, W>(P, d, lane, tab, fpart, cpart, xs, col16);
        }
    }
}

template <int ST, int R, int EPI, int W>
__global__ __launch_bounds__(kPanelThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void spmv_slice_kernel(
    SpmvParams P, PanelParams Q) {
    constexpr int kWaves = kPanelThreads / kWaveSize;
    extern __shared__ float xs[];
    __shared__ f32x4 s_tab[(EPI == EPI_OBJ || EPI == EPI_CURV) ? 256 : 1];
    if constexpr (EPI == EPI_OBJ || EPI == EPI_CURV) {
        if (threadIdx.x < 256) s_tab[threadIdx.x] = reinterpret_cast<const f32x4*>(P.table)[threadIdx.x];
    }
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    float fpart[R];
#pragma unroll
    for (int h = 0; h < R; ++h) fpart[h] = 0.0f;
    double cpart = 0.0;
    for (int64_t t = blockIdx.x; t < Q.n_parts; t += gridDim.x) {
        const int p = Q.part_panel[t];
        const int64_t u0 = Q.panel_u[p];
        const int nu = (int)(Q.panel_u[p + 1] - u0);
        const int q0 = Q.part_units[t], q1 = Q.part_units[t + 1];
        __syncthreads();                              // the previous panel's gathers are done
        const SliceLanes dl = slice_lanes<kWaves>(P, q0, q1, wid, lane, 0);
        // a part of rows without entries (outside the body) needs no slice
        if (P.rowptr[q1] > P.rowptr[q0]) stage_slice<R, false>(xs, Q.ulist + u0, nu, Q.x, Q.ldx, nullptr);
        __syncthreads();
        slice_part<ST, R, EPI, W, kWaves>(P, Q.col16, q0, q1, wid, lane, dl, s_tab, fpart, cpart, xs);
    }
    workgroup_partials_n<R, EPI, kWaves>(P, lane, wid, fpart, cpart);
}

// Largest LDS slice a launch uses; with the objective table (4 KB) and the
// partial sums the workgroup stays within 64 KB.
constexpr size_t kPanelLdsBytes = 56 * 1024;

template <int ST, int R, int EPI>
static void launch_slice_chunk(int W, int nwg, size_t lds, const SpmvParams& P, const PanelParams& Q, hipStream_t s) {
    dim3 grid(nwg), block(kPanelThreads);
    if (W == 16) hipLaunchKernelGGL((spmv_slice_kernel<ST, R, EPI, 16>), grid, block, lds, s, P, Q);
    else if (W == 8) hipLaunchKernelGGL((spmv_slice_kernel<ST, R, EPI, 8>), grid, block, lds, s, P, Q);
    else hipLaunchKernelGGL((spmv_slice_kernel<ST, R, EPI, 4>), grid, block, lds, s, P, Q);
}

template <int ST, int R, int EPI>
static void launch_chunk(int B, int nwg, size_t lds, const SpmvParams& P, const PanelParams& Q, hipStream_t s) {
    dim3 grid(nwg), block(kPanelThreads);
    if (B < 0) launch_slice_chunk<ST, R, EPI>(-B, nwg, lds, P, Q, s);
    else if (B == 4) hipLaunchKernelGGL((spmv_panel_kernel<ST, R, EPI, 4>), grid, block, lds, s, P, Q);
    else if (B == 2) hipLaunchKernelGGL((spmv_panel_kernel<ST, R, EPI, 2>), grid, block, lds, s, P, Q);
    else hipLaunchKernelGGL((spmv_panel_kernel<ST, R, EPI, 1>), grid, block, lds, s, P, Q);
}

template <int ST, int EPI>
static void launch_chunk_r(int R, int B, int nwg, size_t lds, const SpmvParams& P, const PanelParams& Q,
                           hipStream_t s) {
    if constexpr (EPI == EPI_CURV) {
        launch_chunk<ST, 1, EPI>(B, nwg, lds, P, Q, s);
    } else {
        if (R == 8) launch_chunk<ST, 8, EPI>(B, nwg, lds, P, Q, s);
        else if (R == 4) launch_chunk<ST, 4, EPI>(B, nwg, lds, P, Q, s);
        else if (R == 2) launch_chunk<ST, 2, EPI>(B, nwg, lds, P, Q, s);
        else launch_chunk<ST, 1, EPI>(B, nwg, lds, P, Q, s);
    }
}

template <int EPI>
dvmat_status launch_panel(const KernelCfg& cfg, int storage, const CsrDev& c, const SpmvParams& P0, const float* x,
                          int nrhs, hipStream_t s, int* nwg_out, bool xcd_runs) {
    const int64_t want = std::max(1, cfg.workgroups);
    // XCD-contiguous parts need a grid of whole XCD rounds
    const int nwg = xcd_runs ? (int)std::max<int64_t>(kNumXcd, std::min<int64_t>(want, c.n_parts) / kNumXcd * kNumXcd)
                             : (int)std::max<int64_t>(1, std::min<int64_t>(want, c.n_parts));
    *nwg_out = nwg;
    if (c.n_parts == 0) return DVMAT_OK;
    const size_t per_rhs = (size_t)std::max<int64_t>(c.max_panel_cols, 1) * sizeof(float);
    if (per_rhs > kPanelLdsBytes)
        return set_error(DVMAT_E_SHAPE, "panel of %lld columns exceeds the LDS slice", (long long)c.max_panel_cols);
    PanelParams Q{};
    Q.ldx = nrhs;
    Q.col16 = c.col16;
    Q.ulist = c.ulist;
    Q.panel_u = c.panel_u;
    Q.part_units = c.part_units;
    Q.part_panel = c.part_panel;
    Q.n_parts = c.n_parts;
    Q.xcd_runs = xcd_runs ? 1 : 0;
    for (int h0 = 0; h0 < nrhs;) {
        int R = 8;
        while (R > 1 && (R > nrhs - h0 || per_rhs * R > kPanelLdsBytes)) R >>= 1;
        SpmvParams P = P0;
        P.ld = nrhs;
        if (P.y) P.y += h0;
        if (P.g) P.g += h0;
        if (P.partial) P.partial += h0;
        Q.x = x + h0;
        const size_t lds = per_rhs * R;
        // sliced panels pass their lanes per row as a negative block-row count
        const int Bk = c.layout == 2 ? -c.slice_lanes : c.B;
        if (storage == DVMAT_F32) launch_chunk_r<DVMAT_F32, EPI>(R, Bk, nwg, lds, P, Q, s);
        else if (storage == DVMAT_F16) launch_chunk_r<DVMAT_F16, EPI>(R, Bk, nwg, lds, P, Q, s);
        else launch_chunk_r<DVMAT_BF16, EPI>(R, Bk, nwg, lds, P, Q, s);
        h0 += R;
    }
    return check_hip(hipGetLastError(), "panel launch");
}

// ---- batched launch over many plans in the panel layout -------------------
//
// The parts of all plans form one work list; a workgroup's cursor over the
// plans only moves forward.  The dose of 16-bit storage multiplies the staged
// slice by the per-beamlet scale (the values hold D_ij / s_j).  Several
// right-hand sides make the slice large (4 right-hand sides of a 3,584-column
// panel: 56 KB), so the workgroup has sixteen waves: two workgroups fill a
// CU's 32 wave slots within its 160 KB of LDS (with eight waves they filled
// half; the batched dose ran 11 % slower).  Slices of all 8 right-hand sides
// in one pass (112 KB, one workgroup per CU) timed the same as two passes.
constexpr int kBatchPanelThreads = 1024;
constexpr size_t kBatchLdsBytes = 64 * 1024;

template <int ST, int R, int EPI, int B, bool SCALE_STAGE>
__global__ __launch_bounds__(kBatchPanelThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void spmv_batch_panel_kernel(
    BatchParams Bp, int h0, int nrhs) {
    constexpr int kWaves = kBatchPanelThreads / kWaveSize;
    static_assert(EPI == EPI_PLAIN || EPI == EPI_SCALE, "the batched launch has no objective epilogue");
    extern __shared__ float xs[];
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    float fpart[R];
#pragma unroll
    for (int h = 0; h < R; ++h) fpart[h] = 0.0f;
    double cpart = 0.0;
    int p = 0;
    for (int64_t t = blockIdx.x; t < Bp.total_blocks; t += gridDim.x) {
        while (p + 1 < Bp.n_plans && Bp.plans[p + 1].block_base <= t) ++p;      // t only grows
        const PlanDev& pd = Bp.plans[p];
        const int64_t tl = t - pd.block_base;
        const int pan = pd.part_panel[tl];
        const int64_t u0 = pd.panel_u[pan];
        const int nu = (int)(pd.panel_u[pan + 1] - u0);
        const float* x = Bp.x[p];
        __syncthreads();                              // the previous part's gathers are done
        stage_slice<R, SCALE_STAGE, kBatchPanelThreads>(xs, pd.ulist + u0, nu, x + h0, nrhs, pd.scale);
        __syncthreads();
        SpmvParams P{};
        P.n_rows = pd.n_rows;
        P.perm = pd.perm;
        P.perm_runs = pd.perm_runs;
        P.rowptr = pd.rowptr;
        P.val = pd.val;
        P.blocks = pd.blocks;
        P.y = Bp.y[p] + h0;
        P.ld = nrhs;
        P.row_scale = pd.scale;
        const int q0 = pd.part_units[tl], q1 = pd.part_units[tl + 1];
        for (int q = q0 + wid; q < q1; q += kWaves)
            block_rows<ST, R, EPI, false, B, true>(P, P.blocks[q], P.blocks[q + 1], lane, nullptr, fpart, cpart, xs,
                                                   pd.col16);
    }
}

// The batched launch over plans in the sliced panel layout: the same part
// walk, each part's slices as in spmv_slice_kernel (sixteen waves).
template <int ST, int R, int EPI, int W, bool SCALE_STAGE>
__global__ __launch_bounds__(kBatchPanelThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void spmv_batch_slice_kernel(
    BatchParams Bp, int h0, int nrhs) {
    constexpr int kWaves = kBatchPanelThreads / kWaveSize;
    static_assert(EPI == EPI_PLAIN || EPI == EPI_SCALE, "the batched launch has no objective epilogue");
    extern __shared__ float xs[];
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    float fpart[R];
#pragma unroll
    for (int h = 0; h < R; ++h) fpart[h] = 0.0f;
    double cpart = 0.0;
    int p = 0;
    for (int64_t t = blockIdx.x; t < Bp.total_blocks; t += gridDim.x) {
        while (p + 1 < Bp.n_plans && Bp.plans[p + 1].block_base <= t) ++p;      // t only grows
        const PlanDev& pd = Bp.plans[p];
        const int64_t tl = t - pd.block_base;
        const int pan = pd.part_panel[tl];
        const int64_t u0 = pd.panel_u[pan];
        const int nu = (int)(pd.panel_u[pan + 1] - u0);
        SpmvParams P{};
        P.n_rows = pd.n_rows;
        P.perm = pd.perm;
        P.rowptr = pd.rowptr;
        P.val = pd.val;
        P.blocks = pd.blocks;
        P.y = Bp.y[p] + h0;
        P.ld = nrhs;
        P.row_scale = pd.scale;
        const int q0 = pd.part_units[tl], q1 = pd.part_units[tl + 1];
        __syncthreads();                              // the previous part's gathers are done
        const SliceLanes dl = slice_lanes<kWaves>(P, q0, q1, wid, lane, 0);
        if (P.rowptr[q1] > P.rowptr[q0])
            stage_slice<R, SCALE_STAGE, kBatchPanelThreads>(xs, pd.ulist + u0, nu, Bp.x[p] + h0, nrhs, pd.scale);
        __syncthreads();
        slice_part<ST, R, EPI, W, kWaves>(P, pd.col16, q0, q1, wid, lane, dl, nullptr, fpart, cpart, xs);
    }
}

template <int ST, int R, int EPI, int B, bool SCALE_STAGE>
static void launch_batch_one(int nwg, size_t lds, const BatchParams& Bp, int h0, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL((spmv_batch_panel_kernel<ST, R, EPI, B, SCALE_STAGE>), dim3(nwg), dim3(kBatchPanelThreads),
                       lds, s, Bp, h0, nrhs);
}

template <int ST, int R, int EPI, int W, bool SCALE_STAGE>
static void launch_batch_slice(int nwg, size_t lds, const BatchParams& Bp, int h0, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL((spmv_batch_slice_kernel<ST, R, EPI, W, SCALE_STAGE>), dim3(nwg), dim3(kBatchPanelThreads),
                       lds, s, Bp, h0, nrhs);
}

// B > 0: rows per block row of the panel layout; B < 0: -B lanes per row of
// the sliced layout.
template <int ST, int R, int EPI, bool SCALE_STAGE>
static void launch_batch_chunk(int B, int nwg, size_t lds, const BatchParams& Bp, int h0, int nrhs, hipStream_t s) {
    if (B == -16) launch_batch_slice<ST, R, EPI, 16, SCALE_STAGE>(nwg, lds, Bp, h0, nrhs, s);
    else if (B == -8) launch_batch_slice<ST, R, EPI, 8, SCALE_STAGE>(nwg, lds, Bp, h0, nrhs, s);
    else if (B < 0) launch_batch_slice<ST, R, EPI, 4, SCALE_STAGE>(nwg, lds, Bp, h0, nrhs, s);
    else if (B == 4) launch_batch_one<ST, R, EPI, 4, SCALE_STAGE>(nwg, lds, Bp, h0, nrhs, s);
    else if (B == 2) launch_batch_one<ST, R, EPI, 2, SCALE_STAGE>(nwg, lds, Bp, h0, nrhs, s);
    else launch_batch_one<ST, R, EPI, 1, SCALE_STAGE>(nwg, lds, Bp, h0, nrhs, s);
}

template <int ST, int EPI, bool SCALE_STAGE>
static void launch_batch_r(int R, int B, int nwg, size_t lds, const BatchParams& Bp, int h0, int nrhs, hipStream_t s) {
    if (R == 8) launch_batch_chunk<ST, 8, EPI, SCALE_STAGE>(B, nwg, lds, Bp, h0, nrhs, s);
    else if (R == 4) launch_batch_chunk<ST, 4, EPI, SCALE_STAGE>(B, nwg, lds, Bp, h0, nrhs, s);
    else if (R == 2) launch_batch_chunk<ST, 2, EPI, SCALE_STAGE>(B, nwg, lds, Bp, h0, nrhs, s);
    else launch_batch_chunk<ST, 1, EPI, SCALE_STAGE>(B, nwg, lds, Bp, h0, nrhs, s);
}

dvmat_status launch_batch_panel(int storage, int B, int epi_scale, bool scale_stage, int64_t max_panel_cols,
                                const BatchParams& Bp, int nrhs, int workgroups, hipStream_t s) {
    const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>(std::max(1, workgroups), Bp.total_blocks));
    if (Bp.total_blocks == 0) return DVMAT_OK;
    const size_t per_rhs = (size_t)std::max<int64_t>(max_panel_cols, 1) * sizeof(float);
    if (per_rhs > kBatchLdsBytes)
        return set_error(DVMAT_E_SHAPE, "panel of %lld columns exceeds the LDS slice", (long long)max_panel_cols);
    for (int h0 = 0; h0 < nrhs;) {
        int R = 8;
        while (R > 1 && (R > nrhs - h0 || per_rhs * R > kBatchLdsBytes)) R >>= 1;
        const size_t lds = per_rhs * R;
#define DVMAT_BATCH_ST(STT)                                                                          \
        if (epi_scale) launch_batch_r<STT, EPI_SCALE, false>(R, B, nwg, lds, Bp, h0, nrhs, s);       \
        else if (scale_stage) launch_batch_r<STT, EPI_PLAIN, true>(R, B, nwg, lds, Bp, h0, nrhs, s); \
        else launch_batch_r<STT, EPI_PLAIN, false>(R, B, nwg, lds, Bp, h0, nrhs, s);
        if (storage == DVMAT_F32) {
            launch_batch_r<DVMAT_F32, EPI_PLAIN, false>(R, B, nwg, lds, Bp, h0, nrhs, s);
        } else if (storage == DVMAT_F16) {
            DVMAT_BATCH_ST(DVMAT_F16)
        } else {
            DVMAT_BATCH_ST(DVMAT_BF16)
        }
#undef DVMAT_BATCH_ST
        h0 += R;
    }
    return check_hip(hipGetLastError(), "batched panel launch");
}

template dvmat_status launch_panel<EPI_PLAIN>(const KernelCfg&, int, const CsrDev&, const SpmvParams&, const float*,
                                              int, hipStream_t, int*, bool);
template dvmat_status launch_panel<EPI_OBJ>(const KernelCfg&, int, const CsrDev&, const SpmvParams&, const float*, int,
                                            hipStream_t, int*, bool);
template dvmat_status launch_panel<EPI_CURV>(const KernelCfg&, int, const CsrDev&, const SpmvParams&, const float*,
                                             int, hipStream_t, int*, bool);
template dvmat_status launch_panel<EPI_SCALE>(const KernelCfg&, int, const CsrDev&, const SpmvParams&, const float*,
                                              int, hipStream_t, int*, bool);

}  // namespace dvmat
