// Dose z = D x and price p = D^T g on gfx950, plus the objective epilogue.
//
// Both products are CSR row-times-vector kernels over the orientation that
// makes the output a row: CSR(D) for the dose (rows = voxels, the "step 4"
// dose update of Sec. 2.2.2 and Eq. 5 for aperture indicators) and CSR(D^T)
// for the price (rows = beamlets, Eq. 3; the paper's GPU kernel assigns one
// warp per beamlet row, Sec. 2.2.2).  The path is HBM-bound (2 flop per 8
// bytes of matrix at FP32), so no matrix cores are used.
//
// Mapping: rows are grouped on the host into blocks of consecutive rows with
// a bounded number of stored entries.  One wave64 walks one block, one row at
// a time: each lane streams 4 consecutive entries (16-byte value and column
// loads, non-temporal so the matrix stream does not evict the gathered
// vector from L2), gathers x[col], accumulates in FP32; a fixed butterfly
// reduces the wave, lane 0 applies the epilogue.  The grid is a multiple of
// the 8 XCDs; workgroup w runs on XCD w % 8 and each XCD owns a contiguous
// range of blocks, so the waves sharing one L2 touch neighbouring rows.
// Every reduction has a fixed order: results are bitwise reproducible.
#include "common.hpp"

#include <cmath>
#include <cstdlib>

namespace dvmat {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

enum Epi { EPI_PLAIN = 0, EPI_OBJ = 1, EPI_CURV = 2, EPI_SCALE = 3 };

struct SpmvParams {
    const int64_t* rowptr;
    const int32_t* col;
    const void* val;
    const int32_t* blocks;
    int64_t n_blocks;
    const float* x;
    float* y;              // output rows (nullable for EPI_CURV)
    const uint8_t* sid;    // objective epilogue
    const float* table;
    float* g;
    float* partial;
    double* partial_d;
    const float* zref;
    const float* row_scale;  // EPI_SCALE
};

template <int ST>
__device__ __forceinline__ f32x4 load_vals(const void* base, int64_t k) {
    if constexpr (ST == DVMAT_F32) {
        return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(base) + (k >> 2));
    } else if constexpr (ST == DVMAT_F16) {
        f16x4 h = __builtin_nontemporal_load(reinterpret_cast<const f16x4*>(base) + (k >> 2));
        return __builtin_convertvector(h, f32x4);
    } else {
        u16x4 b = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(base) + (k >> 2));
        f32x4 r;
        r.x = __uint_as_float((unsigned)b.x << 16);
        r.y = __uint_as_float((unsigned)b.y << 16);
        r.z = __uint_as_float((unsigned)b.z << 16);
        r.w = __uint_as_float((unsigned)b.w << 16);
        return r;
    }
}

__device__ __forceinline__ i32x4 load_cols(const int32_t* col, int64_t k) {
    return __builtin_nontemporal_load(reinterpret_cast<const i32x4*>(col) + (k >> 2));
}

template <int NRHS>
__device__ __forceinline__ void fma_gather(float (&acc)[NRHS], const float* __restrict__ x, float v, int c) {
    if constexpr (NRHS == 8) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(x + (int64_t)c * 8);
        const f32x4 b = *reinterpret_cast<const f32x4*>(x + (int64_t)c * 8 + 4);
        acc[0] += v * a.x; acc[1] += v * a.y; acc[2] += v * a.z; acc[3] += v * a.w;
        acc[4] += v * b.x; acc[5] += v * b.y; acc[6] += v * b.z; acc[7] += v * b.w;
    } else if constexpr (NRHS == 4) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(x + (int64_t)c * 4);
        acc[0] += v * a.x; acc[1] += v * a.y; acc[2] += v * a.z; acc[3] += v * a.w;
    } else {
#pragma unroll
        for (int h = 0; h < NRHS; ++h) acc[h] += v * x[(int64_t)c * NRHS + h];
    }
}

template <int NRHS>
__device__ __forceinline__ void fma4(float (&acc)[NRHS], const float* __restrict__ x, f32x4 v, i32x4 c) {
    fma_gather<NRHS>(acc, x, v.x, c.x);
    fma_gather<NRHS>(acc, x, v.y, c.y);
    fma_gather<NRHS>(acc, x, v.z, c.z);
    fma_gather<NRHS>(acc, x, v.w, c.w);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int ST, int NRHS, int EPI>
__global__ __launch_bounds__(kSpmvThreads) void spmv_kernel(SpmvParams P) {
    constexpr int kWaves = kSpmvThreads / kWaveSize;
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    const int wg = blockIdx.x;
    const int xcd = wg % kNumXcd;
    const int li = wg / kNumXcd;
    const int waves_per_xcd = (gridDim.x / kNumXcd) * kWaves;
    const int lw = li * kWaves + wid;
    const int64_t b0 = P.n_blocks * xcd / kNumXcd;
    const int64_t b1 = P.n_blocks * (xcd + 1) / kNumXcd;

    float fpart[NRHS];
#pragma unroll
    for (int h = 0; h < NRHS; ++h) fpart[h] = 0.0f;
    double cpart = 0.0;

    for (int64_t b = b0 + lw; b < b1; b += waves_per_xcd) {
        const int r0 = P.blocks[b];
        const int r1 = P.blocks[b + 1];
        for (int r = r0; r < r1; ++r) {
            const int64_t e0 = P.rowptr[r];
            const int64_t e1 = P.rowptr[r + 1];
            float acc[NRHS];
#pragma unroll
            for (int h = 0; h < NRHS; ++h) acc[h] = 0.0f;
            int64_t k = e0 + lane * 4;
            for (; k + 256 < e1; k += 512) {
                const f32x4 v0 = load_vals<ST>(P.val, k);
                const i32x4 c0 = load_cols(P.col, k);
                const f32x4 v1 = load_vals<ST>(P.val, k + 256);
                const i32x4 c1 = load_cols(P.col, k + 256);
                fma4<NRHS>(acc, P.x, v0, c0);
                fma4<NRHS>(acc, P.x, v1, c1);
            }
            if (k < e1) {
                const f32x4 v0 = load_vals<ST>(P.val, k);
                const i32x4 c0 = load_cols(P.col, k);
                fma4<NRHS>(acc, P.x, v0, c0);
            }
#pragma unroll
            for (int h = 0; h < NRHS; ++h) acc[h] = wave_sum(acc[h]);
            if (lane == 0) {
                if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
                    for (int h = 0; h < NRHS; ++h) P.y[(int64_t)r * NRHS + h] = acc[h];
                } else if constexpr (EPI == EPI_SCALE) {
                    const float s = P.row_scale[r];
#pragma unroll
                    for (int h = 0; h < NRHS; ++h) P.y[(int64_t)r * NRHS + h] = acc[h] * s;
                } else if constexpr (EPI == EPI_OBJ) {
                    const int s = P.sid[r];
                    const float T = P.table[s * 4 + 0];
                    const float wo = P.table[s * 4 + 1];
                    const float wu = P.table[s * 4 + 2];
#pragma unroll
                    for (int h = 0; h < NRHS; ++h) {
                        const float z = acc[h];
                        P.y[(int64_t)r * NRHS + h] = z;
                        const float over = fmaxf(z - T, 0.0f);
                        const float under = fmaxf(T - z, 0.0f);
                        if (P.g) P.g[(int64_t)r * NRHS + h] = 2.0f * wo * over - 2.0f * wu * under;
                        fpart[h] += wo * over * over + wu * under * under;
                    }
                } else {  // EPI_CURV
                    const float d = acc[0];
                    if (P.y) P.y[r] = d;
                    const int s = P.sid[r];
                    const float T = P.table[s * 4 + 0];
                    const float zr = P.zref[r];
                    const float w = zr > T ? P.table[s * 4 + 1] : (zr < T ? P.table[s * 4 + 2] : 0.0f);
                    cpart += (double)w * (double)d * (double)d;
                }
            }
        }
    }
    if constexpr (EPI == EPI_OBJ || EPI == EPI_CURV) {
        __shared__ float sp[kWaves][NRHS];
        __shared__ double sd[kWaves];
        if (lane == 0) {
#pragma unroll
            for (int h = 0; h < NRHS; ++h) sp[wid][h] = fpart[h];
            sd[wid] = cpart;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if constexpr (EPI == EPI_OBJ) {
#pragma unroll
                for (int h = 0; h < NRHS; ++h) {
                    float s = 0.0f;
                    for (int w = 0; w < kWaves; ++w) s += sp[w][h];
                    P.partial[(int64_t)wg * NRHS + h] = s;
                }
            } else {
                double s = 0.0;
                for (int w = 0; w < kWaves; ++w) s += sd[w];
                P.partial_d[wg] = s;
            }
        }
    }
}

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

static int spmv_workgroups(int64_t n_blocks) {
    int want = 2048;
    if (const char* s = std::getenv("DVMAT_SPMV_WG")) want = std::atoi(s);
    int64_t need = (n_blocks + 3) / 4;
    int64_t w = std::min<int64_t>(want, need);
    w = (w + kNumXcd - 1) / kNumXcd * kNumXcd;
    w = std::max<int64_t>(kNumXcd, std::min<int64_t>(w, kMaxSpmvWorkgroups));
    return (int)w;
}

template <int ST, int EPI>
static void launch_st(const SpmvParams& P, int nrhs, int nwg, hipStream_t s) {
    dim3 grid(nwg), block(kSpmvThreads);
    switch (nrhs) {
#define DVMAT_CASE(N) \
    case N: hipLaunchKernelGGL((spmv_kernel<ST, N, EPI>), grid, block, 0, s, P); break;
        DVMAT_CASE(1) DVMAT_CASE(2) DVMAT_CASE(3) DVMAT_CASE(4)
        DVMAT_CASE(5) DVMAT_CASE(6) DVMAT_CASE(7) DVMAT_CASE(8)
#undef DVMAT_CASE
        default: break;
    }
}

template <int EPI>
static void launch_spmv(int storage, const SpmvParams& P, int nrhs, int nwg, hipStream_t s) {
    if (storage == DVMAT_F32) launch_st<DVMAT_F32, EPI>(P, nrhs, nwg, s);
    else if (storage == DVMAT_F16) launch_st<DVMAT_F16, EPI>(P, nrhs, nwg, s);
    else launch_st<DVMAT_BF16, EPI>(P, nrhs, nwg, s);
}

// Curvature only needs one right-hand side.
template <int EPI>
static void launch_spmv1(int storage, const SpmvParams& P, int nwg, hipStream_t s) {
    dim3 grid(nwg), block(kSpmvThreads);
    if (storage == DVMAT_F32) hipLaunchKernelGGL((spmv_kernel<DVMAT_F32, 1, EPI>), grid, block, 0, s, P);
    else if (storage == DVMAT_F16) hipLaunchKernelGGL((spmv_kernel<DVMAT_F16, 1, EPI>), grid, block, 0, s, P);
    else hipLaunchKernelGGL((spmv_kernel<DVMAT_BF16, 1, EPI>), grid, block, 0, s, P);
}

static int elementwise_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 2048));
}

dvmat_status launch_expand_scale(const dvmat_ddc_s* d, const float* x, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(scale_x_kernel, dim3(elementwise_grid(d->n_bl * nrhs)), dim3(256), 0, s, x, d->scale,
                       d->n_bl, nrhs, d->xs);
    return check_hip(hipGetLastError(), "scale_x_kernel launch");
}

static dvmat_status check_ddc(const dvmat_ddc_s* d, const char* fn) {
    if (!d) return set_error(DVMAT_E_ARG, "%s: ddc is NULL", fn);
    if (!d->bound) return set_error(DVMAT_E_STATE, "%s: ddc not bound to a device workspace", fn);
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
    // padded 4-wide table; unused rows are zero (no objective)
    static thread_local float host_tab[256 * 4];
    for (int i = 0; i < 256 * 4; ++i) host_tab[i] = 0.0f;
    for (int s = 0; s < n_struct; ++s)
        for (int c = 0; c < 3; ++c) host_tab[s * 4 + c] = table[s * 3 + c];
    hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    st = check_hip(hipMemcpyAsync(o->table, host_tab, sizeof host_tab, hipMemcpyHostToDevice, hs),
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
    const float* xin = x;
    if (d->storage != DVMAT_F32) {
        if ((st = launch_expand_scale(d, x, nrhs, s))) return st;
        xin = d->xs;
    }
    SpmvParams P{};
    P.rowptr = d->dose.rowptr;
    P.col = d->dose.col;
    P.val = d->dose.val;
    P.blocks = d->dose.blocks;
    P.n_blocks = d->dose.n_blocks;
    P.x = xin;
    P.y = z;
    const int nwg = spmv_workgroups(d->dose.n_blocks);
    if (obj) {
        P.sid = obj->sid;
        P.table = obj->table;
        P.g = g;
        P.partial = obj->partial;
        launch_spmv<EPI_OBJ>(d->storage, P, nrhs, nwg, s);
        if (F) hipLaunchKernelGGL(finalize_f_kernel, dim3(1), dim3(256), 0, s, obj->partial, nwg, nrhs, F);
    } else {
        launch_spmv<EPI_PLAIN>(d->storage, P, nrhs, nwg, s);
    }
    return check_hip(hipGetLastError(), "dvmat_dose launch");
}

dvmat_status dvmat_price(dvmat_ddc d, const float* g, int32_t nrhs, float* p, dvmat_stream stream) {
    dvmat_status st = check_ddc(d, "dvmat_price");
    if (st) return st;
    if (!g || !p) return set_error(DVMAT_E_ARG, "dvmat_price: g and p must be non-NULL");
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error(DVMAT_E_ARG, "dvmat_price: nrhs=%d not in 1..8", nrhs);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    SpmvParams P{};
    P.rowptr = d->price.rowptr;
    P.col = d->price.col;
    P.val = d->price.val;
    P.blocks = d->price.blocks;
    P.n_blocks = d->price.n_blocks;
    P.x = g;
    P.y = p;
    P.row_scale = d->scale;
    const int nwg = spmv_workgroups(d->price.n_blocks);
    if (d->storage == DVMAT_F32) launch_spmv<EPI_PLAIN>(d->storage, P, nrhs, nwg, s);
    else launch_spmv<EPI_SCALE>(d->storage, P, nrhs, nwg, s);
    return check_hip(hipGetLastError(), "dvmat_price launch");
}

dvmat_status dvmat_dose_curvature(dvmat_ddc d, const float* x_dir, dvmat_obj obj, const float* z_ref, float* d_out,
                                  double* curv, dvmat_stream stream) {
    dvmat_status st = check_ddc(d, "dvmat_dose_curvature");
    if (st) return st;
    if (!x_dir || !obj || !z_ref || !curv) return set_error(DVMAT_E_ARG, "dvmat_dose_curvature: NULL argument");
    if (obj->n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_dose_curvature: voxel count mismatch");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float* xin = x_dir;
    if (d->storage != DVMAT_F32) {
        if ((st = launch_expand_scale(d, x_dir, 1, s))) return st;
        xin = d->xs;
    }
    SpmvParams P{};
    P.rowptr = d->dose.rowptr;
    P.col = d->dose.col;
    P.val = d->dose.val;
    P.blocks = d->dose.blocks;
    P.n_blocks = d->dose.n_blocks;
    P.x = xin;
    P.y = d_out;
    P.sid = obj->sid;
    P.table = obj->table;
    P.zref = z_ref;
    P.partial_d = obj->partial_d;
    const int nwg = spmv_workgroups(d->dose.n_blocks);
    launch_spmv1<EPI_CURV>(d->storage, P, nwg, s);
    hipLaunchKernelGGL(finalize_d_kernel, dim3(1), dim3(256), 0, s, obj->partial_d, nwg, curv);
    return check_hip(hipGetLastError(), "dvmat_dose_curvature launch");
}

}  // extern "C"
