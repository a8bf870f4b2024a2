// DA-form master problem (Eq. 6 as the paper writes it).
//
// The paper solves the master problem on the aperture DDC vectors
// DA(A_k) = sum_{j in A_k} D_:j (Eq. 5), computed once per chosen aperture,
// with z = sum_k DA_k y_k and the gradient in the aperture domain
// G_k = <DA_k, dF/dz> (Sec. 2.1, Sec. 2.2.2).  Here each DA_k is a dense
// device column of n_vox floats, produced by one dose product of the
// aperture's indicator fluence; a BB iteration then reads the m columns
// instead of the whole matrix twice.
//
// dvmat_da_eval is one pass over the columns: a workgroup owns a contiguous
// chunk of voxels, forms z and dF/dz for it (columns streamed from HBM), keeps
// dF/dz in registers, then re-reads its chunk of every column (now in L2) to
// form its share of each G_k (wave sums, no barrier per column);
// per-workgroup shares are summed in a fixed order.
// The column count is kept on the device too and the kernels read it there
// (grids do not depend on it), so a captured graph of a solve replays as
// columns are appended.
//
// Optionally (dvmat_da_set_support) the columns keep only the rows of the
// objective's support, the voxels whose structure carries a weight: F and G
// depend on nothing else (dF/dz is zero elsewhere), and outside the body,
// over half of the full-scale cube, every column would hold zeros.
#include "bb_device.hpp"

#include <algorithm>
#include <cmath>
#include <new>

namespace dvmat {

// Eight voxels per thread, 2048 per workgroup, columns loaded four at a time:
// 32 loads in flight per thread, and half the workgroups (and shares to sum)
// of four voxels per thread (the DA-form iteration 2.8 ms against 3.45 with
// four voxels and eight columns, 5.0 with two voxels and sixteen columns).
constexpr int kDaThreads = 256;
constexpr int kDaWaves = kDaThreads / 64;
constexpr int kDaPerThread = 8;
constexpr int kDaChunk = kDaThreads * kDaPerThread;   // voxels per workgroup
constexpr int kDaGroup = 4;                            // columns whose loads go out together
constexpr int kDaFanIn = 16;                           // chunk shares per group sum
static_assert(kDaWaves == 4, "the share sums combine four waves");

}  // namespace dvmat

struct dvmat_da_s {
    int64_t n_vox = 0;
    int64_t n_rows = 0;          // rows per column: n_vox, or the support's size
    const int32_t* rows = nullptr;   // voxel of each row (support), or nullptr (identity)
    const uint8_t* row_sid = nullptr;  // structure id of each row when restricted
    int32_t* support = nullptr;  // [n_vox] workspace for the support's voxel list
    uint8_t* csid = nullptr;     // [n_vox] workspace for its structure ids
    int32_t* d_nsup = nullptr;   // device count of the support
    int32_t max_ap = 0;
    int32_t m = 0;
    int32_t n_chunks = 0;
    float* cols = nullptr;       // [max_ap][n_rows]
    float* partial = nullptr;    // [max_ap + 1][n_chunks]: G shares, then F shares
    double* gpart = nullptr;     // [max_ap + 1][n_groups]: group sums of the shares
    double* partial_d = nullptr; // [n_chunks]
    float* gbuf = nullptr;       // [n_vox] dF/dz when the caller does not keep it
    int32_t* d_m = nullptr;      // device copy of m, set by dvmat_da_append
    uint32_t* arrived = nullptr; // [n_groups + 1]: workgroups of each group done, then groups done
                                 // (0 between launches)
};

namespace dvmat {

static size_t da_layout(int64_t n_vox, int32_t max_ap, dvmat_da_s* d, char* base) {
    const int64_t chunks = (n_vox + kDaChunk - 1) / kDaChunk;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return base ? base + o : nullptr; };
    char* p;
    p = take((size_t)max_ap * n_vox * 4);           if (d) d->cols = reinterpret_cast<float*>(p);
    const int64_t groups = (chunks + kDaFanIn - 1) / kDaFanIn;
    p = take((size_t)(max_ap + 1) * chunks * 4);    if (d) d->partial = reinterpret_cast<float*>(p);
    p = take((size_t)(max_ap + 1) * groups * 8);    if (d) d->gpart = reinterpret_cast<double*>(p);
    p = take((size_t)chunks * 8);                   if (d) d->partial_d = reinterpret_cast<double*>(p);
    p = take((size_t)n_vox * 4);                    if (d) d->gbuf = reinterpret_cast<float*>(p);
    p = take(sizeof(int32_t));                      if (d) d->d_m = reinterpret_cast<int32_t*>(p);
    p = take((size_t)(groups + 1) * sizeof(uint32_t)); if (d) d->arrived = reinterpret_cast<uint32_t*>(p);
    p = take((size_t)n_vox * 4);                    if (d) d->support = reinterpret_cast<int32_t*>(p);
    p = take((size_t)n_vox);                        if (d) d->csid = reinterpret_cast<uint8_t*>(p);
    p = take(sizeof(int32_t));                      if (d) d->d_nsup = reinterpret_cast<int32_t*>(p);
    if (d) d->n_chunks = (int32_t)chunks;
    return off;
}

// Sum over the 64 lanes of a wave in a fixed order, returned to every lane.
template <typename T>
__device__ __forceinline__ T wave_sum64(T v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Dynamic LDS of the evaluation kernels: the rates (max_ap floats) and the
// per-wave shares of every G_k and of F (kDaWaves x (max_ap + 1) floats).
static size_t da_lds_bytes(int max_ap) { return ((size_t)max_ap + (size_t)kDaWaves * (max_ap + 1)) * sizeof(float); }

__global__ void da_set_count_kernel(int32_t* d_m, int m, uint32_t* arrived, int n_counters) {
    if (threadIdx.x == 0) *d_m = m;
    for (int i = threadIdx.x; i < n_counters; i += blockDim.x) arrived[i] = 0u;
}

// One workgroup's chunk of the evaluation: z and dF/dz of its voxels (stored
// where z, g are given), its shares of every G_k and of F into partial.
// Rows are positions in the columns (n_rows of them); rows != nullptr maps a
// row to its voxel for the stored z and dF/dz; rsid is the structure id of
// each row.
__device__ __forceinline__ void da_eval_chunk(const float* __restrict__ cols, int64_t n_rows, int m, int max_ap,
                                              const float* __restrict__ y, const uint8_t* __restrict__ rsid,
                                              const int32_t* __restrict__ rows,
                                              const float* __restrict__ table, float* __restrict__ z,
                                              float* __restrict__ g, float* __restrict__ partial, int n_chunks) {
    extern __shared__ float da_lds[];
    float* sy = da_lds;                       // [max_ap]
    float* wpart = da_lds + max_ap;           // [kDaWaves][max_ap + 1]
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kDaChunk;
    int64_t iv[kDaPerThread];
    bool in[kDaPerThread];
    float zi[kDaPerThread], gi[kDaPerThread];
    int sid[kDaPerThread];
#pragma unroll
    for (int u = 0; u < kDaPerThread; ++u) {
        iv[u] = c0 + u * kDaThreads + threadIdx.x;
        in[u] = iv[u] < n_rows;
        zi[u] = 0.0f;
    }
    // z_i = sum_k DA_k,i y_k in the order of k; the loads of kDaGroup columns
    // for all the thread's voxels are in flight together (a last, partial
    // group loads and adds only its columns below m).  The first group's
    // loads, the structure ids and the rates go out together, before the
    // barrier that publishes the rates in LDS.
    float c[kDaGroup][kDaPerThread];
    auto load_group = [&](int k) {
#pragma unroll
        for (int j = 0; j < kDaGroup; ++j)
#pragma unroll
            for (int u = 0; u < kDaPerThread; ++u)
                c[j][u] = (in[u] && k + j < m) ? cols[(int64_t)(k + j) * n_rows + iv[u]] : 0.0f;
    };
    load_group(0);
#pragma unroll
    for (int u = 0; u < kDaPerThread; ++u) sid[u] = in[u] ? (int)rsid[iv[u]] : 0;
    for (int k = threadIdx.x; k < m; k += kDaThreads) sy[k] = y[k];
    __syncthreads();
    for (int k = 0; k < m; k += kDaGroup) {
        if (k > 0) load_group(k);
#pragma unroll
        for (int j = 0; j < kDaGroup; ++j) {
            if (k + j < m) {
                const float yk = sy[k + j];
#pragma unroll
                for (int u = 0; u < kDaPerThread; ++u) zi[u] += c[j][u] * yk;
            }
        }
    }
    float fpart = 0.0f;
#pragma unroll
    for (int u = 0; u < kDaPerThread; ++u) {
        gi[u] = 0.0f;
        if (in[u]) {
            const int s = sid[u];
            const float T = table[s * 4 + 0], wo = table[s * 4 + 1], wu = table[s * 4 + 2];
            const float over = fmaxf(zi[u] - T, 0.0f), under = fmaxf(T - zi[u], 0.0f);
            gi[u] = 2.0f * wo * over - 2.0f * wu * under;
            fpart += wo * over * over + wu * under * under;
            const int64_t vox = rows ? (int64_t)rows[iv[u]] : iv[u];
            if (z) z[vox] = zi[u];
            if (g) g[vox] = gi[u];
        }
    }
    // G_k shares: this chunk of every column (just streamed, so in L2), summed
    // per wave, then over the waves in order; kDaGroup columns' loads at a time
    for (int k = 0; k < m; k += kDaGroup) {
        float c[kDaGroup][kDaPerThread];
#pragma unroll
        for (int j = 0; j < kDaGroup; ++j)
#pragma unroll
            for (int u = 0; u < kDaPerThread; ++u)
                c[j][u] = (in[u] && k + j < m) ? cols[(int64_t)(k + j) * n_rows + iv[u]] : 0.0f;
#pragma unroll
        for (int j = 0; j < kDaGroup; ++j) {
            if (k + j < m) {
                float a = 0.0f;
#pragma unroll
                for (int u = 0; u < kDaPerThread; ++u)
                    if (in[u]) a += c[j][u] * gi[u];
                a = wave_sum64(a);
                if (lane == 0) wpart[wid * (max_ap + 1) + k + j] = a;
            }
        }
    }
    fpart = wave_sum64(fpart);
    if (lane == 0) wpart[wid * (max_ap + 1) + m] = fpart;
    __syncthreads();
    for (int k = threadIdx.x; k <= m; k += kDaThreads) {
        float a = 0.0f;
#pragma unroll
        for (int w = 0; w < kDaWaves; ++w) a += wpart[w * (max_ap + 1) + k];
        partial[(int64_t)k * n_chunks + blockIdx.x] = a;
    }
}


// G[k] = sum of the chunk shares (k < m), F = sum of the F shares, in a fixed
// order, FP64, as a two-level tree: the chunks form groups of kDaFanIn; the
// last workgroup of a group to finish (a device-scope counter per group)
// sums the group's shares in chunk order into gpart, and the last group to
// finish (one more counter) sums the group sums in a fixed order into G and F.
// Every evaluation (the separate one and the fused step) runs this same
// tree, so their results agree bit for bit; each counter is reset by the
// workgroup it elects.

// Level 1: thread t takes share t % kDaFanIn of aperture t / kDaFanIn of the
// current pass (32 apertures per pass, two loads per thread).
__device__ __forceinline__ void da_group_sum(const float* __restrict__ partial, int m, int n_chunks, int grp,
                                             int n_groups, double* __restrict__ gpart) {
    __shared__ double s[2][kDaThreads];
    constexpr int kPer = kDaThreads / kDaFanIn;          // apertures per half pass
    const int c0 = grp * kDaFanIn;
    const int nc = min(kDaFanIn, n_chunks - c0);
    const int c = threadIdx.x % kDaFanIn, kk = threadIdx.x / kDaFanIn;
    for (int kb = 0; kb <= m; kb += 2 * kPer) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = kb + h * kPer + kk;
            s[h][threadIdx.x] = (k <= m && c < nc) ? (double)partial[(int64_t)k * n_chunks + c0 + c] : 0.0;
        }
        __syncthreads();
        if (c == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = kb + h * kPer + kk;
                if (k <= m) {
                    double a = 0.0;
                    for (int j = 0; j < nc; ++j) a += s[h][threadIdx.x + j];
                    gpart[(int64_t)k * n_groups + grp] = a;
                }
            }
        }
        __syncthreads();
    }
}

// Level 2: strand t / 32 of aperture t % 32 sums the groups congruent to it
// mod 8, in order; the eight strands are then added in order.
__device__ __forceinline__ void da_total_sum(const double* __restrict__ gpart, int m, int n_groups,
                                             float* __restrict__ G, float* __restrict__ F) {
    constexpr int kStrands = kDaThreads / 32;
    __shared__ double r[kStrands][32];
    const int kk = threadIdx.x % 32, st = threadIdx.x / 32;
    for (int kb = 0; kb <= m; kb += 32) {
        const int k = kb + kk;
        double a = 0.0;
        if (k <= m) {
#pragma unroll 8
            for (int gi = st; gi < n_groups; gi += kStrands) a += gpart[(int64_t)k * n_groups + gi];
        }
        r[st][kk] = a;
        __syncthreads();
        if (threadIdx.x < 32 && k <= m) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < kStrands; ++q) t += r[q][kk];
            if (k < m) G[k] = (float)t;
            else if (F) F[0] = (float)t;
        }
        __syncthreads();
    }
}

// After a workgroup's shares are stored: the group and total elections and
// the tree's sums.  Returns true in the one workgroup that wrote G and F.
__device__ __forceinline__ bool da_reduce_shares(const float* __restrict__ partial, double* __restrict__ gpart,
                                                 int m, int n_chunks, uint32_t* arrived, float* __restrict__ G,
                                                 float* __restrict__ F) {
    __shared__ int s_last;
    const int n_groups = (n_chunks + kDaFanIn - 1) / kDaFanIn;
    const int grp = (int)blockIdx.x / kDaFanIn;
    const uint32_t in_group = (uint32_t)min(kDaFanIn, n_chunks - grp * kDaFanIn);
    __syncthreads();                                   // every wave's shares are stored
    if (threadIdx.x == 0) {
        const uint32_t before = __hip_atomic_fetch_add(arrived + grp, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = before == in_group - 1;
    }
    __syncthreads();
    if (!s_last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) __hip_atomic_store(arrived + grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    da_group_sum(partial, m, n_chunks, grp, n_groups, gpart);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t before =
            __hip_atomic_fetch_add(arrived + n_groups, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = before == (uint32_t)n_groups - 1;
    }
    __syncthreads();
    if (!s_last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) __hip_atomic_store(arrived + n_groups, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    da_total_sum(gpart, m, n_groups, G, F);
    __syncthreads();
    return true;
}

__global__ __launch_bounds__(kDaThreads) void da_eval_kernel(const float* __restrict__ cols, int64_t n_rows,
                                                             const int32_t* __restrict__ d_m,
                                                             const float* __restrict__ y, const uint8_t* __restrict__ rsid,
                                                             const int32_t* __restrict__ rows,
                                                             const float* __restrict__ table, float* __restrict__ z,
                                                             float* __restrict__ g, float* __restrict__ partial,
                                                             double* __restrict__ gpart, int n_chunks, int max_ap,
                                                             uint32_t* arrived, float* __restrict__ G,
                                                             float* __restrict__ F) {
    const int m = *d_m;
    da_eval_chunk(cols, n_rows, m, max_ap, y, rsid, rows, table, z, g, partial, n_chunks);
    da_reduce_shares(partial, gpart, m, n_chunks, arrived, G, F);
}

// One BB iteration of the DA form in one launch: every workgroup evaluates its
// chunk at the current rates (no z or dF/dz stored); the workgroup that the
// share tree elects last also takes the BB step of bb_update_kernel, so the
// result equals the separate evaluation + step launches bit for bit.
__global__ __launch_bounds__(kDaThreads) void da_bb_step_kernel(const float* __restrict__ cols, int64_t n_rows,
                                                                const int32_t* __restrict__ d_m,
                                                                const uint8_t* __restrict__ rsid,
                                                                const float* __restrict__ table,
                                                                float* __restrict__ partial,
                                                                double* __restrict__ gpart, int n_chunks,
                                                                uint32_t* arrived, float* __restrict__ G,
                                                                float* __restrict__ F, BBDev B, dvmat_bb_params prm,
                                                                const double* curv, uint32_t* flags_out, int max_ap) {
    const int m = *d_m;
    da_eval_chunk(cols, n_rows, m, max_ap, B.y, rsid, nullptr, table, nullptr, nullptr, partial, n_chunks);
    if (!da_reduce_shares(partial, gpart, m, n_chunks, arrived, G, F)) return;
    bb_update_block(B, MODE_STEP, F, curv, flags_out, prm, G);
}

__global__ __launch_bounds__(kDaThreads) void da_curv_kernel(const float* __restrict__ cols, int64_t n_rows,
                                                             const int32_t* __restrict__ d_m,
                                                             const float* __restrict__ dirv,
                                                             const uint8_t* __restrict__ rsid,
                                                             const int32_t* __restrict__ rows,
                                                             const float* __restrict__ table,
                                                             const float* __restrict__ zref,
                                                             double* __restrict__ partial_d) {
    __shared__ float sd[1024];
    __shared__ double red[kDaThreads / 64];
    const int m = *d_m;
    const int64_t c0 = (int64_t)blockIdx.x * kDaChunk;
    for (int k = threadIdx.x; k < m; k += kDaThreads) sd[k] = dirv[k];
    __syncthreads();
    double a = 0.0;
    for (int u = 0; u < kDaPerThread; ++u) {
        const int64_t i = c0 + u * kDaThreads + threadIdx.x;
        if (i >= n_rows) continue;
        float di = 0.0f;
        for (int k = 0; k < m; ++k) di += cols[(int64_t)k * n_rows + i] * sd[k];
        const int s = rsid[i];
        const float T = table[s * 4 + 0];
        const float zr = zref[rows ? (int64_t)rows[i] : i];
        const float w = zr > T ? table[s * 4 + 1] : (zr < T ? table[s * 4 + 2] : 0.0f);
        a += (double)w * (double)di * (double)di;
    }
    for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kDaThreads / 64; ++w) t += red[w];
        partial_d[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(256) void da_finalize_d_kernel(const double* __restrict__ partial, int n, double* out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += partial[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// The objective's support in voxel order, in one workgroup: each round of
// 1024 voxels flags the weighted ones, a wave ballot and a scan of the wave
// counts place them after the previous rounds'.  One-time set-up work.
__global__ __launch_bounds__(1024) void da_support_kernel(int64_t n_vox, const uint8_t* __restrict__ sid,
                                                          const float* __restrict__ table, int32_t* __restrict__ out,
                                                          uint8_t* __restrict__ out_sid, int32_t* __restrict__ count) {
    __shared__ int wave_count[16];
    __shared__ int base;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int64_t r0 = 0; r0 < n_vox; r0 += 1024) {
        const int64_t i = r0 + threadIdx.x;
        int s = 0;
        bool w = false;
        if (i < n_vox) {
            s = sid[i];
            w = table[s * 4 + 1] != 0.0f || table[s * 4 + 2] != 0.0f;
        }
        const uint64_t mask = __ballot(w);
        const int before = __popcll(mask & ((uint64_t(1) << lane) - 1));
        if (lane == 0) wave_count[wid] = __popcll(mask);
        __syncthreads();
        int off = base;
        for (int q = 0; q < wid; ++q) off += wave_count[q];
        if (w) {
            out[off + before] = (int32_t)i;
            out_sid[off + before] = (uint8_t)s;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int q = 0; q < 16; ++q) t += wave_count[q];
            base += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// col[r] = full[rows[r]]: a dense column cut to the support.
__global__ __launch_bounds__(256) void da_gather_rows_kernel(int64_t n_rows, const int32_t* __restrict__ rows,
                                                             const float* __restrict__ full, float* __restrict__ col) {
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n_rows; r += (int64_t)gridDim.x * 256)
        col[r] = full[rows[r]];
}

}  // namespace dvmat

using namespace dvmat;

extern "C" {

dvmat_status dvmat_da_workspace_size(int64_t n_vox, int32_t max_ap, size_t* bytes) {
    if (!bytes) return set_error(DVMAT_E_ARG, "dvmat_da_workspace_size: bytes is NULL");
    if (n_vox < 1 || max_ap < 1 || max_ap > 1024)
        return set_error(DVMAT_E_ARG, "dvmat_da_workspace_size: n_vox=%lld max_apertures=%d (1..1024)",
                         (long long)n_vox, max_ap);
    *bytes = da_layout(n_vox, max_ap, nullptr, nullptr);
    return DVMAT_OK;
}

dvmat_status dvmat_da_create(int64_t n_vox, int32_t max_ap, void* ws, size_t bytes, dvmat_da* out) {
    if (!out) return set_error(DVMAT_E_ARG, "dvmat_da_create: out is NULL");
    *out = nullptr;
    size_t need = 0;
    dvmat_status st = dvmat_da_workspace_size(n_vox, max_ap, &need);
    if (st) return st;
    if (!ws) return set_error(DVMAT_E_ARG, "dvmat_da_create: workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return set_error(DVMAT_E_ARG, "dvmat_da_create: workspace misaligned");
    if (bytes < need) return set_error(DVMAT_E_NOMEM, "dvmat_da_create: workspace %zu < %zu bytes", bytes, need);
    dvmat_da_s* d = new (std::nothrow) dvmat_da_s();
    if (!d) return set_error(DVMAT_E_NOMEM, "dvmat_da_create: host allocation failed");
    d->n_vox = n_vox;
    d->n_rows = n_vox;
    d->max_ap = max_ap;
    da_layout(n_vox, max_ap, d, static_cast<char*>(ws));
    *out = d;
    return DVMAT_OK;
}

dvmat_status dvmat_da_set_support(dvmat_da d, dvmat_obj obj, int64_t* n_rows, dvmat_stream stream) {
    if (!d || !obj) return set_error(DVMAT_E_ARG, "dvmat_da_set_support: NULL argument");
    if (obj->n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_da_set_support: voxel count mismatch");
    if (d->m != 0) return set_error(DVMAT_E_STATE, "dvmat_da_set_support: %d columns exist already", d->m);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(da_support_kernel, dim3(1), dim3(1024), 0, s, d->n_vox, obj->sid, (const float*)obj->table,
                       d->support, d->csid, d->d_nsup);
    dvmat_status st = check_hip(hipGetLastError(), "dvmat_da_set_support launch");
    if (st) return st;
    int32_t n = 0;
    if ((st = check_hip(hipMemcpyAsync(&n, d->d_nsup, sizeof(n), hipMemcpyDeviceToHost, s), "dvmat_da_set_support copy")))
        return st;
    if ((st = check_hip(hipStreamSynchronize(s), "dvmat_da_set_support synchronize"))) return st;
    if (n > 0) {                               // no weighted voxel at all: keep every row
        d->n_rows = n;
        d->rows = d->support;
        d->row_sid = d->csid;
        d->n_chunks = (int32_t)((d->n_rows + kDaChunk - 1) / kDaChunk);
    }
    if (n_rows) *n_rows = d->n_rows;
    return DVMAT_OK;
}

void dvmat_da_destroy(dvmat_da d) { delete d; }

int32_t dvmat_da_count(dvmat_da d) { return d ? d->m : -1; }

dvmat_status dvmat_da_append(dvmat_da d, dvmat_ddc ddc, const float* x_ind, dvmat_stream stream) {
    if (!d || !ddc || !x_ind) return set_error(DVMAT_E_ARG, "dvmat_da_append: NULL argument");
    if (d->m >= d->max_ap) return set_error(DVMAT_E_STATE, "dvmat_da_append: %d columns already", d->m);
    dvmat_ddc_info_t info;
    dvmat_status st = dvmat_ddc_info(ddc, &info);
    if (st) return st;
    if (info.n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_da_append: voxel count mismatch");
    float* col = d->cols + (int64_t)d->m * d->n_rows;
    st = dvmat_dose(ddc, x_ind, 1, d->rows ? d->gbuf : col, nullptr, nullptr, nullptr, stream);
    if (st) return st;
    if (d->rows) {
        const int64_t nb = std::min<int64_t>((d->n_rows + 255) / 256, 4096);
        hipLaunchKernelGGL(da_gather_rows_kernel, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(256), 0,
                           reinterpret_cast<hipStream_t>(stream), d->n_rows, d->rows, (const float*)d->gbuf, col);
    }
    const int n_counters = (d->n_chunks + kDaFanIn - 1) / kDaFanIn + 1;
    hipLaunchKernelGGL(da_set_count_kernel, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), d->d_m,
                       d->m + 1, d->arrived, n_counters);
    if ((st = check_hip(hipGetLastError(), "dvmat_da_append launch"))) return st;
    d->m++;
    return DVMAT_OK;
}

dvmat_status dvmat_da_eval(dvmat_da d, dvmat_obj obj, const float* y, float* z, float* g, float* G, float* F,
                           dvmat_stream stream) {
    if (!d || !obj || !y || !G) return set_error(DVMAT_E_ARG, "dvmat_da_eval: NULL argument");
    if (obj->n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_da_eval: voxel count mismatch");
    if (d->m == 0) return set_error(DVMAT_E_STATE, "dvmat_da_eval: no columns");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(da_eval_kernel, dim3(d->n_chunks), dim3(kDaThreads), da_lds_bytes(d->max_ap), s, d->cols,
                       d->n_rows, d->d_m, y, d->rows ? d->row_sid : obj->sid, d->rows, obj->table, z,
                       g ? g : d->gbuf, d->partial, d->gpart, d->n_chunks, d->max_ap, d->arrived, G, F);
    return check_hip(hipGetLastError(), "dvmat_da_eval launch");
}

dvmat_status dvmat_da_bb_step(dvmat_da d, dvmat_bb bb, dvmat_obj obj, float* G, float* F, const double* curv,
                              uint32_t* flags, dvmat_stream stream) {
    if (!d || !bb || !obj || !G || !F) return set_error(DVMAT_E_ARG, "dvmat_da_bb_step: NULL argument");
    if (obj->n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_da_bb_step: voxel count mismatch");
    if (d->m == 0) return set_error(DVMAT_E_STATE, "dvmat_da_bb_step: no columns");
    if (bb->m != d->m)
        return set_error(DVMAT_E_STATE, "dvmat_da_bb_step: %d apertures but %d columns", bb->m, d->m);
    hipLaunchKernelGGL(da_bb_step_kernel, dim3(d->n_chunks), dim3(kDaThreads), da_lds_bytes(d->max_ap),
                       reinterpret_cast<hipStream_t>(stream), d->cols, d->n_rows, d->d_m,
                       d->rows ? d->row_sid : obj->sid, obj->table, d->partial, d->gpart, d->n_chunks, d->arrived,
                       G, F, bb->dev, bb->params, curv, flags, d->max_ap);
    return check_hip(hipGetLastError(), "dvmat_da_bb_step launch");
}

dvmat_status dvmat_da_curvature(dvmat_da d, dvmat_obj obj, const float* dir, const float* z_ref, double* curv,
                                dvmat_stream stream) {
    if (!d || !obj || !dir || !z_ref || !curv) return set_error(DVMAT_E_ARG, "dvmat_da_curvature: NULL argument");
    if (obj->n_vox != d->n_vox) return set_error(DVMAT_E_SHAPE, "dvmat_da_curvature: voxel count mismatch");
    if (d->m == 0) return set_error(DVMAT_E_STATE, "dvmat_da_curvature: no columns");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(da_curv_kernel, dim3(d->n_chunks), dim3(kDaThreads), 0, s, d->cols, d->n_rows, d->d_m, dir,
                       d->rows ? d->row_sid : obj->sid, d->rows, obj->table, z_ref, d->partial_d);
    hipLaunchKernelGGL(da_finalize_d_kernel, dim3(1), dim3(256), 0, s, d->partial_d, d->n_chunks, curv);
    return check_hip(hipGetLastError(), "dvmat_da_curvature launch");
}

dvmat_status dvmat_da_column(dvmat_da d, int32_t k, const float** col) {
    if (!d || !col) return set_error(DVMAT_E_ARG, "dvmat_da_column: NULL argument");
    if (k < 0 || k >= d->m) return set_error(DVMAT_E_ARG, "dvmat_da_column: column %d of %d", k, d->m);
    *col = d->cols + (int64_t)k * d->n_rows;
    return DVMAT_OK;
}

}  // extern "C"
