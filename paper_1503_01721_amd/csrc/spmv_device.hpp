// Device building blocks of the sparse products (shared by the CSR kernels,
// the batched launch and the panel kernel): vector loads of the matrix
// stream, gathers, the per-row epilogues and the block-row processors.
#pragma once

#include "common.hpp"

namespace dvmat {


typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

enum Epi { EPI_PLAIN = 0, EPI_OBJ = 1, EPI_CURV = 2, EPI_SCALE = 3 };

struct SpmvParams {
    int64_t n_rows;          // rows of the orientation (the last block row may be partial)
    const int64_t* rowptr;
    const int32_t* col;
    const void* val;
    const int32_t* blocks;
    int64_t n_blocks;
    const int32_t* perm;     // stored position -> row, or nullptr
    int perm_runs;           // 1: the B rows of every block row are consecutive natural rows
    const float* x;
    float* y;                // output rows (nullable for EPI_CURV)
    const uint8_t* sid;      // objective epilogue
    const float* table;
    float* g;
    float* partial;
    double* partial_d;
    const float* zref;
    const float* row_scale;  // EPI_SCALE: y_r *= row_scale[r]
    const float* x_scale;    // batched 16-bit dose: v *= x_scale[col]
    int ld;                  // row stride of y and g, and of the per-workgroup partials
};

__device__ __forceinline__ i32x4 load_cols16(const uint16_t* col16, int64_t k) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(col16) + (k >> 2));
    return i32x4{(int)(w.x & 0xffffu), (int)(w.x >> 16), (int)(w.y & 0xffffu), (int)(w.y >> 16)};
}

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

template <int NRHS, bool SCALE_X>
__device__ __forceinline__ void fma4(float (&acc)[NRHS], const SpmvParams& P, f32x4 v, i32x4 c) {
    if constexpr (SCALE_X) {
        v.x *= P.x_scale[c.x];
        v.y *= P.x_scale[c.y];
        v.z *= P.x_scale[c.z];
        v.w *= P.x_scale[c.w];
    }
    fma_gather<NRHS>(acc, P.x, v.x, c.x);
    fma_gather<NRHS>(acc, P.x, v.y, c.y);
    fma_gather<NRHS>(acc, P.x, v.z, c.z);
    fma_gather<NRHS>(acc, P.x, v.w, c.w);
}

// Sum over the 64 lanes of a wave, in a fixed order, returned to every lane.
// Lane permutes within each row of 16 lanes run on the vector ALU (DPP: swap
// neighbours, swap pairs, mirror 8, mirror 16), so every lane of a row holds
// the row's sum; the four row sums are then read as scalars and added.  No
// LDS traffic, unlike a shuffle butterfly (the panel kernel's gathers use LDS).
template <int CTRL>
__device__ __forceinline__ float dpp_step(float v) {
    return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float wave_sum(float v) {
    v = dpp_step<0xB1>(v);    // quad_perm [1,0,3,2]
    v = dpp_step<0x4E>(v);    // quad_perm [2,3,0,1]
    v = dpp_step<0x141>(v);   // row_half_mirror
    v = dpp_step<0x140>(v);   // row_mirror
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inputs of one row's epilogue that sit in memory: they are loaded before
// the row's products are formed, so their latency overlaps the matrix stream.
// The natural row index (rows may be stored in another order) is looked up at
// the epilogue: only the beamlet rows are reordered, and those are long.
struct EpiRow {
    int sid;     // structure id (objective, curvature)
    float zr;    // reference dose (curvature)
    float rs;    // row scale (16-bit price)
};

__device__ __forceinline__ int64_t natural_row(const SpmvParams& P, int64_t r) { return P.perm ? P.perm[r] : r; }

template <int EPI>
__device__ __forceinline__ EpiRow epi_load(const SpmvParams& P, int64_t r) {
    EpiRow e{0, 0.0f, 1.0f};
    if constexpr (EPI != EPI_PLAIN) {
        if (r < P.n_rows) {
            const int64_t n = natural_row(P, r);
            if constexpr (EPI == EPI_OBJ || EPI == EPI_CURV) e.sid = P.sid[n];
            if constexpr (EPI == EPI_CURV) e.zr = P.zref[n];
            if constexpr (EPI == EPI_SCALE) e.rs = P.row_scale[n];
        }
    }
    return e;
}

// Row epilogue (one lane per row): plain, per-row scale, objective, curvature.
// tab: the objective table (T, w+, w-, 0) per structure, staged in LDS.
template <int NRHS, int EPI>
__device__ __forceinline__ void row_epilogue(const SpmvParams& P, int64_t r, const EpiRow& e, const f32x4* tab,
                                             const float (&acc)[NRHS], float (&fpart)[NRHS], double& cpart) {
    const int64_t o = r * P.ld;
    if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
        for (int h = 0; h < NRHS; ++h) P.y[o + h] = acc[h];
    } else if constexpr (EPI == EPI_SCALE) {
#pragma unroll
        for (int h = 0; h < NRHS; ++h) P.y[o + h] = acc[h] * e.rs;
    } else if constexpr (EPI == EPI_OBJ) {
        const f32x4 t = tab[e.sid];
        const float T = t.x, wo = t.y, wu = t.z;
#pragma unroll
        for (int h = 0; h < NRHS; ++h) {
            const float z = acc[h];
            P.y[o + h] = z;
            const float over = fmaxf(z - T, 0.0f);
            const float under = fmaxf(T - z, 0.0f);
            if (P.g) P.g[o + h] = 2.0f * wo * over - 2.0f * wu * under;
            fpart[h] += wo * over * over + wu * under * under;
        }
    } else {  // EPI_CURV
        const float d = acc[0];
        if (P.y) P.y[r] = d;
        const f32x4 t = tab[e.sid];
        const float T = t.x;
        const float w = e.zr > T ? t.y : (e.zr < T ? t.z : 0.0f);
        cpart += (double)w * (double)d * (double)d;
    }
}

// ---- block processors --------------------------------------------------------

// 4 block entries x B values from value index 4*B*k/4 on: V[t] holds values
// 4t..4t+3 of the 4B consecutive values; entry q's value b is element q*B + b.
template <int ST, int B>
__device__ __forceinline__ void load_block_vals(const void* base, int64_t k, f32x4 (&V)[B]) {
#pragma unroll
    for (int t = 0; t < B; ++t) V[t] = load_vals<ST>(base, k * B + 4 * t);
}

// xsrc: the gathered vector, NRHS values per column (global memory, or a
// panel's slice in LDS with panel-local columns).
template <int NRHS, int B, bool SCALE_X>
__device__ __forceinline__ void fma4_blocked(float (&acc)[B][NRHS], const SpmvParams& P, const float* xsrc,
                                             const f32x4 (&V)[B], i32x4 c) {
    const int cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float xv[NRHS];
        if constexpr (NRHS == 8) {
            const f32x4 a = *reinterpret_cast<const f32x4*>(xsrc + (int64_t)cc[q] * 8);
            const f32x4 b = *reinterpret_cast<const f32x4*>(xsrc + (int64_t)cc[q] * 8 + 4);
            xv[0] = a.x; xv[1] = a.y; xv[2] = a.z; xv[3] = a.w;
            xv[4] = b.x; xv[5] = b.y; xv[6] = b.z; xv[7] = b.w;
        } else if constexpr (NRHS == 4) {
            const f32x4 a = *reinterpret_cast<const f32x4*>(xsrc + (int64_t)cc[q] * 4);
            xv[0] = a.x; xv[1] = a.y; xv[2] = a.z; xv[3] = a.w;
        } else {
#pragma unroll
            for (int h = 0; h < NRHS; ++h) xv[h] = xsrc[(int64_t)cc[q] * NRHS + h];
        }
        if constexpr (SCALE_X) {
            const float sc = P.x_scale[cc[q]];
#pragma unroll
            for (int h = 0; h < NRHS; ++h) xv[h] *= sc;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int e = q * B + b;
            const float v = V[e / 4][e % 4];
#pragma unroll
            for (int h = 0; h < NRHS; ++h) acc[b][h] += v * xv[h];
        }
    }
}

// Kernel body "row": block rows in order; per block row each lane streams 4
// consecutive block entries per step (16-byte column load, B 16-byte value
// loads at FP32), two steps in flight; the wave reduction (wave_sum) sums each
// of the B rows; for B x NRHS <= 4 the sums stay in the lane of their block
// row and every lane finishes its own rows after the unit, else lane 0
// finishes each block row.  The row pointers and epilogue inputs of
// every block row of the unit are loaded up front, lane i for block row i, so
// the short block rows of the dose do not each wait for them in turn.
// LDSG: gather from a panel's slice of the vector in LDS (xsrc) through the
// panel-local 16-bit column indices col16, instead of from P.x through P.col.
// DEEP: four steps in flight where a row is long (one right-hand side, B = 1).
template <int ST, int NRHS, int EPI, bool SCALE_X, int B, bool LDSG = false, bool DEEP = false>
__device__ __forceinline__ void block_rows(const SpmvParams& P, int r0, int r1, int lane, const f32x4* tab,
                                           float (&fpart)[NRHS], double& cpart, const float* xsrc = nullptr,
                                           const uint16_t* col16 = nullptr) {
    if constexpr (!LDSG) xsrc = P.x;
    auto cols = [&](int64_t k) -> i32x4 {
        if constexpr (LDSG) return load_cols16(col16, k);
        else return load_cols(P.col, k);
    };
    const int nbr = r1 - r0;                              // 1 .. kBlockRowsMax
    const int li = lane < nbr ? lane : nbr - 1;
    // block row starts relative to the unit's first entry (a unit holds fewer
    // than 2^31 stored positions)
    const int64_t base = P.rowptr[r0];
    const int64_t last = P.rowptr[r1];
    const int rel = (int)(P.rowptr[r0 + li] - base);
    // end of each lane's block row (the next row's start; the unit's end for the last)
    const int rel_dn = __shfl_down(rel, 1);
    const int rel_end = lane + 1 < nbr ? rel_dn : (int)(last - base);
    // epilogue inputs: structure ids packed one byte per row, or floats; the
    // natural index of the block row's first row when its rows run consecutively
    int sid4 = 0;
    float ef[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
        const EpiRow e = epi_load<EPI>(P, (int64_t)(r0 + li) * B + q);
        sid4 |= e.sid << (8 * q);
        ef[q] = EPI == EPI_CURV ? e.zr : e.rs;
    }
    const int nat0 = P.perm && P.perm_runs ? P.perm[(int64_t)(r0 + li) * B] : 0;
    // Small blocks keep each block row's sums in the lane of that block row and
    // finish all rows together after the unit; larger ones finish each block
    // row in lane 0 (registers).
    constexpr bool kLaneEpilogue = B * NRHS <= 4;
    float mine[kLaneEpilogue ? B : 1][kLaneEpilogue ? NRHS : 1];
#pragma unroll
    for (int q = 0; q < (kLaneEpilogue ? B : 1); ++q)
#pragma unroll
        for (int h = 0; h < (kLaneEpilogue ? NRHS : 1); ++h) mine[q][h] = 0.0f;
    auto row = [&](int i) {
        const int64_t e0 = base + __builtin_amdgcn_readlane(rel, i);
        const int64_t e1 = base + __builtin_amdgcn_readlane(rel_end, i);
        float acc[B][NRHS];
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
            for (int h = 0; h < NRHS; ++h) acc[q][h] = 0.0f;
        int64_t k = e0 + lane * 4;
        // two steps in flight unless a step already holds 64 bytes of values
        // per lane (FP32 with 4 rows per block row): registers, not bytes, bind there
        constexpr bool kTwoSteps = (ST == DVMAT_F32 ? 4 : 2) * B < 16;
        constexpr bool kFourSteps = DEEP && kTwoSteps && B == 1 && NRHS == 1;
        if constexpr (kFourSteps) {
            for (; k + 768 < e1; k += 1024) {
                f32x4 V0[B], V1[B], V2[B], V3[B];
                load_block_vals<ST, B>(P.val, k, V0);
                const i32x4 c0 = cols(k);
                load_block_vals<ST, B>(P.val, k + 256, V1);
                const i32x4 c1 = cols(k + 256);
                load_block_vals<ST, B>(P.val, k + 512, V2);
                const i32x4 c2 = cols(k + 512);
                load_block_vals<ST, B>(P.val, k + 768, V3);
                const i32x4 c3 = cols(k + 768);
                fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V0, c0);
                fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V1, c1);
                fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V2, c2);
                fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V3, c3);
            }
        }
        if constexpr (kTwoSteps) {
            for (; k + 256 < e1; k += 512) {
                f32x4 V0[B], V1[B];
                load_block_vals<ST, B>(P.val, k, V0);
                const i32x4 c0 = cols(k);
                load_block_vals<ST, B>(P.val, k + 256, V1);
                const i32x4 c1 = cols(k + 256);
                fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V0, c0);
                fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V1, c1);
            }
        } else {
            for (; k + 256 < e1; k += 256) {
                f32x4 V0[B];
                load_block_vals<ST, B>(P.val, k, V0);
                const i32x4 c0 = cols(k);
                fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V0, c0);
            }
        }
        if (k < e1) {
            f32x4 V0[B];
            load_block_vals<ST, B>(P.val, k, V0);
            const i32x4 c0 = cols(k);
            fma4_blocked<NRHS, B, SCALE_X>(acc, P, xsrc, V0, c0);
        }
        if (e1 > e0) {                                   // an empty block row sums to zero
#pragma unroll
            for (int q = 0; q < B; ++q)
#pragma unroll
                for (int h = 0; h < NRHS; ++h) acc[q][h] = wave_sum(acc[q][h]);
        }
        if constexpr (kLaneEpilogue) {
            // the sums are wave-uniform: lane i keeps block row i's
            if (lane == i) {
#pragma unroll
                for (int q = 0; q < B; ++q)
#pragma unroll
                    for (int h = 0; h < NRHS; ++h) mine[q][h] = acc[q][h];
            }
        } else {
            const int sids = __builtin_amdgcn_readlane(sid4, i);
            const int n0 = __builtin_amdgcn_readlane(nat0, i);
            float efs[B];
#pragma unroll
            for (int q = 0; q < B; ++q) efs[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ef[q]), i));
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < B; ++q) {
                    const int64_t r = (int64_t)(r0 + i) * B + q;
                    if (r < P.n_rows) {
                        const EpiRow e{(sids >> (8 * q)) & 0xff, efs[q], efs[q]};
                        const int64_t nat = !P.perm ? r : P.perm_runs ? (int64_t)n0 + q : (int64_t)P.perm[r];
                        row_epilogue<NRHS, EPI>(P, nat, e, tab, acc[q], fpart, cpart);
                    }
                }
            }
        }
    };
    if constexpr (kLaneEpilogue) {
        // empty block rows (voxels no beamlet reaches) take no pass: their
        // lanes keep zero sums, and the epilogue below writes them
        uint64_t todo = __ballot(lane < nbr && rel_end > rel);
        while (todo) {
            const int i = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(todo));
            todo &= todo - 1;
            row(i);
        }
    } else {
        for (int i = 0; i < nbr; ++i) row(i);
    }
    if constexpr (kLaneEpilogue) {
        // every lane finishes its own block row: coalesced stores, parallel epilogue
        if (lane < nbr) {
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int64_t r = (int64_t)(r0 + lane) * B + q;
                if (r < P.n_rows) {
                    const EpiRow e{(sid4 >> (8 * q)) & 0xff, ef[q], ef[q]};
                    const int64_t nat = !P.perm ? r : P.perm_runs ? (int64_t)nat0 + q : (int64_t)P.perm[r];
                    row_epilogue<NRHS, EPI>(P, nat, e, tab, mine[q], fpart, cpart);
                }
            }
        }
    }
}

// One step of the pipelined kernel: the 4 block entries of this lane at
// position k (relative to base), or zeros past the block row's end e.
template <int ST, int B>
__device__ __forceinline__ void load_step(const SpmvParams& P, int64_t base, int k, int e, int lane, f32x4 (&V)[B],
                                          i32x4& c) {
    const int kl = k + 4 * lane;
    if (kl < e) {
        load_block_vals<ST, B>(P.val, base + kl, V);
        c = load_cols(P.col, base + kl);
    } else {
#pragma unroll
        for (int t = 0; t < B; ++t) V[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        c = i32x4{0, 0, 0, 0};
    }
}

// Kernel body "pipe": the row kernel's arithmetic, software-pipelined over the
// steps of the whole unit: the loads of the next step (which may be the first
// step of a later block row) are issued before the gathers of the current
// step, so the matrix stream of one step overlaps the gathers of the other.
// Empty block rows take no step; their outputs are written when the wave
// passes them.
template <int ST, int NRHS, int EPI, bool SCALE_X, int B>
__device__ __forceinline__ void block_pipe(const SpmvParams& P, int r0, int r1, int lane, const f32x4* tab,
                                           float (&fpart)[NRHS], double& cpart) {
    const int nbr = r1 - r0;                              // 1 .. kBlockRowsMax
    const int li = lane < nbr ? lane : nbr - 1;
    const int64_t base = P.rowptr[r0];
    const int total = (int)(P.rowptr[r1] - base);
    const int rel = (int)(P.rowptr[r0 + li] - base);
    int sid4 = 0;
    float ef[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
        const EpiRow e = epi_load<EPI>(P, (int64_t)(r0 + li) * B + q);
        sid4 |= e.sid << (8 * q);
        ef[q] = EPI == EPI_CURV ? e.zr : e.rs;
    }
    // end of block row j, relative to base
    auto row_end = [&](int j) -> int { return j + 1 < nbr ? __builtin_amdgcn_readlane(rel, j + 1) : total; };
    // outputs of block row j from its (already reduced) sums
    auto finish = [&](int j, const float (&sum)[B][NRHS]) {
        const int sids = __builtin_amdgcn_readlane(sid4, j);
        float efs[B];
#pragma unroll
        for (int q = 0; q < B; ++q) efs[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ef[q]), j));
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const int64_t r = (int64_t)(r0 + j) * B + q;
                if (r < P.n_rows) {
                    const EpiRow e{(sids >> (8 * q)) & 0xff, efs[q], efs[q]};
                    row_epilogue<NRHS, EPI>(P, natural_row(P, r), e, tab, sum[q], fpart, cpart);
                }
            }
        }
    };
    float zero[B][NRHS];
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
        for (int h = 0; h < NRHS; ++h) zero[q][h] = 0.0f;
    // leading empty block rows
    int i = 0, k = 0, e1 = row_end(0);
    while (k >= e1) {
        finish(i, zero);
        if (++i == nbr) return;
        e1 = row_end(i);
    }
    float acc[B][NRHS];
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
        for (int h = 0; h < NRHS; ++h) acc[q][h] = 0.0f;
    f32x4 V[B];
    i32x4 c;
    load_step<ST, B>(P, base, k, e1, lane, V, c);
    while (true) {
        // the step after (i, k): the next 256 entries of row i, else the first
        // step of the next non-empty block row
        int kn = k + 256, in = i, e1n = e1;
        if (kn >= e1) {
            kn = e1;
            in = i + 1;
            e1n = in < nbr ? row_end(in) : kn;
            while (in < nbr && kn >= e1n) {
                ++in;
                e1n = in < nbr ? row_end(in) : kn;
            }
        }
        const bool more = in < nbr;
        f32x4 Vn[B];
        i32x4 cn;
        if (more) load_step<ST, B>(P, base, kn, e1n, lane, Vn, cn);
        if (k + 4 * lane < e1) fma4_blocked<NRHS, B, SCALE_X>(acc, P, P.x, V, c);
        if (in != i) {
#pragma unroll
            for (int q = 0; q < B; ++q)
#pragma unroll
                for (int h = 0; h < NRHS; ++h) acc[q][h] = wave_sum(acc[q][h]);
            finish(i, acc);
#pragma unroll
            for (int q = 0; q < B; ++q)
#pragma unroll
                for (int h = 0; h < NRHS; ++h) acc[q][h] = 0.0f;
            for (int j = i + 1; j < in; ++j) finish(j, zero);
        }
        if (!more) break;
        i = in;
        k = kn;
        e1 = e1n;
#pragma unroll
        for (int t = 0; t < B; ++t) V[t] = Vn[t];
        c = cn;
    }
}

// acc_l: this wave's LDS row accumulators [kBlockRowsMax * NRHS]; rel: [kBlockRowsMax + 1].
template <int ST, int NRHS, int EPI, bool SCALE_X>
__device__ __forceinline__ void block_stream(const SpmvParams& P, int r0, int r1, int lane, float* acc_l, int* rel,
                                             const f32x4* tab, float (&fpart)[NRHS], double& cpart) {
    const int nr = r1 - r0;                            // 1 .. kBlockRowsMax
    const EpiRow ein = epi_load<EPI>(P, lane < nr ? (int64_t)r0 + lane : P.n_rows);
    const int64_t nat = lane < nr ? natural_row(P, (int64_t)r0 + lane) : 0;
    const int64_t e0 = P.rowptr[r0];
    const int ne = (int)(P.rowptr[r0 + nr] - e0);
    for (int i = lane; i <= nr; i += kWaveSize) rel[i] = (int)(P.rowptr[r0 + i] - e0);
    for (int i = lane; i < nr * NRHS; i += kWaveSize) acc_l[i] = 0.0f;
    wave_sync_lds();
    int cur = 0;
    f32x4 vn = {0.0f, 0.0f, 0.0f, 0.0f};
    i32x4 cn = {0, 0, 0, 0};
    if (lane * 4 < ne) {
        vn = load_vals<ST>(P.val, e0 + lane * 4);
        cn = load_cols(P.col, e0 + lane * 4);
    }
    for (int c0 = 0; c0 < ne; c0 += 256) {
        const int k = c0 + lane * 4;
        const f32x4 v = vn;
        const i32x4 c = cn;
        if (k + 256 < ne) {
            vn = load_vals<ST>(P.val, e0 + k + 256);
            cn = load_cols(P.col, e0 + k + 256);
        }
        float part[NRHS];
#pragma unroll
        for (int h = 0; h < NRHS; ++h) part[h] = 0.0f;
        int row = -1;
        if (k < ne) {
            fma4<NRHS, SCALE_X>(part, P, v, c);
            while (rel[cur + 1] <= k) ++cur;
            row = cur;
        }
#pragma unroll
        for (int d = 1; d < kWaveSize; d <<= 1) {
            const int orow = __shfl_down(row, d);
            float o[NRHS];
#pragma unroll
            for (int h = 0; h < NRHS; ++h) o[h] = __shfl_down(part[h], d);
            if (lane + d < kWaveSize && orow == row) {
#pragma unroll
                for (int h = 0; h < NRHS; ++h) part[h] += o[h];
            }
        }
        const int prow = __shfl_up(row, 1);
        if (row >= 0 && (lane == 0 || prow != row)) {
#pragma unroll
            for (int h = 0; h < NRHS; ++h) acc_l[row * NRHS + h] += part[h];
        }
    }
    wave_sync_lds();
    if (lane < nr) {
        float a[NRHS];
#pragma unroll
        for (int h = 0; h < NRHS; ++h) a[h] = acc_l[lane * NRHS + h];
        row_epilogue<NRHS, EPI>(P, nat, ein, tab, a, fpart, cpart);
    }
    wave_sync_lds();
}

// Per-workgroup partial of the objective / curvature (fixed order).
template <int NRHS, int EPI, int kWaves>
__device__ __forceinline__ void workgroup_partials_n(const SpmvParams& P, int lane, int wid, float (&fpart)[NRHS],
                                                     double cpart) {
    if constexpr (EPI == EPI_OBJ || EPI == EPI_CURV) {
        __shared__ float sp[kWaves][NRHS];
        __shared__ double sd[kWaves];
        if constexpr (EPI == EPI_OBJ) {
#pragma unroll
            for (int h = 0; h < NRHS; ++h) fpart[h] = wave_sum(fpart[h]);
        } else {
            cpart = wave_sum_d(cpart);
        }
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
                    P.partial[(int64_t)blockIdx.x * P.ld + h] = s;
                }
            } else {
                double s = 0.0;
                for (int w = 0; w < kWaves; ++w) s += sd[w];
                P.partial_d[blockIdx.x] = s;
            }
        }
    }
}

template <int NRHS, int EPI>
__device__ __forceinline__ void workgroup_partials(const SpmvParams& P, int lane, int wid, float (&fpart)[NRHS],
                                                   double cpart) {
    workgroup_partials_n<NRHS, EPI, kSpmvThreads / kWaveSize>(P, lane, wid, fpart, cpart);
}

// One plan of a batched launch: its orientation's arrays, and its first
// global work unit (CSR) or part (panels) in the batch's work list.
struct PlanDev {
    const int64_t* rowptr;
    const int32_t* col;
    const void* val;
    const int32_t* blocks;
    const float* scale;   // per-beamlet scale (16-bit storage) or nullptr
    const int32_t* perm;  // stored position -> row, or nullptr
    int64_t n_rows;       // rows of the orientation
    int64_t block_base;   // first global unit (CSR) or part (panels) of this plan
    int64_t n_blocks;     // units (CSR) or parts (panels)
    int perm_runs;
    // panel layout
    const uint16_t* col16;
    const int32_t* ulist;
    const int64_t* panel_u;
    const int32_t* part_units;
    const int32_t* part_panel;
};

struct BatchParams {
    const PlanDev* plans;     // device [n_plans]
    int n_plans;
    int64_t total_blocks;     // units (CSR) or parts (panels) over all plans
    const float* x[kMaxBatch];
    float* y[kMaxBatch];
};

// Batched products on the panel layouts (spmv_panel.hip): right-hand sides
// [h0, h0 + chunk) of nrhs, chunk by chunk; scale_stage multiplies the staged
// slice by the per-beamlet scale (16-bit dose).  B: rows per block row of the
// panel layout, or minus the lanes per row of the sliced layout.
dvmat_status launch_batch_panel(int storage, int B, int epi_scale, bool scale_stage, int64_t max_panel_cols,
                                const BatchParams& Bp, int nrhs, int workgroups, hipStream_t s);

// Products on the panel layout (spmv_panel.hip): x is the input vector with
// nrhs values per column; P carries the outputs and epilogue inputs; the
// number of workgroups launched is returned in nwg (for the partial sums).
template <int EPI>
dvmat_status launch_panel(const KernelCfg& cfg, int storage, const CsrDev& c, const SpmvParams& P, const float* x,
                          int nrhs, hipStream_t s, int* nwg, bool xcd_runs);

// Wave position: workgroup w on XCD w % 8; the XCD's waves share its block range.
struct WaveSlot {
    int lane, wid, lw, waves_per_xcd, xcd;
};

__device__ __forceinline__ WaveSlot wave_slot() {
    constexpr int kWaves = kSpmvThreads / kWaveSize;
    WaveSlot s;
    s.lane = threadIdx.x & (kWaveSize - 1);
    s.wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    s.xcd = blockIdx.x % kNumXcd;
    s.lw = (blockIdx.x / kNumXcd) * kWaves + s.wid;
    s.waves_per_xcd = (gridDim.x / kNumXcd) * kWaves;
    return s;
}


}  // namespace dvmat
