// Aperture selection (pricing problem, second step; Sec. 2.1 and Sec. 2.2.2).
//
// Without the interdigitation constraint the MLC leaf rows are independent,
// so the paper uses two kernels: one thread per (control point, leaf row)
// finds the best opening, then one thread per control point sums its rows and
// the best aperture is chosen.  Here: one workgroup per control point stages
// the point's prices in LDS (coalesced), one thread per leaf row scans it in
// O(n_cols), thread 0 sums the rows in order; a second single-workgroup
// kernel takes the arg-min over control points.
//
// Row scan: with prefix sums P_0 = 0, P_R = p_0 + ... + p_{R-1}, the best
// opening ending at R is [L*, R) with L* the LAST index of max_{L<R} P_L
// (largest prefix = smallest sum; last = shortest).  Keeping the running best
// with strict comparisons on (sum, length) visits R in increasing order, so
// equal (sum, length) keeps the smaller L.  The closed row (0, 0) with sum 0
// is the starting best.
#include "common.hpp"

#include <cmath>

namespace dvmat {

__global__ __launch_bounds__(256) void select_rows_kernel(int n_rows, int n_cols, const float* __restrict__ p,
                                                          const uint8_t* __restrict__ occ, int32_t* __restrict__ L,
                                                          int32_t* __restrict__ R, float* __restrict__ cp_price) {
    extern __shared__ float sm[];
    float* sp = sm;                          // [n_rows * n_cols]
    float* rowsum = sm + n_rows * n_cols;    // [n_rows]
    const int k = blockIdx.x;
    const int per_cp = n_rows * n_cols;
    const bool occupied = occ != nullptr && occ[k] != 0;
    if (occupied) {
        for (int r = threadIdx.x; r < n_rows; r += blockDim.x) {
            L[(int64_t)k * n_rows + r] = 0;
            R[(int64_t)k * n_rows + r] = 0;
        }
        if (threadIdx.x == 0) cp_price[k] = INFINITY;
        return;
    }
    const float* pk = p + (int64_t)k * per_cp;
    for (int i = threadIdx.x; i < per_cp; i += blockDim.x) sp[i] = pk[i];
    __syncthreads();
    for (int r = threadIdx.x; r < n_rows; r += blockDim.x) {
        const float* row = sp + r * n_cols;
        float prefix = 0.0f;
        float max_prefix = 0.0f;
        int arg_l = 0;
        float best_s = 0.0f;
        int best_l = 0, best_r = 0, best_len = 0;
        for (int rr = 1; rr <= n_cols; ++rr) {
            prefix += row[rr - 1];
            const float s = prefix - max_prefix;
            const int len = rr - arg_l;
            if (s < best_s || (s == best_s && len < best_len)) {
                best_s = s;
                best_l = arg_l;
                best_r = rr;
                best_len = len;
            }
            if (prefix >= max_prefix) {
                max_prefix = prefix;
                arg_l = rr;
            }
        }
        L[(int64_t)k * n_rows + r] = best_l;
        R[(int64_t)k * n_rows + r] = best_r;
        rowsum[r] = best_s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int r = 0; r < n_rows; ++r) s += rowsum[r];
        cp_price[k] = s;
    }
}

__global__ __launch_bounds__(256) void select_best_kernel(int n_cp, const float* __restrict__ cp_price,
                                                          int32_t* best, float* best_price) {
    __shared__ float sv[256];
    __shared__ int si[256];
    float v = INFINITY;
    int idx = -1;
    for (int k = threadIdx.x; k < n_cp; k += 256) {
        const float c = cp_price[k];
        if (c < v) { v = c; idx = k; }      // increasing k: first minimum kept
    }
    sv[threadIdx.x] = v;
    si[threadIdx.x] = idx;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const float v2 = sv[threadIdx.x + o];
            const int i2 = si[threadIdx.x + o];
            const float v1 = sv[threadIdx.x];
            const int i1 = si[threadIdx.x];
            if (i2 >= 0 && (i1 < 0 || v2 < v1 || (v2 == v1 && i2 < i1))) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool improving = si[0] >= 0 && sv[0] < 0.0f;
        *best = improving ? si[0] : -1;
        *best_price = sv[0];
    }
}

}  // namespace dvmat

using namespace dvmat;

extern "C" dvmat_status dvmat_aperture_select(dvmat_geom geom, const float* p, const uint8_t* occupied, int32_t* L,
                                              int32_t* R, float* cp_price, int32_t* best, float* best_price,
                                              dvmat_stream stream) {
    if (geom.n_cp < 1 || geom.n_rows < 1 || geom.n_cols < 1)
        return set_error(DVMAT_E_SHAPE, "dvmat_aperture_select: geometry %d x %d x %d", geom.n_cp, geom.n_rows,
                         geom.n_cols);
    if (geom.n_cols > 1024 || (int64_t)geom.n_rows * (geom.n_cols + 1) > 16384)
        return set_error(DVMAT_E_SHAPE, "dvmat_aperture_select: beamlet grid %d x %d needs n_rows*(n_cols+1) <= 16384 and n_cols <= 1024",
                         geom.n_rows, geom.n_cols);
    if (!p || !L || !R || !cp_price || !best || !best_price)
        return set_error(DVMAT_E_ARG, "dvmat_aperture_select: NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t lds = ((size_t)geom.n_rows * geom.n_cols + geom.n_rows) * sizeof(float);
    hipLaunchKernelGGL(select_rows_kernel, dim3(geom.n_cp), dim3(256), lds, s, geom.n_rows, geom.n_cols, p, occupied,
                       L, R, cp_price);
    hipLaunchKernelGGL(select_best_kernel, dim3(1), dim3(256), 0, s, geom.n_cp, cp_price, best, best_price);
    return check_hip(hipGetLastError(), "dvmat_aperture_select launch");
}
