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
#include <mutex>

namespace dvmat {

// Library-owned scratch for the interdigitated selection's per-row dynamic-
// programming values when the caller cannot pass a workspace.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code
// the name stands for a host-side shadow, not the device address: kernels get
// the address that hipGetSymbolAddress returns for the current device.
constexpr size_t kSelectScratchBytes = DVMAT_SELECT_SCRATCH_BYTES;
static_assert(kSelectScratchBytes % 256 == 0, "scratch size");
static __device__ __align__(256) float scratch[kSelectScratchBytes / sizeof(float)];

// Leaf window of one row: (Lmin, Lmax, Rmin, Rmax), clamped to [0, n]; the
// full window when none is given.
struct Window {
    int lmin, lmax, rmin, rmax;
};

__device__ __forceinline__ Window row_window(const int32_t* win, int64_t kr, int n) {
    if (!win) return Window{0, n, 0, n};
    const int4 w = reinterpret_cast<const int4*>(win)[kr];
    return Window{max(w.x, 0), min(w.y, n), max(w.z, 0), min(w.w, n)};
}

__global__ __launch_bounds__(256) void select_rows_kernel(int n_rows, int n_cols, const float* __restrict__ p,
                                                          const uint8_t* __restrict__ occ,
                                                          const int32_t* __restrict__ win, int32_t* __restrict__ L,
                                                          int32_t* __restrict__ R, float* __restrict__ cp_price) {
    extern __shared__ float sm[];
    float* sp = sm;                          // [n_rows * n_cols]
    float* rowsum = sm + n_rows * n_cols;    // [n_rows]
    __shared__ int infeasible;
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
    if (threadIdx.x == 0) infeasible = 0;
    const float* pk = p + (int64_t)k * per_cp;
    for (int i = threadIdx.x; i < per_cp; i += blockDim.x) sp[i] = pk[i];
    __syncthreads();
    for (int r = threadIdx.x; r < n_rows; r += blockDim.x) {
        const float* row = sp + r * n_cols;
        const Window w = row_window(win, (int64_t)k * n_rows + r, n_cols);
        // R runs 0..n; before R is considered, L = R joins the running maximum
        // of prefix sums over allowed L (last index of the maximum = shortest)
        float prefix = 0.0f;
        float max_prefix = 0.0f;
        int arg_l = -1;
        float best_s = INFINITY;
        int best_l = 0, best_r = 0, best_len = 0;
        for (int rr = 0; rr <= n_cols; ++rr) {
            if (rr > 0) prefix += row[rr - 1];
            if (rr >= w.lmin && rr <= w.lmax && (arg_l < 0 || prefix >= max_prefix)) {
                max_prefix = prefix;
                arg_l = rr;
            }
            if (rr >= w.rmin && rr <= w.rmax && arg_l >= 0) {
                const float s = prefix - max_prefix;
                const int len = rr - arg_l;
                if (s < best_s || (s == best_s && len < best_len)) {
                    best_s = s;
                    best_l = arg_l;
                    best_r = rr;
                    best_len = len;
                }
            }
        }
        if (best_s == INFINITY) atomicOr(&infeasible, 1);    // LDS flag: no allowed opening
        L[(int64_t)k * n_rows + r] = best_l;
        R[(int64_t)k * n_rows + r] = best_r;
        rowsum[r] = best_s;
    }
    __syncthreads();
    if (infeasible) {
        for (int r = threadIdx.x; r < n_rows; r += blockDim.x) {
            L[(int64_t)k * n_rows + r] = 0;
            R[(int64_t)k * n_rows + r] = 0;
        }
        if (threadIdx.x == 0) cp_price[k] = INFINITY;
        return;
    }
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int r = 0; r < n_rows; ++r) s += rowsum[r];
        cp_price[k] = s;
    }
}

// Leaf windows from the openings L, R [n_cp][n_rows] of the occupied
// neighbouring control points k-1 and k+1: each leaf within travel beamlets.
__global__ __launch_bounds__(256) void leaf_windows_kernel(int n_cp, int n_rows, int n_cols,
                                                           const uint8_t* __restrict__ occ,
                                                           const int32_t* __restrict__ L,
                                                           const int32_t* __restrict__ R, int travel,
                                                           int32_t* __restrict__ win) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_cp * n_rows) return;
    const int k = (int)(i / n_rows), r = (int)(i % n_rows);
    int4 w = make_int4(0, n_cols, 0, n_cols);
    for (int nb = k - 1; nb <= k + 1; nb += 2) {
        if (nb < 0 || nb >= n_cp || !occ[nb]) continue;
        const int64_t j = (int64_t)nb * n_rows + r;
        w.x = max(w.x, L[j] - travel);
        w.y = min(w.y, L[j] + travel);
        w.z = max(w.z, R[j] - travel);
        w.w = min(w.w, R[j] + travel);
    }
    reinterpret_cast<int4*>(win)[i] = w;
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

// ---- interdigitation -------------------------------------------------------
//
// With the constraint L_r <= min(R_{r-1}, R_{r+1}) (Sec. 2.2.2) adjacent rows
// must satisfy L_r <= R_{r+1} and L_{r+1} <= R_r; a closed row may park at any
// position p (L = R = p).  Dynamic programming over the rows, state = opening
// (L, R), 0 <= L <= R <= n, triangular index L*(n+1) - L*(L-1)/2 + (R - L):
//   V_r(L, R) = rowsum_r(L, R) + min { V_{r-1}(L', R') : L' <= R, R' >= L }.
// The inner minimum is M(R, L) with M(a, b) = min_{L' <= a} min_{R' >= max(b, L')}
// V_{r-1}(L', R'): a suffix minimum over R' per L', then a prefix minimum
// over L'.  Each row's V goes to the workspace; backtracking picks, per row,
// the smallest-index compatible state attaining the minimum.

__device__ __forceinline__ int tri_index(int L, int R, int n) { return L * (n + 1) - L * (L - 1) / 2 + (R - L); }

__global__ __launch_bounds__(256) void select_interdig_kernel(int n_rows, int n, const float* __restrict__ p,
                                                              const uint8_t* __restrict__ occ,
                                                              const int32_t* __restrict__ win,
                                                              int32_t* __restrict__ L, int32_t* __restrict__ R,
                                                              float* __restrict__ cp_price,
                                                              float* __restrict__ hist) {
    extern __shared__ float sm[];
    const int S = (n + 1) * (n + 2) / 2;
    const int W = n + 1;
    float* grid = sm;                 // [W][W]: suffix minima, then M
    float* cur = grid + W * W;        // [S]
    float* pre = cur + S;             // [W] prefix sums of the current row
    __shared__ float rv[256];
    __shared__ int ri[256];
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    if (occ != nullptr && occ[k] != 0) {
        for (int r = tid; r < n_rows; r += blockDim.x) {
            L[(int64_t)k * n_rows + r] = 0;
            R[(int64_t)k * n_rows + r] = 0;
        }
        if (tid == 0) cp_price[k] = INFINITY;
        return;
    }
    const float* pk = p + (int64_t)k * n_rows * n;
    float* hk = hist + (int64_t)k * n_rows * S;
    for (int r = 0; r < n_rows; ++r) {
        if (tid == 0) {
            float a = 0.0f;
            pre[0] = 0.0f;
            for (int c = 0; c < n; ++c) {
                a += pk[(int64_t)r * n + c];
                pre[c + 1] = a;
            }
        }
        if (r > 0) {
            // suffix minima over R' >= b for each L' (thread per L')
            for (int l = tid; l < W; l += blockDim.x) {
                float m = INFINITY;
                for (int b = n; b >= 0; --b) {
                    if (b >= l) m = fminf(m, cur[tri_index(l, b, n)]);
                    grid[l * W + b] = m;
                }
            }
            __syncthreads();
            // prefix minima over L' <= a (thread per b)
            for (int b = tid; b < W; b += blockDim.x) {
                float m = INFINITY;
                for (int a = 0; a < W; ++a) {
                    m = fminf(m, grid[a * W + b]);
                    grid[a * W + b] = m;
                }
            }
        }
        __syncthreads();
        for (int s = tid; s < S; s += blockDim.x) {
            // decode s -> (Lo, Ro)
            int Lo = 0, off = 0;
            while (off + (n + 1 - Lo) <= s) { off += n + 1 - Lo; ++Lo; }
            const int Ro = Lo + (s - off);
            float v = pre[Ro] - pre[Lo];
            if (r > 0) v += grid[Ro * W + Lo];
            if (win) {
                const Window w = row_window(win, (int64_t)k * n_rows + r, n);
                if (Lo < w.lmin || Lo > w.lmax || Ro < w.rmin || Ro > w.rmax) v = INFINITY;   // outside the leaf window
            }
            cur[s] = v;
            hk[(int64_t)r * S + s] = v;
        }
        __syncthreads();
    }
    // best final state: smallest value, then smallest index
    float bv = INFINITY;
    int bi = S;
    for (int s = tid; s < S; s += blockDim.x)
        if (cur[s] < bv) { bv = cur[s]; bi = s; }
    rv[tid] = bv;
    ri[tid] = bi;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (tid < o) {
            const float v2 = rv[tid + o];
            const int i2 = ri[tid + o];
            if (v2 < rv[tid] || (v2 == rv[tid] && i2 < ri[tid])) { rv[tid] = v2; ri[tid] = i2; }
        }
        __syncthreads();
    }
    // state = the final row's best state, or -1 when no aperture fits the
    // leaf windows; every wave tests it, not rv[0], which the first wave to
    // reach the backtracking below may already be overwriting
    __shared__ int state;
    if (tid == 0) {
        cp_price[k] = rv[0];
        state = rv[0] < INFINITY ? ri[0] : -1;
    }
    __syncthreads();
    if (state < 0) {                                 // no aperture fits the leaf windows
        for (int r = tid; r < n_rows; r += blockDim.x) {
            L[(int64_t)k * n_rows + r] = 0;
            R[(int64_t)k * n_rows + r] = 0;
        }
        return;
    }
    for (int r = n_rows - 1; r >= 0; --r) {
        const int s = state;
        int Ls = 0, off = 0;
        while (off + (n + 1 - Ls) <= s) { off += n + 1 - Ls; ++Ls; }
        const int Rs = Ls + (s - off);
        if (tid == 0) {
            L[(int64_t)k * n_rows + r] = Ls;
            R[(int64_t)k * n_rows + r] = Rs;
        }
        if (r == 0) break;
        // smallest-index compatible state of row r-1 with the minimal value
        float v = INFINITY;
        int vi = S;
        for (int q = tid; q < S; q += blockDim.x) {
            int Lq = 0, oq = 0;
            while (oq + (n + 1 - Lq) <= q) { oq += n + 1 - Lq; ++Lq; }
            const int Rq = Lq + (q - oq);
            if (Lq <= Rs && Ls <= Rq) {
                const float hv = hk[(int64_t)(r - 1) * S + q];
                if (hv < v) { v = hv; vi = q; }
            }
        }
        rv[tid] = v;
        ri[tid] = vi;
        __syncthreads();
        for (int o = 128; o >= 1; o >>= 1) {
            if (tid < o) {
                const float v2 = rv[tid + o];
                const int i2 = ri[tid + o];
                if (v2 < rv[tid] || (v2 == rv[tid] && i2 < ri[tid])) { rv[tid] = v2; ri[tid] = i2; }
            }
            __syncthreads();
        }
        if (tid == 0) state = ri[0];
        __syncthreads();
    }
}

}  // namespace dvmat

using namespace dvmat;

extern "C" dvmat_status dvmat_aperture_select(dvmat_geom geom, const float* p, const uint8_t* occupied,
                                              const int32_t* leaf_window, int32_t* L, int32_t* R, float* cp_price,
                                              int32_t* best, float* best_price, dvmat_stream stream) {
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
                       leaf_window, L, R, cp_price);
    hipLaunchKernelGGL(select_best_kernel, dim3(1), dim3(256), 0, s, geom.n_cp, cp_price, best, best_price);
    return check_hip(hipGetLastError(), "dvmat_aperture_select launch");
}

extern "C" dvmat_status dvmat_aperture_select_ws_size(dvmat_geom geom, size_t* bytes) {
    if (!bytes) return set_error(DVMAT_E_ARG, "dvmat_aperture_select_ws_size: bytes is NULL");
    if (geom.n_cp < 1 || geom.n_rows < 1 || geom.n_cols < 1 || geom.n_cols > 96)
        return set_error(DVMAT_E_SHAPE, "dvmat_aperture_select_ws_size: geometry %d x %d x %d (n_cols <= 96)",
                         geom.n_cp, geom.n_rows, geom.n_cols);
    const int64_t S = (int64_t)(geom.n_cols + 1) * (geom.n_cols + 2) / 2;
    *bytes = (size_t)geom.n_cp * geom.n_rows * S * sizeof(float);
    return DVMAT_OK;
}

extern "C" dvmat_status dvmat_aperture_select_interdigitated(dvmat_geom geom, const float* p, const uint8_t* occupied,
                                                             const int32_t* leaf_window, int32_t* L, int32_t* R, float* cp_price, int32_t* best,
                                                             float* best_price, void* d_workspace, size_t bytes,
                                                             dvmat_stream stream) {
    size_t need = 0;
    dvmat_status st = dvmat_aperture_select_ws_size(geom, &need);
    if (st) return st;
    if (!p || !L || !R || !cp_price || !best || !best_price || !d_workspace)
        return set_error(DVMAT_E_ARG, "dvmat_aperture_select_interdigitated: NULL argument");
    if (bytes < need)
        return set_error(DVMAT_E_NOMEM, "dvmat_aperture_select_interdigitated: workspace %zu < %zu bytes", bytes, need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int W = geom.n_cols + 1;
    const int S = W * (W + 1) / 2;
    const size_t lds = ((size_t)W * W + S + W) * sizeof(float);
    hipLaunchKernelGGL(select_interdig_kernel, dim3(geom.n_cp), dim3(256), lds, s, geom.n_rows, geom.n_cols, p,
                       occupied, leaf_window, L, R, cp_price, static_cast<float*>(d_workspace));
    hipLaunchKernelGGL(select_best_kernel, dim3(1), dim3(256), 0, s, geom.n_cp, cp_price, best, best_price);
    return check_hip(hipGetLastError(), "dvmat_aperture_select_interdigitated launch");
}

namespace dvmat {

constexpr int kMaxScratchDevices = 64;

// Device address of the scratch array on the current device, looked up once
// per device (with that device current) and kept.
static dvmat_status scratch_address(float** out, const char* fn) {
    static std::mutex mu;
    static float* addr[kMaxScratchDevices] = {};
    int dev = -1;
    dvmat_status st = check_hip(hipGetDevice(&dev), fn);
    if (st) return st;
    if (dev < 0 || dev >= kMaxScratchDevices)
        return set_error(DVMAT_E_ARG, "%s: device %d beyond the %d supported", fn, dev, kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), fn);
        if (st) return st;
        if (!p) return set_error(DVMAT_E_HIP, "%s: no device address for the scratch array", fn);
        addr[dev] = static_cast<float*>(p);
    }
    *out = addr[dev];
    return DVMAT_OK;
}

}  // namespace dvmat

extern "C" dvmat_status dvmat_aperture_select_interdigitated_noalloc(dvmat_geom geom, const float* p,
                                                                     const uint8_t* occupied,
                                                                     const int32_t* leaf_window, int32_t* L,
                                                                     int32_t* R, float* cp_price, int32_t* best,
                                                                     float* best_price, dvmat_stream stream) {
    const char* fn = "dvmat_aperture_select_interdigitated_noalloc";
    size_t need = 0;
    dvmat_status st = dvmat_aperture_select_ws_size(geom, &need);
    if (st) return st;
    if (!p || !L || !R || !cp_price || !best || !best_price) return set_error(DVMAT_E_ARG, "%s: NULL argument", fn);
    if (need > kSelectScratchBytes)
        return set_error(DVMAT_E_NOMEM, "%s: geometry %d x %d x %d needs %zu bytes of scratch, the limit is %zu", fn,
                         geom.n_cp, geom.n_rows, geom.n_cols, need, kSelectScratchBytes);
    float* hist = nullptr;
    st = scratch_address(&hist, fn);
    if (st) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int W = geom.n_cols + 1;
    const int S = W * (W + 1) / 2;
    const size_t lds = ((size_t)W * W + S + W) * sizeof(float);
    // every value a call reads from the scratch is written earlier in the same
    // call (row r's values before row r+1 and the backtracking read them)
    hipLaunchKernelGGL(select_interdig_kernel, dim3(geom.n_cp), dim3(256), lds, s, geom.n_rows, geom.n_cols, p,
                       occupied, leaf_window, L, R, cp_price, hist);
    hipLaunchKernelGGL(select_best_kernel, dim3(1), dim3(256), 0, s, geom.n_cp, cp_price, best, best_price);
    return check_hip(hipGetLastError(), "dvmat_aperture_select_interdigitated_noalloc launch");
}

extern "C" dvmat_status dvmat_leaf_windows(dvmat_geom geom, const uint8_t* occupied, const int32_t* L,
                                           const int32_t* R, int32_t travel, int32_t* leaf_window,
                                           dvmat_stream stream) {
    if (geom.n_cp < 1 || geom.n_rows < 1 || geom.n_cols < 1)
        return set_error(DVMAT_E_SHAPE, "dvmat_leaf_windows: geometry %d x %d x %d", geom.n_cp, geom.n_rows,
                         geom.n_cols);
    if (!occupied || !L || !R || !leaf_window) return set_error(DVMAT_E_ARG, "dvmat_leaf_windows: NULL argument");
    if (travel < 0) return set_error(DVMAT_E_ARG, "dvmat_leaf_windows: travel %d < 0", travel);
    const int64_t n = (int64_t)geom.n_cp * geom.n_rows;
    hipLaunchKernelGGL(leaf_windows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), geom.n_cp, geom.n_rows, geom.n_cols, occupied, L, R,
                       travel, leaf_window);
    return check_hip(hipGetLastError(), "dvmat_leaf_windows launch");
}
