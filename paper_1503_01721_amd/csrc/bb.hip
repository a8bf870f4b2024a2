// Master problem (Eq. 6) by Barzilai-Borwein steps with the subspace bound
// rules, Eqs. (7)-(10); the four steps of Sec. 2.2.2 (gradient in the aperture
// domain, step size, bounded update, dose update) with the dose update done by
// the caller through dvmat_dose on the full matrix.
//
// Device state lives in the caller's workspace; each iteration is three small
// launches: gather G_k = sum_{j in A_k} p_j (one workgroup per aperture, fixed
// reduction order), the update (one workgroup: bound rules, FP64 inner
// products, step length, stopping tests, clipped step), and the expansion of
// the rates to the beamlet fluence x = B y (one thread per beamlet).  The
// aperture count lives on the device as well and every kernel reads it there,
// with grids sized for the largest set: the launches of a solve do not change
// as apertures are added, so a captured graph of them replays for every
// column-generation iteration.
#include "bb_device.hpp"

#include <cmath>
#include <new>

namespace dvmat {

static size_t bb_layout(const dvmat_geom& g, int32_t max_ap, BBDev* dev, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return base ? base + o : nullptr; };
    char* p;
    p = take(sizeof(BBState));                    if (dev) dev->state = reinterpret_cast<BBState*>(p);
    p = take((size_t)max_ap * 4);                 if (dev) dev->cp = reinterpret_cast<int32_t*>(p);
    p = take((size_t)max_ap * g.n_rows * 4);      if (dev) dev->L = reinterpret_cast<int32_t*>(p);
    p = take((size_t)max_ap * g.n_rows * 4);      if (dev) dev->R = reinterpret_cast<int32_t*>(p);
    float** fl[] = {dev ? &dev->lo : nullptr, dev ? &dev->hi : nullptr, dev ? &dev->y : nullptr,
                    dev ? &dev->y_prev : nullptr, dev ? &dev->G : nullptr, dev ? &dev->Gt : nullptr,
                    dev ? &dev->Gt_prev : nullptr};
    for (float** f : fl) {
        p = take((size_t)max_ap * 4);
        if (f) *f = reinterpret_cast<float*>(p);
    }
    p = take((size_t)g.n_cp * 4);                 if (dev) dev->cp_slot = reinterpret_cast<int32_t*>(p);
    p = take((size_t)g.n_cp);                     if (dev) dev->occ = reinterpret_cast<uint8_t*>(p);
    return off;
}

__global__ void bb_init_kernel(BBDev B, int n_cp) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_cp; i += gridDim.x * blockDim.x) {
        B.cp_slot[i] = -1;
        B.occ[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        B.state->t = 0;
        B.state->flags = 0;
        B.state->alpha = 0.0f;
        B.state->m = 0;
        for (int i = 0; i < kFHist; ++i) B.state->F_hist[i] = 0.0f;
    }
}

__global__ void bb_add_kernel(BBDev B, int slot, int cp, int n_rows, const int32_t* dL, const int32_t* dR, float lo,
                              float hi, float y0) {
    for (int r = threadIdx.x; r < n_rows; r += blockDim.x) {
        B.L[(int64_t)slot * n_rows + r] = dL[r];
        B.R[(int64_t)slot * n_rows + r] = dR[r];
    }
    if (threadIdx.x == 0) {
        B.state->m = slot + 1;
        B.cp[slot] = cp;
        B.cp_slot[cp] = slot;
        B.occ[cp] = 1;
        B.lo[slot] = lo;
        B.hi[slot] = hi;
        const float y = fminf(fmaxf(y0, lo), hi);
        B.y[slot] = y;
        B.y_prev[slot] = y;
        B.G[slot] = 0.0f;
        B.Gt[slot] = 0.0f;
        B.Gt_prev[slot] = 0.0f;
    }
}

// Boxes from per-control-point arrays; each rate clipped into its new box.
__global__ void bb_set_boxes_kernel(BBDev B, const float* __restrict__ lo_cp, const float* __restrict__ hi_cp) {
    const int m = B.state->m;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
        const int c = B.cp[k];
        const float lo = lo_cp[c], hi = hi_cp[c];
        B.lo[k] = lo;
        B.hi[k] = hi;
        B.y[k] = fminf(fmaxf(B.y[k], lo), hi);
    }
}

__global__ void bb_begin_kernel(BBDev B) {
    if (threadIdx.x == 0) {
        B.state->t = 0;
        B.state->flags = 0;
        B.state->alpha = 0.0f;
        for (int i = 0; i < kFHist; ++i) B.state->F_hist[i] = 0.0f;
    }
}

// G_k = sum of p over the beamlets of aperture k (one workgroup per aperture).
__global__ __launch_bounds__(256) void bb_gather_kernel(BBDev B, int n_rows, int n_cols, const float* __restrict__ p) {
    __shared__ float s[256];
    const int k = blockIdx.x;
    if (k >= B.state->m) return;                      // grid sized for the largest set
    const int cp = B.cp[k];
    const int64_t base = (int64_t)cp * n_rows * n_cols;
    const int per_cp = n_rows * n_cols;
    float a = 0.0f;
    for (int i = threadIdx.x; i < per_cp; i += 256) {
        const int r = i / n_cols, c = i - r * n_cols;
        if (c >= B.L[(int64_t)k * n_rows + r] && c < B.R[(int64_t)k * n_rows + r]) a += p[base + i];
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) B.G[k] = s[0];
}

// Bound rules, step length, stopping tests and the clipped step (one workgroup).
__global__ __launch_bounds__(256) void bb_update_kernel(BBDev B, int mode, const float* Fp, const double* curv,
                                                        uint32_t* flags_out, dvmat_bb_params prm,
                                                        const float* __restrict__ G_ext) {
    bb_update_block(B, mode, Fp, curv, flags_out, prm, G_ext);
}

// x_j = src_k for beamlet j in aperture k, else 0.
__global__ __launch_bounds__(256) void bb_expand_kernel(BBDev B, int n_rows, int n_cols, int64_t n_bl,
                                                        const float* __restrict__ src, float* __restrict__ x) {
    const int64_t per_cp = (int64_t)n_rows * n_cols;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n_bl; j += (int64_t)gridDim.x * 256) {
        const int cp = (int)(j / per_cp);
        const int rc = (int)(j - (int64_t)cp * per_cp);
        const int r = rc / n_cols, c = rc - r * n_cols;
        const int slot = B.cp_slot[cp];
        float v = 0.0f;
        if (slot >= 0 && c >= B.L[(int64_t)slot * n_rows + r] && c < B.R[(int64_t)slot * n_rows + r]) v = src[slot];
        x[j] = v;
    }
}

__global__ void bb_copy_y_kernel(BBDev B, float* y) {
    const int m = B.state->m;
    for (int k = threadIdx.x; k < m; k += blockDim.x) y[k] = B.y[k];
}

// x = B y for an explicit aperture list: one workgroup per control point finds
// the aperture sitting there (if any) and writes all of the point's beamlets.
__global__ __launch_bounds__(256) void aperture_expand_kernel(int n_rows, int n_cols, int m,
                                                              const int32_t* __restrict__ cps,
                                                              const int32_t* __restrict__ L,
                                                              const int32_t* __restrict__ R,
                                                              const float* __restrict__ y, float* __restrict__ x) {
    __shared__ int slot;
    const int cp = blockIdx.x;
    if (threadIdx.x == 0) slot = -1;
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += blockDim.x)
        if (cps[k] == cp) atomicMax(&slot, k);      // distinct control points: at most one match
    __syncthreads();
    const int s = slot;
    const int per_cp = n_rows * n_cols;
    float* xc = x + (int64_t)cp * per_cp;
    for (int i = threadIdx.x; i < per_cp; i += blockDim.x) {
        const int r = i / n_cols, c = i - r * n_cols;
        float v = 0.0f;
        if (s >= 0 && c >= L[(int64_t)s * n_rows + r] && c < R[(int64_t)s * n_rows + r]) v = y[s];
        xc[i] = v;
    }
}

// G_k = sum of p over the beamlets of aperture k (explicit aperture list).
__global__ __launch_bounds__(256) void aperture_gather_kernel(int n_rows, int n_cols, const int32_t* __restrict__ cps,
                                                              const int32_t* __restrict__ L,
                                                              const int32_t* __restrict__ R,
                                                              const float* __restrict__ p, float* __restrict__ G) {
    __shared__ float s[256];
    const int k = blockIdx.x;
    const int64_t base = (int64_t)cps[k] * n_rows * n_cols;
    const int per_cp = n_rows * n_cols;
    float a = 0.0f;
    for (int i = threadIdx.x; i < per_cp; i += 256) {
        const int r = i / n_cols, c = i - r * n_cols;
        if (c >= L[(int64_t)k * n_rows + r] && c < R[(int64_t)k * n_rows + r]) a += p[base + i];
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) G[k] = s[0];
}

static dvmat_status check_geom(const dvmat_geom& g, const char* fn) {
    if (g.n_cp < 1 || g.n_rows < 1 || g.n_cols < 1)
        return set_error(DVMAT_E_SHAPE, "%s: geometry %d x %d x %d", fn, g.n_cp, g.n_rows, g.n_cols);
    if ((int64_t)g.n_cp * g.n_rows * g.n_cols >= (int64_t(1) << 31))
        return set_error(DVMAT_E_SHAPE, "%s: more than 2^31 beamlets", fn);
    return DVMAT_OK;
}

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

}  // namespace dvmat

using namespace dvmat;

extern "C" {

dvmat_status dvmat_bb_workspace_size(dvmat_geom geom, int32_t max_ap, size_t* bytes) {
    dvmat_status st = check_geom(geom, "dvmat_bb_workspace_size");
    if (st) return st;
    if (!bytes) return set_error(DVMAT_E_ARG, "dvmat_bb_workspace_size: bytes is NULL");
    if (max_ap < 1 || max_ap > geom.n_cp)
        return set_error(DVMAT_E_ARG, "dvmat_bb_workspace_size: max_apertures=%d not in 1..n_cp", max_ap);
    *bytes = bb_layout(geom, max_ap, nullptr, nullptr);
    return DVMAT_OK;
}

dvmat_status dvmat_bb_create(dvmat_geom geom, int32_t max_ap, dvmat_bb_params params, void* ws, size_t bytes,
                             dvmat_stream stream, dvmat_bb* out) {
    if (!out) return set_error(DVMAT_E_ARG, "dvmat_bb_create: out is NULL");
    *out = nullptr;
    size_t need = 0;
    dvmat_status st = dvmat_bb_workspace_size(geom, max_ap, &need);
    if (st) return st;
    if (!ws) return set_error(DVMAT_E_ARG, "dvmat_bb_create: workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return set_error(DVMAT_E_ARG, "dvmat_bb_create: workspace misaligned");
    if (bytes < need) return set_error(DVMAT_E_NOMEM, "dvmat_bb_create: workspace %zu < %zu bytes", bytes, need);
    if (params.max_iter < 1 || !(params.eps_f >= 0.0f) || !(params.eps_step >= 0.0f))
        return set_error(DVMAT_E_ARG, "dvmat_bb_create: bad parameters (max_iter=%d eps_f=%g eps_step=%g)",
                         params.max_iter, params.eps_f, params.eps_step);
    dvmat_bb_s* b = new (std::nothrow) dvmat_bb_s();
    if (!b) return set_error(DVMAT_E_NOMEM, "dvmat_bb_create: host allocation failed");
    b->geom = geom;
    b->max_ap = max_ap;
    b->params = params;
    b->occupied.assign(geom.n_cp, 0);
    bb_layout(geom, max_ap, &b->dev, static_cast<char*>(ws));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(bb_init_kernel, dim3(grid_for(geom.n_cp)), dim3(256), 0, s, b->dev, geom.n_cp);
    st = check_hip(hipGetLastError(), "dvmat_bb_create launch");
    if (st) { delete b; return st; }
    *out = b;
    return DVMAT_OK;
}

void dvmat_bb_destroy(dvmat_bb b) { delete b; }

int32_t dvmat_bb_count(dvmat_bb b) { return b ? b->m : -1; }

dvmat_status dvmat_bb_state(dvmat_bb b, const float** y, const float** gt) {
    if (!b) return set_error(DVMAT_E_ARG, "dvmat_bb_state: NULL handle");
    if (y) *y = b->dev.y;
    if (gt) *gt = b->dev.Gt;
    return DVMAT_OK;
}

dvmat_status dvmat_bb_occupancy(dvmat_bb b, const uint8_t** d_occupied) {
    if (!b || !d_occupied) return set_error(DVMAT_E_ARG, "dvmat_bb_occupancy: NULL argument");
    *d_occupied = b->dev.occ;
    return DVMAT_OK;
}

dvmat_status dvmat_bb_add_aperture(dvmat_bb b, int32_t cp, const int32_t* dL, const int32_t* dR, float lo, float hi,
                                   float y0, dvmat_stream stream) {
    if (!b || !dL || !dR) return set_error(DVMAT_E_ARG, "dvmat_bb_add_aperture: NULL argument");
    if (cp < 0 || cp >= b->geom.n_cp)
        return set_error(DVMAT_E_ARG, "dvmat_bb_add_aperture: control point %d not in [0,%d)", cp, b->geom.n_cp);
    if (std::isnan(lo) || std::isnan(hi) || lo > hi || std::isinf(lo) || std::isnan(y0))
        return set_error(DVMAT_E_ARG, "dvmat_bb_add_aperture: bad box [%g, %g] or y0 %g", lo, hi, y0);
    if (b->occupied[cp]) return set_error(DVMAT_E_STATE, "dvmat_bb_add_aperture: control point %d already occupied", cp);
    if (b->m >= b->max_ap) return set_error(DVMAT_E_STATE, "dvmat_bb_add_aperture: aperture set full (%d)", b->max_ap);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(bb_add_kernel, dim3(1), dim3(256), 0, s, b->dev, b->m, cp, b->geom.n_rows, dL, dR, lo, hi, y0);
    dvmat_status st = check_hip(hipGetLastError(), "dvmat_bb_add_aperture launch");
    if (st) return st;
    b->occupied[cp] = 1;
    b->m++;
    return DVMAT_OK;
}

dvmat_status dvmat_bb_set_boxes(dvmat_bb b, const float* lo_cp, const float* hi_cp, dvmat_stream stream) {
    if (!b || !lo_cp || !hi_cp) return set_error(DVMAT_E_ARG, "dvmat_bb_set_boxes: NULL argument");
    if (b->m == 0) return DVMAT_OK;
    hipLaunchKernelGGL(bb_set_boxes_kernel, dim3((unsigned)((b->max_ap + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), b->dev, lo_cp, hi_cp);
    return check_hip(hipGetLastError(), "dvmat_bb_set_boxes launch");
}

dvmat_status dvmat_bb_begin(dvmat_bb b, dvmat_stream stream) {
    if (!b) return set_error(DVMAT_E_ARG, "dvmat_bb_begin: NULL handle");
    hipLaunchKernelGGL(bb_begin_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), b->dev);
    return check_hip(hipGetLastError(), "dvmat_bb_begin launch");
}

}  // extern "C"

namespace dvmat {
static dvmat_status bb_direction_impl(dvmat_bb b, const float* p, const float* G_ext, float* x_dir,
                                      dvmat_stream stream, const char* fn) {
    if (!b || !(p || G_ext) || !x_dir) return set_error(DVMAT_E_ARG, "%s: NULL argument", fn);
    if (b->m == 0) return set_error(DVMAT_E_STATE, "%s: no apertures", fn);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dvmat_geom& g = b->geom;
    const int64_t n_bl = (int64_t)g.n_cp * g.n_rows * g.n_cols;
    if (!G_ext) hipLaunchKernelGGL(bb_gather_kernel, dim3(b->max_ap), dim3(256), 0, s, b->dev, g.n_rows, g.n_cols, p);
    hipLaunchKernelGGL(bb_update_kernel, dim3(1), dim3(256), 0, s, b->dev, (int)MODE_DIRECTION,
                       (const float*)nullptr, (const double*)nullptr, (uint32_t*)nullptr, b->params, G_ext);
    hipLaunchKernelGGL(bb_expand_kernel, dim3(grid_for(n_bl)), dim3(256), 0, s, b->dev, g.n_rows, g.n_cols, n_bl,
                       (const float*)b->dev.Gt, x_dir);
    return check_hip(hipGetLastError(), fn);
}

static dvmat_status bb_step_impl(dvmat_bb b, const float* p, const float* G_ext, const float* F, const double* curv,
                                 float* x_next, uint32_t* flags, dvmat_stream stream, const char* fn) {
    if (!b || !(p || G_ext) || !F || (!x_next && !G_ext)) return set_error(DVMAT_E_ARG, "%s: NULL argument", fn);
    if (b->m == 0) return set_error(DVMAT_E_STATE, "%s: no apertures", fn);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dvmat_geom& g = b->geom;
    const int64_t n_bl = (int64_t)g.n_cp * g.n_rows * g.n_cols;
    if (!G_ext) hipLaunchKernelGGL(bb_gather_kernel, dim3(b->max_ap), dim3(256), 0, s, b->dev, g.n_rows, g.n_cols, p);
    hipLaunchKernelGGL(bb_update_kernel, dim3(1), dim3(256), 0, s, b->dev, (int)MODE_STEP, F, curv, flags,
                       b->params, G_ext);
    if (x_next)
        hipLaunchKernelGGL(bb_expand_kernel, dim3(grid_for(n_bl)), dim3(256), 0, s, b->dev, g.n_rows, g.n_cols, n_bl,
                           (const float*)b->dev.y, x_next);
    return check_hip(hipGetLastError(), fn);
}
}  // namespace dvmat

extern "C" {

dvmat_status dvmat_bb_direction(dvmat_bb b, const float* p, float* x_dir, dvmat_stream stream) {
    if (!p) return set_error(DVMAT_E_ARG, "dvmat_bb_direction: p is NULL");
    return bb_direction_impl(b, p, nullptr, x_dir, stream, "dvmat_bb_direction");
}

dvmat_status dvmat_bb_direction_g(dvmat_bb b, const float* G, float* x_dir, dvmat_stream stream) {
    if (!G) return set_error(DVMAT_E_ARG, "dvmat_bb_direction_g: G is NULL");
    return bb_direction_impl(b, nullptr, G, x_dir, stream, "dvmat_bb_direction_g");
}

dvmat_status dvmat_bb_step(dvmat_bb b, const float* p, const float* F, const double* curv, float* x_next,
                           uint32_t* flags, dvmat_stream stream) {
    if (!p) return set_error(DVMAT_E_ARG, "dvmat_bb_step: p is NULL");
    return bb_step_impl(b, p, nullptr, F, curv, x_next, flags, stream, "dvmat_bb_step");
}

dvmat_status dvmat_bb_step_g(dvmat_bb b, const float* G, const float* F, const double* curv, float* x_next,
                             uint32_t* flags, dvmat_stream stream) {
    if (!G) return set_error(DVMAT_E_ARG, "dvmat_bb_step_g: G is NULL");
    return bb_step_impl(b, nullptr, G, F, curv, x_next, flags, stream, "dvmat_bb_step_g");
}

dvmat_status dvmat_bb_expand(dvmat_bb b, float* x, dvmat_stream stream) {
    if (!b || !x) return set_error(DVMAT_E_ARG, "dvmat_bb_expand: NULL argument");
    const dvmat_geom& g = b->geom;
    const int64_t n_bl = (int64_t)g.n_cp * g.n_rows * g.n_cols;
    hipLaunchKernelGGL(bb_expand_kernel, dim3(grid_for(n_bl)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       b->dev, g.n_rows, g.n_cols, n_bl, (const float*)b->dev.y, x);
    return check_hip(hipGetLastError(), "dvmat_bb_expand launch");
}

dvmat_status dvmat_aperture_expand(dvmat_geom geom, int32_t m, const int32_t* cps, const int32_t* L, const int32_t* R,
                                   const float* y, float* x, dvmat_stream stream) {
    dvmat_status st = check_geom(geom, "dvmat_aperture_expand");
    if (st) return st;
    if (m < 0 || m > geom.n_cp) return set_error(DVMAT_E_ARG, "dvmat_aperture_expand: m=%d not in 0..n_cp", m);
    if (!x || (m > 0 && (!cps || !L || !R || !y))) return set_error(DVMAT_E_ARG, "dvmat_aperture_expand: NULL argument");
    hipLaunchKernelGGL(aperture_expand_kernel, dim3(geom.n_cp), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       geom.n_rows, geom.n_cols, m, cps, L, R, y, x);
    return check_hip(hipGetLastError(), "dvmat_aperture_expand launch");
}

dvmat_status dvmat_aperture_gather(dvmat_geom geom, int32_t m, const int32_t* cps, const int32_t* L, const int32_t* R,
                                   const float* p, float* G, dvmat_stream stream) {
    dvmat_status st = check_geom(geom, "dvmat_aperture_gather");
    if (st) return st;
    if (m < 0 || m > geom.n_cp) return set_error(DVMAT_E_ARG, "dvmat_aperture_gather: m=%d not in 0..n_cp", m);
    if (m == 0) return DVMAT_OK;
    if (!cps || !L || !R || !p || !G) return set_error(DVMAT_E_ARG, "dvmat_aperture_gather: NULL argument");
    hipLaunchKernelGGL(aperture_gather_kernel, dim3(m), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       geom.n_rows, geom.n_cols, cps, L, R, p, G);
    return check_hip(hipGetLastError(), "dvmat_aperture_gather launch");
}

dvmat_status dvmat_bb_get_y(dvmat_bb b, float* y, dvmat_stream stream) {
    if (!b || !y) return set_error(DVMAT_E_ARG, "dvmat_bb_get_y: NULL argument");
    if (b->m == 0) return DVMAT_OK;
    hipLaunchKernelGGL(bb_copy_y_kernel, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), b->dev, y);
    return check_hip(hipGetLastError(), "dvmat_bb_get_y launch");
}

}  // extern "C"
