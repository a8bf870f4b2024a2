// Machine constraints of Eq. (2) as the rate boxes of the master problem,
// Eq. (6): y_k in [R^L / S^U_k, R^U / S^L_k].
//
// S^U_k is the largest gantry speed at control point k that the chosen
// apertures allow: the leaf motion from A_k to A_{k+1} must fit in the time
// the gantry needs for one control-point gap (S^U_{k,k+1} of Eq. 2, applied to
// the speed s_k of the arc from k to k+1 when both points hold apertures), and
// the speed changes by at most dS between neighbours along the whole arc.  The
// largest profile under those bounds has the closed form
//     S^U_k = min_j ( U_j + |k - j| dS ),  U_j = min(S^U, S^U_{j,j+1}),
// evaluated here directly (one workgroup; the bounds U_j sit in LDS).  Upper
// bounds never raise the lower one, so S^L_k = S^L.
#include <cmath>
#include <cstdlib>

#include "common.hpp"

using namespace dvmat;

namespace {

constexpr int kMachineThreads = 256;
constexpr int kMachineMaxCp = 8192;   // U_j of every control point in LDS (32 KB)

__global__ __launch_bounds__(kMachineThreads) void machine_boxes_kernel(dvmat_geom g, dvmat_machine m,
                                                                        const uint8_t* __restrict__ occ,
                                                                        const int32_t* __restrict__ L,
                                                                        const int32_t* __restrict__ R,
                                                                        float* __restrict__ s_hi,
                                                                        float* __restrict__ lo,
                                                                        float* __restrict__ hi) {
    extern __shared__ float u[];
    const int K = g.n_cp, nr = g.n_rows;
    for (int k = threadIdx.x; k < K; k += kMachineThreads) {
        float v = m.speed_max;
        if (k + 1 < K && occ[k] && occ[k + 1]) {
            int d = 0;
            const int32_t* l0 = L + (int64_t)k * nr;
            const int32_t* r0 = R + (int64_t)k * nr;
            for (int r = 0; r < nr; ++r) {
                d = max(d, abs(l0[r] - l0[r + nr]));
                d = max(d, abs(r0[r] - r0[r + nr]));
            }
            if (d > 0) v = fminf(v, m.leaf_speed * m.gantry_step / (float)d);
        }
        u[k] = v;
    }
    __syncthreads();
    const float hi_v = m.speed_min > 0.0f ? m.rate_max / m.speed_min : INFINITY;
    for (int k = threadIdx.x; k < K; k += kMachineThreads) {
        float s = u[k];
        for (int j = 0; j < K; ++j)
            if (j != k) s = fminf(s, u[j] + (float)abs(k - j) * m.speed_change);
        s_hi[k] = s;
        lo[k] = m.rate_min / s;
        hi[k] = hi_v;
    }
}

dvmat_status check_machine(const dvmat_machine* m, const char* fn) {
    if (!m) return set_error(DVMAT_E_ARG, "%s: NULL machine", fn);
    const bool ok = m->gantry_step > 0.0f && std::isfinite(m->gantry_step) && m->speed_min >= 0.0f &&
                    std::isfinite(m->speed_min) && m->speed_max > 0.0f && m->speed_max >= m->speed_min &&
                    m->speed_change >= 0.0f && m->rate_min >= 0.0f && std::isfinite(m->rate_min) &&
                    m->rate_max >= m->rate_min && m->leaf_speed > 0.0f;   // NaN fails every comparison
    if (!ok)
        return set_error(DVMAT_E_ARG,
                         "%s: machine out of range (gantry_step %g, speed [%g, %g], speed_change %g, rate [%g, %g], "
                         "leaf_speed %g)",
                         fn, m->gantry_step, m->speed_min, m->speed_max, m->speed_change, m->rate_min, m->rate_max,
                         m->leaf_speed);
    return DVMAT_OK;
}

}  // namespace

extern "C" {

dvmat_status dvmat_machine_leaf_travel(const dvmat_machine* m, int32_t n_cols, int32_t* travel) {
    if (dvmat_status st = check_machine(m, "dvmat_machine_leaf_travel")) return st;
    if (!travel || n_cols < 1) return set_error(DVMAT_E_ARG, "dvmat_machine_leaf_travel: n_cols %d or NULL output", n_cols);
    if (m->speed_min == 0.0f || std::isinf(m->leaf_speed)) {
        *travel = n_cols;
        return DVMAT_OK;
    }
    const double t = std::floor((double)m->leaf_speed * (double)m->gantry_step / (double)m->speed_min);
    *travel = t >= (double)n_cols ? n_cols : (int32_t)t;
    return DVMAT_OK;
}

dvmat_status dvmat_machine_boxes(dvmat_geom geom, const dvmat_machine* m, const uint8_t* occupied, const int32_t* L,
                                 const int32_t* R, float* speed_hi, float* lo, float* hi, dvmat_stream stream) {
    if (dvmat_status st = check_machine(m, "dvmat_machine_boxes")) return st;
    if (geom.n_cp < 1 || geom.n_rows < 1 || geom.n_cols < 1 || geom.n_cp > kMachineMaxCp)
        return set_error(DVMAT_E_SHAPE, "dvmat_machine_boxes: geometry %d x %d x %d (n_cp <= %d)", geom.n_cp,
                         geom.n_rows, geom.n_cols, kMachineMaxCp);
    if (!occupied || !L || !R || !speed_hi || !lo || !hi)
        return set_error(DVMAT_E_ARG, "dvmat_machine_boxes: NULL argument");
    hipLaunchKernelGGL(machine_boxes_kernel, dim3(1), dim3(kMachineThreads), (size_t)geom.n_cp * sizeof(float),
                       reinterpret_cast<hipStream_t>(stream), geom, *m, occupied, L, R, speed_hi, lo, hi);
    return check_hip(hipGetLastError(), "dvmat_machine_boxes launch");
}

}  // extern "C"
