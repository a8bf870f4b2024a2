// Master-problem state on the device and the BB update as a workgroup
// routine, shared by the BB kernels and the fused DA-form step.
#pragma once

#include "common.hpp"

#include <cmath>

namespace dvmat {

constexpr uint32_t kStopMask = DVMAT_BB_REL_F | DVMAT_BB_SMALL_STEP | DVMAT_BB_MAX_ITER | DVMAT_BB_CONVERGED |
                               DVMAT_BB_NONFINITE;
constexpr int kFHist = 8;

struct BBState {
    int32_t t;         // iteration counter of the current solve
    uint32_t flags;
    float alpha;       // last step length
    int32_t m;         // apertures in the set
    float F_hist[kFHist];
};

struct BBDev {
    BBState* state;
    int32_t* cp;       // [max_ap]
    int32_t* L;        // [max_ap * n_rows]
    int32_t* R;
    float* lo;         // [max_ap]
    float* hi;
    float* y;
    float* y_prev;
    float* G;
    float* Gt;
    float* Gt_prev;
    int32_t* cp_slot;  // [n_cp] aperture index or -1
    uint8_t* occ;      // [n_cp] 1 where a control point holds an aperture
};

}  // namespace dvmat

struct dvmat_bb_s {
    dvmat_geom geom{};
    int32_t max_ap = 0;
    int32_t m = 0;
    dvmat_bb_params params{};
    std::vector<uint8_t> occupied;   // host mirror of control-point occupancy
    dvmat::BBDev dev{};
};

namespace dvmat {

enum { MODE_DIRECTION = 0, MODE_STEP = 1 };

// Bound rules, step length, stopping tests and the clipped step, run by one
// workgroup of 256 threads (its own launch, or the last workgroup of a fused
// DA-form step).  G from G_ext, else from the state's gathered B.G; F read
// from *Fp by thread 0 after the reductions.
__device__ __forceinline__ void bb_update_block(const BBDev& B, int mode, const float* Fp, const double* curv,
                                                uint32_t* flags_out, dvmat_bb_params prm,
                                                const float* __restrict__ G_ext) {
    __shared__ double r_ss[256], r_sq[256], r_qq[256], r_gg[256];
    __shared__ float r_ds[256], r_y[256], r_g[256];
    __shared__ int r_nz[256];
    __shared__ float s_alpha;
    __shared__ uint32_t s_stop;
    const int tid = threadIdx.x;
    const int t = B.state->t;
    const int m = B.state->m;
    uint32_t flags = B.state->flags;
    if (mode == MODE_STEP && (flags & kStopMask)) {   // solve already stopped: rates stay
        if (tid == 0 && flags_out) *flags_out = flags;
        return;
    }
    // Eqs. (9)-(10) on G = dF/dy (the paper's g_A = -G)
    double ss = 0.0, sq = 0.0, qq = 0.0, gg = 0.0;
    float ds = 0.0f, ymax = 0.0f, gmax = 0.0f;
    int nz = 0;
    for (int k = tid; k < m; k += 256) {
        const float lo = B.lo[k], hi = B.hi[k];
        const float y = fminf(fmaxf(B.y[k], lo), hi);
        const float G = G_ext ? G_ext[k] : B.G[k];
        float gt = G;
        if (y <= lo && G > 0.0f) gt = 0.0f;
        if (y >= hi && G < 0.0f) gt = 0.0f;
        B.y[k] = y;
        B.Gt[k] = gt;
        if (mode == MODE_STEP) {
            nz += gt != 0.0f;
            gg += (double)gt * (double)gt;
            ymax = fmaxf(ymax, fabsf(y));
            gmax = fmaxf(gmax, fabsf(gt));
            if (t >= 1) {
                const double s = (double)y - (double)B.y_prev[k];
                const double q = (double)gt - (double)B.Gt_prev[k];
                ss += s * s;
                sq += s * q;
                qq += q * q;
                ds = fmaxf(ds, fabsf(y - B.y_prev[k]));
            }
        }
    }
    if (mode == MODE_DIRECTION) return;
    r_ss[tid] = ss; r_sq[tid] = sq; r_qq[tid] = qq; r_gg[tid] = gg;
    r_ds[tid] = ds; r_y[tid] = ymax; r_g[tid] = gmax; r_nz[tid] = nz;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (tid < o) {
            r_ss[tid] += r_ss[tid + o];
            r_sq[tid] += r_sq[tid + o];
            r_qq[tid] += r_qq[tid + o];
            r_gg[tid] += r_gg[tid + o];
            r_ds[tid] = fmaxf(r_ds[tid], r_ds[tid + o]);
            r_y[tid] = fmaxf(r_y[tid], r_y[tid + o]);
            r_g[tid] = fmaxf(r_g[tid], r_g[tid + o]);
            r_nz[tid] += r_nz[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const float F = *Fp;
        B.state->F_hist[t % kFHist] = F;
        uint32_t stop = 0;
        if (!isfinite(F)) {
            stop = DVMAT_BB_NONFINITE;
        } else if (prm.eps_f > 0.0f && t >= 5 &&
                   fabs((double)B.state->F_hist[(t - 5) % kFHist] - (double)F) <= (double)prm.eps_f * fabs((double)F)) {
            stop = DVMAT_BB_REL_F;
        } else if (prm.eps_step > 0.0f && t >= 1 && r_ds[0] <= prm.eps_step * fmaxf(1.0f, r_y[0])) {
            stop = DVMAT_BB_SMALL_STEP;
        } else if (r_nz[0] == 0) {
            stop = DVMAT_BB_CONVERGED;
        }
        float alpha = B.state->alpha;
        if (!stop) {
            if (t == 0) {
                const double den = curv ? 2.0 * (*curv) : 0.0;
                if (den > 0.0 && isfinite(den)) {
                    alpha = (float)(r_gg[0] / den);
                } else {
                    alpha = (r_y[0] > 0.0f ? r_y[0] : 1.0f) / r_g[0];
                    flags |= DVMAT_BB_FALLBACK;
                }
            } else {
                const double sqv = r_sq[0];
                const double cand = (t & 1) ? r_ss[0] / sqv : sqv / r_qq[0];
                if (sqv > 0.0 && isfinite(cand) && cand > 0.0) alpha = (float)cand;
                else flags |= DVMAT_BB_FALLBACK;
            }
            if (!isfinite(alpha)) stop = DVMAT_BB_NONFINITE;
        }
        flags |= stop;
        s_alpha = alpha;
        s_stop = stop;
        B.state->alpha = alpha;
    }
    __syncthreads();
    const uint32_t stop = s_stop;
    const float alpha = s_alpha;
    if (!stop) {
        for (int k = tid; k < m; k += 256) {
            const float y = B.y[k];
            const float gt = B.Gt[k];
            B.y_prev[k] = y;
            B.Gt_prev[k] = gt;
            const double yn = (double)y - (double)alpha * (double)gt;
            B.y[k] = fminf(fmaxf((float)yn, B.lo[k]), B.hi[k]);
        }
    }
    if (tid == 0) {
        if (!stop) {
            if (t + 1 >= prm.max_iter) flags |= DVMAT_BB_MAX_ITER;
            B.state->t = t + 1;
        }
        B.state->flags = flags;
        if (flags_out) *flags_out = flags;
    }
}

}  // namespace dvmat
