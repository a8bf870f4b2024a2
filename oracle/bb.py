"""Master problem (Eq. 6) by the Barzilai-Borwein method with subspace bound
handling (Eqs. 7-10), in float64.  Test infrastructure only.

The master problem optimises the fluence rates y_k of the chosen apertures:
    min F(z)  s.t.  z = sum_k DA(A_k) y_k,  y_k in [lo_k, hi_k].
Let G_k = dF/dy_k (the gradient in the aperture domain).  The paper's g_A is
its negative (Eq. 4 defines g = -grad F, and only that sign makes the bound
rules (9)-(10) keep a descent direction).

One iteration, in the order of Sec. 2.2.2 (gradient, step size, update within
the subspace, dose):
  1. G = gradient in the aperture domain at the current y.
  2. Subspace rule, Eqs. (9)-(10): where y_k sits at (or beyond) its lower
     bound and G_k > 0, or at its upper bound and G_k < 0, clamp y_k to the
     bound and zero that component; the masked gradient is Gt.
  3. Step length alpha: the first iteration of a solve has no history, so it
     takes the Cauchy step of the current quadratic piece
         alpha0 = <Gt,Gt> / (2 sum_i w_i(z) (A Gt)_i^2)
     (w_i the active weight of voxel i, A the map y -> z); later iterations
     use Eq. (7) (BB1 = <s,s>/<s,q>) on odd t and Eq. (8) (BB2 = <s,q>/<q,q>)
     on even t, with s = y_t - y_{t-1}, q = Gt_t - Gt_{t-1}.  Eqs. (7)-(8)
     are written with g_A = -G and so are negative; the step is their
     magnitude, taken along -Gt.  If <s,q> <= 0 or the ratio is not finite
     and positive, the previous alpha is reused and a flag is raised.
  4. y <- clip(y - alpha Gt, lo, hi); then the dose z at the new y.
Stopping (Sec. 2.1): relative change of F over the last five iterations
|F_{t-5} - F_t| <= eps_f |F_t|, step max|y_t - y_{t-1}| <= eps_step max(1, max|y_t|),
an all-zero masked gradient, or max_iter iterations.  The paper gives no
values for the two thresholds; a threshold of 0 switches its test off.

The solver is written against two callables so the same steps run in the
paper's DA-form (A = [DA_1 .. DA_m]) and in D-form (A = D B with B the
aperture -> beamlet indicator); the two must agree.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import objective as obj

FLAG_REL_F = 1
FLAG_SMALL_STEP = 2
FLAG_MAX_ITER = 4
FLAG_FALLBACK = 8
FLAG_CONVERGED = 16
FLAG_NONFINITE = 32
STOP_MASK = FLAG_REL_F | FLAG_SMALL_STEP | FLAG_MAX_ITER | FLAG_CONVERGED | FLAG_NONFINITE


@dataclasses.dataclass(frozen=True)
class BBParams:
    max_iter: int = 50
    eps_f: float = 1e-5
    eps_step: float = 1e-7


def mask_gradient(y, G, lo, hi):
    """Eqs. (9)-(10) on G = dF/dy: returns (clamped y, masked gradient Gt)."""
    y = np.clip(np.asarray(y, np.float64), lo, hi)
    Gt = np.array(G, np.float64, copy=True)
    Gt[(y <= lo) & (Gt > 0.0)] = 0.0
    Gt[(y >= hi) & (Gt < 0.0)] = 0.0
    return y, Gt


def cauchy_step(Gt, d, z, sid, table, y):
    """alpha0 = <Gt,Gt> / (2 sum_i w_i(z) d_i^2), d = A Gt.  Returns (alpha, fell_back)."""
    num = float(np.dot(Gt, Gt))
    den = 2.0 * obj.curvature(d, z, sid, table)
    if den > 0.0 and np.isfinite(den) and np.isfinite(num):
        return num / den, False
    gmax = float(np.max(np.abs(Gt)))
    ymax = float(np.max(np.abs(y))) if len(y) else 0.0
    return (ymax if ymax > 0.0 else 1.0) / gmax, True


def solve(apply, adjoint, sid, table, y0, lo, hi, params=BBParams(), record=False):
    """Run the BB master-problem solve from y0.

    apply(y) -> z (dose of the fluence rates), adjoint(gradF) -> G (gradient in
    the aperture domain).  Returns dict(y, z, F, G, flags, iters, hist)."""
    lo = np.broadcast_to(np.asarray(lo, np.float64), np.shape(y0))
    hi = np.broadcast_to(np.asarray(hi, np.float64), np.shape(y0))
    y = np.clip(np.asarray(y0, np.float64), lo, hi)
    z = apply(y)
    F = float(obj.objective(z, sid, table))
    G = adjoint(obj.gradient(z, sid, table))
    F_hist, flags, alpha = [], 0, np.nan
    y_prev = Gt_prev = None
    hist = dict(y=[], alpha=[], F=F_hist)
    t = 0
    for t in range(params.max_iter):
        y, Gt = mask_gradient(y, G, lo, hi)
        F_hist.append(F)
        if record:
            hist["y"].append(y.copy())
        if not np.isfinite(F):
            flags |= FLAG_NONFINITE
            break
        if params.eps_f > 0 and t >= 5 and abs(F_hist[t - 5] - F_hist[t]) <= params.eps_f * abs(F_hist[t]):
            flags |= FLAG_REL_F
            break
        if (params.eps_step > 0 and t >= 1 and
                np.max(np.abs(y - y_prev)) <= params.eps_step * max(1.0, float(np.max(np.abs(y))))):
            flags |= FLAG_SMALL_STEP
            break
        if not np.any(Gt != 0.0):
            flags |= FLAG_CONVERGED
            break
        if t == 0:
            alpha, fb = cauchy_step(Gt, apply(Gt), z, sid, table, y)
            if fb:
                flags |= FLAG_FALLBACK
        else:
            s = y - y_prev
            q = Gt - Gt_prev
            ss, sq, qq = np.dot(s, s), np.dot(s, q), np.dot(q, q)     # float64 scalars: x/0 is inf/nan
            with np.errstate(divide="ignore", invalid="ignore"):
                cand = float(ss / sq if (t % 2 == 1) else sq / qq)
            if sq > 0.0 and np.isfinite(cand) and cand > 0.0:
                alpha = cand
            else:
                flags |= FLAG_FALLBACK
        if record:
            hist["alpha"].append(alpha)
        y_prev, Gt_prev = y, Gt
        y = np.clip(y - alpha * Gt, lo, hi)
        z = apply(y)
        F = float(obj.objective(z, sid, table))
        G = adjoint(obj.gradient(z, sid, table))
    else:
        flags |= FLAG_MAX_ITER
        F_hist.append(F)
        t = params.max_iter
    return dict(y=y, z=z, F=F, G=G, flags=flags, iters=t, hist=hist)


class ApertureSet:
    """Chosen apertures as a beamlet -> aperture owner map (apertures sit at
    distinct control points, so their beamlet sets are disjoint)."""

    def __init__(self, n_cp, n_rows, n_cols):
        self.n_cp, self.n_rows, self.n_cols = n_cp, n_rows, n_cols
        self.n_bl = n_cp * n_rows * n_cols
        self.owner = -np.ones(self.n_bl, np.int64)
        self.cps, self.L, self.R = [], [], []

    @property
    def m(self):
        return len(self.cps)

    def add(self, cp, L, R):
        k = self.m
        base = cp * self.n_rows * self.n_cols
        for r in range(self.n_rows):
            a, b = int(L[r]), int(R[r])
            self.owner[base + r * self.n_cols + a: base + r * self.n_cols + b] = k
        self.cps.append(int(cp))
        self.L.append(np.asarray(L, np.int32).copy())
        self.R.append(np.asarray(R, np.int32).copy())
        return k

    def expand(self, y):
        """x = B y: x_j = y_k for j in aperture k, else 0."""
        y = np.asarray(y, np.float64)
        x = np.zeros(self.n_bl, np.float64)
        sel = self.owner >= 0
        x[sel] = y[self.owner[sel]]
        return x

    def gather(self, p):
        """G = B^T p: G_k = sum of p_j over the beamlets of aperture k."""
        sel = self.owner >= 0
        return np.bincount(self.owner[sel], weights=np.asarray(p, np.float64)[sel],
                           minlength=self.m)


def d_form_ops(row, col, val, n_vox, n_bl, apset):
    """apply/adjoint of the D-form: z = D (B y), G = B^T D^T grad F."""
    from .products import dose, price

    def apply(y):
        return dose(row, col, val, apset.expand(y), n_vox)

    def adjoint(gradF):
        return apset.gather(price(row, col, val, gradF, n_bl))
    return apply, adjoint


def da_form_ops(DA):
    """apply/adjoint of the paper's DA-form (Eq. 6): z = sum_k DA_k y_k, G_k = <DA_k, grad F>.

    DA: [n_vox, m] float64, column k = DA(A_k) of Eq. (5)."""
    DA = np.asarray(DA, np.float64)

    def apply(y):
        return DA @ np.asarray(y, np.float64)

    def adjoint(gradF):
        return DA.T @ gradF
    return apply, adjoint
