"""Differentiation form: the dose as a torch.autograd.Function.

The master problem (Eq. 6) minimises F(z) with z = D B y over the fluence
rates y of the chosen apertures; its gradient dF/dy = B^T D^T dF/dz is what
the paper's first BB step computes by hand (Sec. 2.2.2, Eqs. 3-5).  Here each
factor is an autograd node whose backward is the adjoint HIP kernel:

    y --ApertureFluence--> x = B y --Dose--> z = D x --Objective--> F(z)
         backward: G = B^T gx       backward: gx = D^T gz (price kernel)
                                               backward: gz = dF/dz * gF

so loss.backward() yields dF/dy, which drives the device-resident BB solver
(dvmat_bb_step_g).
"""
from __future__ import annotations

import torch

from . import dvmat


class DoseFn(torch.autograd.Function):
    """z = D x; backward is the price product D^T (the SpMV^T kernel)."""

    @staticmethod
    def forward(ctx, x, ddc: dvmat.DDC):
        ctx.ddc = ddc
        return ddc.dose(x.contiguous())

    @staticmethod
    def backward(ctx, gz):
        return ctx.ddc.price(gz.contiguous()), None


class ApertureFluenceFn(torch.autograd.Function):
    """x = B y (fluence of the chosen apertures); backward G = B^T gx."""

    @staticmethod
    def forward(ctx, y, aps: dvmat.Apertures):
        ctx.aps = aps
        x = torch.empty(aps.n_bl, dtype=torch.float32, device=y.device)
        aps.expand_(y.contiguous(), x)
        return x

    @staticmethod
    def backward(ctx, gx):
        G = torch.empty(ctx.aps.m, dtype=torch.float32, device=gx.device)
        ctx.aps.gather_(gx.contiguous(), G)
        return G, None


class ObjectiveFn(torch.autograd.Function):
    """F(z) of Eq. (1) (a 1-element tensor); the gradient dF/dz comes from the
    same objective kernel and is saved for backward."""

    @staticmethod
    def forward(ctx, z, obj: dvmat.Objective):
        F, g = obj(z.contiguous(), with_grad=True)
        ctx.save_for_backward(g)
        return F

    @staticmethod
    def backward(ctx, gF):
        (g,) = ctx.saved_tensors
        return g * gF, None


def plan_objective(y, aps: dvmat.Apertures, ddc: dvmat.DDC, obj: dvmat.Objective):
    """F(D B y) as a differentiable function of the aperture rates y."""
    return ObjectiveFn.apply(DoseFn.apply(ApertureFluenceFn.apply(y, aps), ddc), obj)


def solve_master_problem(aps: dvmat.Apertures, ddc: dvmat.DDC, obj: dvmat.Objective, y0, lo=0.0,
                         hi=float("inf"), steps=50, eps_f=1e-5, eps_step=1e-7):
    """BB master-problem solve driven by autograd gradients dF/dy.

    The step rules (Eqs. 7-10) run in the library's BB state; each iteration
    evaluates F and dF/dy through the autograd graph above.  Returns (y, F, flags)."""
    dev = y0.device
    n_cp, n_rows, n_cols = aps.geom.n_cp, aps.geom.n_rows, aps.geom.n_cols
    bb = dvmat.BB(n_cp, n_rows, n_cols, max(aps.m, 1), max_iter=steps, eps_f=eps_f, eps_step=eps_step,
                  device=dev)
    y0 = y0.detach().to(torch.float32)
    for k in range(aps.m):
        bb.add_aperture(int(aps.cps[k]), aps.L[k], aps.R[k], lo, hi, float(y0[k]))
    x = torch.empty(aps.n_bl, dtype=torch.float32, device=dev)
    x_dir = torch.empty_like(x)
    z = torch.empty(ddc.n_vox, dtype=torch.float32, device=dev)
    curv = torch.empty(1, dtype=torch.float64, device=dev)

    def value_and_grad():
        y = bb.y().clone().requires_grad_(True)
        F = plan_objective(y, aps, ddc, obj)
        F.backward()
        return F.detach(), y.grad.detach().contiguous()

    bb.begin()
    F, G = value_and_grad()
    bb.expand_(x)
    ddc.dose_(x, z)
    bb.direction_g_(G, x_dir)
    ddc.curvature_(x_dir, obj, z, curv)
    for _ in range(steps):
        bb.step_g_(G, F, curv, x)
        F, G = value_and_grad()
    return bb.y(), F, int(bb.flags.item())
