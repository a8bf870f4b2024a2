"""Column-generation VMAT optimisation on one GPU, driving libdvmat.

Sec. 2.1: start from z = 0 with no apertures; each iteration prices the
beamlets (Eq. 3), selects the best aperture at an unoccupied control point,
and re-optimises the fluence rates of all chosen apertures (master problem,
Eq. 6) by Barzilai-Borwein steps (Eqs. 7-10).  The paper's GPU workflow keeps
D^T on the devices for the price and forms each aperture's DDC vector on the
CPU (Sec. 2.2.2); here the whole DDC sits in HBM and every master-problem
iteration runs the dose and price products on it.

Per iteration the host reads back one small record (chosen control point,
its price, the solve's flags and F); all other data stays on the device.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import torch

from . import dvmat


@dataclasses.dataclass
class IterationRecord:
    it: int
    cp: int
    best_price: float
    F: float
    flags: int


class ColumnGeneration:
    """Device buffers and handles for one plan."""

    def __init__(self, ddc: dvmat.DDC, obj: dvmat.Objective, n_cp: int, n_rows: int, n_cols: int,
                 max_apertures: Optional[int] = None, bb_steps: int = 50, eps_f: float = 1e-5,
                 eps_step: float = 1e-7, lo: float = 0.0, hi: float = float("inf")):
        if n_cp * n_rows * n_cols != ddc.n_bl:
            raise ValueError("control-point geometry does not match the number of beamlets")
        dev = ddc.device
        self.ddc, self.obj = ddc, obj
        self.n_cp, self.n_rows, self.n_cols = n_cp, n_rows, n_cols
        self.bb_steps = bb_steps
        self.max_apertures = max_apertures or n_cp
        self.lo, self.hi = lo, hi
        self.bb = dvmat.BB(n_cp, n_rows, n_cols, self.max_apertures, max_iter=bb_steps, eps_f=eps_f,
                           eps_step=eps_step, device=dev)
        self.sel = dvmat.ApertureSelector(n_cp, n_rows, n_cols, device=dev)
        f32 = dict(dtype=torch.float32, device=dev)
        self.x = torch.zeros(ddc.n_bl, **f32)
        self.x_dir = torch.zeros(ddc.n_bl, **f32)
        self.p = torch.empty(ddc.n_bl, **f32)
        self.z = torch.empty(ddc.n_vox, **f32)
        self.g = torch.empty(ddc.n_vox, **f32)
        self.F = torch.empty(1, **f32)
        self.curv = torch.empty(1, dtype=torch.float64, device=dev)
        self.records: List[IterationRecord] = []
        # optional HIP-event log of (dose start, dose end = price start, price end)
        # per master-problem iteration; events are recorded on torch's current
        # stream, the stream every library call here is enqueued on
        self.events: Optional[list] = None
        self.iterations = 0
        self.done = False

    def start(self):
        """z = 0 (no apertures): F, dF/dz and the first prices."""
        self.bb.expand_(self.x)                       # all zero: no apertures yet
        self.ddc.dose_(self.x, self.z, self.obj, self.g, self.F)
        self.ddc.price_(self.g, self.p)

    def select(self):
        """Pricing problem, second step (device); returns the selector."""
        return self.sel(self.p, self.bb.occupied_ptr)

    def master_problem(self, steps: Optional[int] = None):
        """BB solve over the current aperture set: begin, the first step
        length's curvature product, then `steps` x (step, dose+objective, price)."""
        steps = self.bb_steps if steps is None else steps
        self.bb.begin()
        self.bb.direction_(self.p, self.x_dir)
        self.ddc.curvature_(self.x_dir, self.obj, self.z, self.curv)
        ev = self.events
        for _ in range(steps):
            self.bb.step_(self.p, self.F, self.curv, self.x)
            if ev is None:
                self.ddc.dose_(self.x, self.z, self.obj, self.g, self.F)
                self.ddc.price_(self.g, self.p)
            else:
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record()
                self.ddc.dose_(self.x, self.z, self.obj, self.g, self.F)
                e[1].record()
                self.ddc.price_(self.g, self.p)
                e[2].record()
                ev.append(e)

    def iteration(self) -> Optional[IterationRecord]:
        """One column-generation iteration; None when no improving aperture is left."""
        if self.done:
            return None
        self.select()
        best, best_price = int(self.sel.best.item()), float(self.sel.best_price.item())
        if best < 0 or self.bb.count >= self.max_apertures:
            self.done = True
            return None
        self.bb.add_aperture(best, self.sel.L[best], self.sel.R[best], self.lo, self.hi)
        self.master_problem()
        rec = IterationRecord(self.iterations, best, best_price, float(self.F.item()), int(self.bb.flags.item()))
        self.records.append(rec)
        self.iterations += 1
        return rec

    def run(self, max_iterations: int) -> List[IterationRecord]:
        self.start()
        for _ in range(max_iterations):
            if self.iteration() is None:
                break
        return self.records
