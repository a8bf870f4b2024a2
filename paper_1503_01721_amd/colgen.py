"""Column-generation VMAT optimisation on one GPU, driving libdvmat.

Sec. 2.1: start from z = 0 with no apertures; each iteration prices the
beamlets (Eq. 3), selects the best aperture at an unoccupied control point,
and re-optimises the fluence rates of all chosen apertures (master problem,
Eq. 6) by Barzilai-Borwein steps (Eqs. 7-10).  The paper's GPU workflow keeps
D^T on the devices for the price and forms each aperture's DDC vector on the
CPU (Sec. 2.2.2); here the whole DDC sits in HBM and every master-problem
iteration runs the dose and price products on it.

Two forms of the master problem: "D" runs every BB iteration through the
dose and price products over the whole DDC matrix; "DA" is the paper's own
form (Eq. 6): each chosen aperture's dose vector DA_k = D 1_{A_k} (Eq. 5) is
formed once and the iterations read only those m columns.  Both compute the
same iterates up to rounding.

Aperture options: the interdigitation constraint of the MLC leaves (Sec.
2.2.2) and leaf windows that keep a candidate deliverable after the apertures
already chosen at the neighbouring control points (Sec. 2.1): each leaf within
leaf_travel beamlets of its position there.  A machine model (Eq. 2: gantry
speed and dose-rate ranges, speed change, leaf speed) sets that travel and,
after each new aperture, every aperture's rate box (Eq. 6).

Per iteration the host reads back one small record, in one copy: the chosen
control point and its price, with F and the flags of the latest solve; all
other data stays on the device.  With sync=False an iteration's own F and
flags arrive with the next iteration's read-back (or finish()), so the loop
waits on the device once per iteration.  With graph=True the master problem's
launches are captured once in a HIP graph (per step count) and replayed in
every later iteration: the library keeps the aperture count on the device and
sizes every grid for the largest set, so the captured launches stay valid as
apertures are added.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
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
                 eps_step: float = 1e-7, lo: float = 0.0, hi: float = float("inf"), form: str = "D",
                 interdigitated: bool = False, leaf_travel: Optional[int] = None,
                 machine: Optional[dvmat.Machine] = None, graph: bool = False):
        if form not in ("D", "DA"):
            raise ValueError("form must be 'D' or 'DA'")
        self.form = form
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
        # [chosen control point, its price, F, flags]: written in place by the
        # selection, the dose's objective epilogue and the BB step, read back
        # in one copy per iteration
        self.status = torch.zeros(4, dtype=torch.int32, device=dev)
        self.host_status = torch.zeros(4, dtype=torch.int32, pin_memory=True)
        self._host = self.host_status.numpy()
        self.bb.flags = self.status[3:4]
        self.sel = dvmat.ApertureSelector(n_cp, n_rows, n_cols, device=dev, interdigitated=interdigitated,
                                          best=self.status[0:1], best_price=self.status[1:2].view(torch.float32))
        self.machine = machine
        if machine is not None:
            t = dvmat.machine_leaf_travel(machine, n_cols)
            leaf_travel = t if leaf_travel is None else min(leaf_travel, t)
            self.boxes = tuple(torch.empty(n_cp, dtype=torch.float32, device=dev) for _ in range(3))
        self.leaf_travel = leaf_travel
        if leaf_travel is not None:
            i32 = dict(dtype=torch.int32, device=dev)
            self.ap_L = torch.zeros((n_cp, n_rows), **i32)       # openings of the chosen apertures
            self.ap_R = torch.zeros((n_cp, n_rows), **i32)
            self.windows = torch.empty((n_cp, n_rows, 4), **i32)
        f32 = dict(dtype=torch.float32, device=dev)
        self.x = torch.zeros(ddc.n_bl, **f32)
        self.x_dir = torch.zeros(ddc.n_bl, **f32)
        self.p = torch.empty(ddc.n_bl, **f32)
        self.z = torch.empty(ddc.n_vox, **f32)
        self.g = torch.empty(ddc.n_vox, **f32)
        self.F = self.status[2:3].view(torch.float32)
        self.curv = torch.empty(1, dtype=torch.float64, device=dev)
        if form == "DA":
            # columns over the objective's support only; z and dF/dz elsewhere
            # stay as start() leaves them (zero dose, zero gradient there when
            # the matrix has no entries outside the structures)
            self.da = dvmat.DAColumns(ddc.n_vox, self.max_apertures, device=dev, obj=obj)
            self.G = torch.empty(self.max_apertures, dtype=torch.float32, device=dev)
            self.one = torch.ones(1, dtype=torch.float32, device=dev)
            self.cp_dev = torch.empty(1, dtype=torch.int32, device=dev)
            self.x_ind = torch.empty(ddc.n_bl, dtype=torch.float32, device=dev)
        self.records: List[IterationRecord] = []
        # optional HIP-event log of (dose start, dose end = price start, price end)
        # per master-problem iteration; events are recorded on torch's current
        # stream, the stream every library call here is enqueued on
        self.events: Optional[list] = None
        self.iterations = 0
        self.done = False
        self.graph = graph
        self._graphs: Dict[int, torch.cuda.CUDAGraph] = {}
        self._pending: Optional[IterationRecord] = None

    def start(self):
        """z = 0 (no apertures): F, dF/dz and the first prices."""
        self.bb.expand_(self.x)                       # all zero: no apertures yet
        self.ddc.dose_(self.x, self.z, self.obj, self.g, self.F)
        self.ddc.price_(self.g, self.p)

    def select(self):
        """Pricing problem, second step (device); returns the selector."""
        if self.leaf_travel is None:
            return self.sel(self.p, self.bb.occupied_ptr)
        dvmat.leaf_windows(self.n_cp, self.n_rows, self.n_cols, self.bb.occupied_ptr, self.ap_L, self.ap_R,
                           self.leaf_travel, out=self.windows)
        return self.sel(self.p, self.bb.occupied_ptr, windows=self.windows)

    def _master_problem_da(self, steps):
        # the whole G buffer: the kernels read the aperture count on the device
        G = self.G
        y_ptr, gt_ptr = self.bb.state_ptrs()
        self.bb.begin()
        self.da.eval_(self.obj, y_ptr, G, z=self.z, g=self.g, F=self.F)
        self.bb.direction_g_(G, self.x_dir)
        self.da.curvature_(self.obj, gt_ptr, self.z, self.curv)
        if steps > 0:
            # no beamlet fluence per step: the dose comes from the m columns.
            # Step t uses G, F at y_t: the first from the evaluation above, the
            # next ones from the fused launch (evaluation, then the step)
            self.bb.step_g_(G, self.F, self.curv, None)
            for _ in range(steps - 1):
                self.da.bb_step_(self.bb, self.obj, G, self.F, self.curv)
            self.da.eval_(self.obj, y_ptr, G, z=self.z, g=self.g, F=self.F)
        self.bb.expand_(self.x)                       # the fluence of the final rates
        self.ddc.price_(self.g, self.p)

    def _append_da_column(self, cp):
        """DA of the new aperture: dose of its indicator fluence (Eq. 5)."""
        self.cp_dev.fill_(cp)
        dvmat._check(dvmat.lib.dvmat_aperture_expand(self.sel.geom, 1, dvmat._ptr(self.cp_dev),
                                                     dvmat._ptr(self.sel.L[cp]), dvmat._ptr(self.sel.R[cp]),
                                                     dvmat._ptr(self.one), dvmat._ptr(self.x_ind),
                                                     dvmat._stream()))
        self.da.append_(self.ddc, self.x_ind)

    def master_problem(self, steps: Optional[int] = None):
        """BB solve over the current aperture set: begin, the first step
        length's curvature product, then `steps` x (step, dose+objective, price)."""
        steps = self.bb_steps if steps is None else steps
        if self.graph:
            if self.events is not None:
                raise ValueError("per-launch events cannot be recorded inside a captured graph")
            g = self._graphs.get(steps)
            if g is None:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    self._master_problem_body(steps)
                self._graphs[steps] = g
            g.replay()
            return
        self._master_problem_body(steps)

    def _master_problem_body(self, steps):
        if self.form == "DA":
            return self._master_problem_da(steps)
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

    def _read_status(self):
        """The one device-to-host copy of an iteration: (best control point,
        its price, F and flags of the latest solve)."""
        self.host_status.copy_(self.status, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        h = self._host
        return int(h[0]), float(h[1:2].view(np.float32)[0]), float(h[2:3].view(np.float32)[0]), int(h[3])

    def _complete(self, F, flags):
        if self._pending is not None:
            self._pending.F, self._pending.flags = F, flags
            self._pending = None

    def finish(self):
        """Fill in F and flags of the last iteration run with sync=False."""
        if self._pending is not None:
            _, _, F, flags = self._read_status()
            self._complete(F, flags)

    def iteration(self, sync: bool = True) -> Optional[IterationRecord]:
        """One column-generation iteration; None when no improving aperture is left.
        sync=False leaves the record's F and flags to the next read-back."""
        if self.done:
            return None
        self.select()
        best, best_price, F_prev, flags_prev = self._read_status()
        self._complete(F_prev, flags_prev)
        if best < 0 or self.bb.count >= self.max_apertures:
            self.done = True
            return None
        self.bb.add_aperture(best, self.sel.L[best], self.sel.R[best], self.lo, self.hi)
        if self.leaf_travel is not None:
            self.ap_L[best].copy_(self.sel.L[best])
            self.ap_R[best].copy_(self.sel.R[best])
        if self.machine is not None:
            # the new aperture tightens its neighbours' speed bounds: every box anew
            dvmat.machine_boxes(self.n_cp, self.n_rows, self.n_cols, self.machine, self.bb.occupied_ptr,
                                self.ap_L, self.ap_R, out=self.boxes)
            self.bb.set_boxes(self.boxes[1], self.boxes[2])
        if self.form == "DA":
            self._append_da_column(best)
        elif self.lo > 0.0 or self.machine is not None:
            # the new rate starts at lo, and new boxes may have moved every
            # rate: dose, objective and price at the solve's starting point
            # (with lo = 0 and fixed boxes the fluence is unchanged)
            self.bb.expand_(self.x)
            self.ddc.dose_(self.x, self.z, self.obj, self.g, self.F)
            self.ddc.price_(self.g, self.p)
        self.master_problem()
        rec = IterationRecord(self.iterations, best, best_price, math.nan, 0)
        self._pending = rec
        if sync:
            _, _, F, flags = self._read_status()
            self._complete(F, flags)
        self.records.append(rec)
        self.iterations += 1
        return rec

    def run(self, max_iterations: int, sync: bool = True) -> List[IterationRecord]:
        self.start()
        for _ in range(max_iterations):
            if self.iteration(sync=sync) is None:
                break
        self.finish()
        return self.records
