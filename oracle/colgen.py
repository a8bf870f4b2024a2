"""The column-generation loop of Sec. 2.1, in float64.  Test infrastructure only.

Start from z = 0 and no apertures.  Each iteration solves the pricing problem
(beamlet prices, Eq. 3, then the best aperture at an unoccupied control
point) and, if that aperture can still lower F, adds it and re-solves the
master problem (Eq. 6) for the fluence rates of all chosen apertures.

Readings where the paper is silent: a new aperture starts at its lower bound
and the other rates keep their values (warm start); the loop stops when the
best aperture price is >= 0, when every control point is occupied, or after
max_cg iterations; the prices used by the next pricing step are those at the
master problem's final iterate.  Options: the interdigitation constraint
(Sec. 2.2.2) and leaf windows from the apertures at occupied neighbouring
control points (Sec. 2.1, maximum leaf travel per control-point step; the
readings are in aperture.py); the machine model of Eq. (2), which sets the
leaf travel and, after each new aperture, every aperture's rate box (Eq. 6;
readings in machine.py).
"""
from __future__ import annotations

import numpy as np

from . import aperture as ap
from . import bb
from . import machine as mach
from . import objective as obj
from . import products


def select_aperture(p, n_cp, n_rows, n_cols, occupied, L_all, R_all, interdigitated=False, leaf_travel=None):
    """The aperture selection of one iteration under the chosen constraints."""
    windows = None
    if leaf_travel is not None:
        windows = ap.leaf_windows(n_cp, n_rows, n_cols, occupied, L_all, R_all, leaf_travel)
    if interdigitated:
        return ap.select_interdigitated(p, n_cp, n_rows, n_cols, occupied, windows)
    if windows is not None:
        return ap.select_windowed(p, n_cp, n_rows, n_cols, occupied, windows)
    return ap.select(p, n_cp, n_rows, n_cols, occupied)


def run(row, col, val, n_vox, n_cp, n_rows, n_cols, sid, table, max_cg,
        params=bb.BBParams(), lo=0.0, hi=np.inf, form="D", interdigitated=False, leaf_travel=None,
        machine=None):
    """Returns dict(apertures=[(cp, L, R)], y, z, F, log=[per-iteration dicts]).
    With a machine model the boxes come from it and lo, hi are unused."""
    if machine is not None:
        t = mach.leaf_travel(machine, n_cols)
        leaf_travel = t if leaf_travel is None else min(leaf_travel, t)
    n_bl = n_cp * n_rows * n_cols
    apset = bb.ApertureSet(n_cp, n_rows, n_cols)
    occupied = np.zeros(n_cp, bool)
    y = np.zeros(0)
    z = np.zeros(n_vox)
    p = products.price(row, col, val, obj.gradient(z, sid, table), n_bl)
    log = []
    DA_cols = []
    L_all = np.zeros((n_cp, n_rows), np.int32)
    R_all = np.zeros((n_cp, n_rows), np.int32)
    for it in range(max_cg):
        sel = select_aperture(p, n_cp, n_rows, n_cols, occupied, L_all, R_all, interdigitated, leaf_travel)
        if sel["best"] < 0:
            break
        k = sel["best"]
        occupied[k] = True
        L_all[k], R_all[k] = sel["L"][k], sel["R"][k]
        apset.add(k, sel["L"][k], sel["R"][k])
        if machine is not None:
            _, lo_cp, hi_cp = mach.boxes(machine, occupied, L_all, R_all)
            lo_k, hi_k = lo_cp[apset.cps], hi_cp[apset.cps]
        else:
            lo_k, hi_k = np.full(apset.m, lo), np.full(apset.m, hi)
        y = np.append(y, lo_k[-1])
        if form == "DA":
            member = apset.owner == apset.m - 1
            DA_cols.append(products.aperture_ddc(row, col, val, member, n_vox))
            apply, adjoint = bb.da_form_ops(np.stack(DA_cols, axis=1))
        else:
            apply, adjoint = bb.d_form_ops(row, col, val, n_vox, n_bl, apset)
        m = apset.m
        res = bb.solve(apply, adjoint, sid, table, y, lo_k, hi_k, params)
        y, z = res["y"], res["z"]
        p = products.price(row, col, val, obj.gradient(z, sid, table), n_bl)
        log.append(dict(it=it, cp=k, best_price=sel["best_price"], F=res["F"],
                        flags=res["flags"], bb_iters=res["iters"]))
    return dict(apertures=list(zip(apset.cps, apset.L, apset.R)), y=y, z=z,
                F=float(obj.objective(z, sid, table)), log=log, price=p, L=L_all, R=R_all,
                occupied=occupied)
