"""Layout autotuner for the DDC products.

The device layout of each orientation has knobs that no formula settles:
panels or sliced panels, the voxel tile of the dose panels, the beamlet tile
of the price panels, the rows per block row (panels) or lanes per row (sliced
panels) of each, the panel column budget and the part size that shares large
panels between workgroups.  tune() builds the matrix once per candidate,
lets the library pick each orientation's launch shape (dvmat_ddc_autotune),
then times the two products exactly as the column-generation loop runs them
(the dose with the objective epilogue writing F and dF/dz, the price of that
gradient, nrhs right-hand sides) and keeps the fastest candidate per
orientation; the panel budget and part size, which both orientations share,
are taken from the candidate with the fastest dose + price.

Results are cached per matrix signature (sizes, entries, storage, grids,
right-hand sides) in a JSON file: DVMAT_TUNE_CACHE names it, else the
package's tuned_layouts.json (the choices measured for the benchmark
workloads, committed with the sources).  layout_for() returns the cached
options or None; the benchmark builds its matrices from them.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional

import torch

from . import dvmat

CACHE_ENV = "DVMAT_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_layouts.json")

# Candidate knobs per storage type.  Dose tiles are voxel bricks (x, y, z);
# 32-voxel rows write whole 128-byte lines of the dose output.  Price tiles are
# (beamlet columns, MLC rows, control points).
def _sl(side, tile, lanes):
    return {side + "_layout": "sliced", side + "_tile": tile, side + "_slice_lanes": lanes, side + "_block_rows": 1}


def _pn(side, tile, B):
    return {side + "_layout": "panel", side + "_tile": tile, side + "_block_rows": B}


DOSE_CANDIDATES = {
    "f32": [_sl("dose", (32, 16, 2), 8), _sl("dose", (32, 16, 2), 4), _sl("dose", (32, 16, 4), 8),
            _sl("dose", (16, 8, 8), 8), _pn("dose", (32, 16, 2), 1)],
    "16bit": [_sl("dose", (16, 8, 8), 4), _sl("dose", (32, 16, 2), 4), _sl("dose", (16, 8, 8), 8),
              _sl("dose", (32, 16, 4), 4), _pn("dose", (16, 8, 8), 2)],
}
PRICE_CANDIDATES = [_sl("price", (4, 2, 8), 8), _sl("price", (4, 2, 8), 16), _sl("price", (8, 2, 4), 8),
                    _sl("price", (4, 4, 4), 4), _pn("price", (4, 2, 8), 1)]
SHARED_CANDIDATES = [dict(panel_cols=8192, part_entries=131072), dict(panel_cols=12288, part_entries=131072),
                     dict(panel_cols=8192, part_entries=196608)]


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or DEFAULT_CACHE


def signature(n_vox: int, n_bl: int, nnz: int, storage: str, grids: dict, nrhs: int = 1) -> str:
    dg, pg = grids.get("dose_grid"), grids.get("price_grid")
    return (f"vox{n_vox}_bl{n_bl}_nnz{nnz}_{storage}_dg{'x'.join(map(str, dg or ()))}"
            f"_pg{'x'.join(map(str, pg or ()))}_rhs{nrhs}")


def _load(path: str) -> Dict[str, dict]:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def layout_for(sig: str, path: Optional[str] = None) -> Optional[dict]:
    """Build options cached for a signature (keyword arguments of dvmat.DDC), or None."""
    entry = _load(path or cache_path()).get(sig)
    if entry is None:
        return None
    opts = dict(entry["options"])
    for k in ("dose_tile", "price_tile"):
        if k in opts:
            opts[k] = tuple(opts[k])
    return opts


def _time_products(ddc, obj, nrhs: int, reps: int) -> tuple:
    dev = ddc.device
    gen = torch.Generator(device=dev).manual_seed(7)
    shape_x = (ddc.n_bl,) if nrhs == 1 else (ddc.n_bl, nrhs)
    shape_z = (ddc.n_vox,) if nrhs == 1 else (ddc.n_vox, nrhs)
    x = torch.rand(shape_x, device=dev, generator=gen)
    z = torch.empty(shape_z, device=dev)
    g = torch.empty(shape_z, device=dev)
    F = torch.empty(nrhs, device=dev)
    p = torch.empty(shape_x, device=dev)
    for _ in range(2):
        ddc.dose_(x, z, obj, g, F)
        ddc.price_(g, p)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_dose = t_price = 0.0
    for _ in range(reps):
        ev[0].record()
        ddc.dose_(x, z, obj, g, F)
        ev[1].record()
        ddc.price_(g, p)
        ev[2].record()
        torch.cuda.synchronize()
        t_dose += ev[0].elapsed_time(ev[1])
        t_price += ev[1].elapsed_time(ev[2])
    return t_dose / reps, t_price / reps


def tune(row, col, val, n_vox: int, n_bl: int, storage: str, grids: dict, obj: "dvmat.Objective",
         nrhs: int = 1, reps: int = 10, path: Optional[str] = None, log=print) -> dict:
    """Time the candidate layouts on this matrix, cache and return the best
    build options (keyword arguments of dvmat.DDC, grids excluded)."""
    dose_c = DOSE_CANDIDATES["f32" if storage == "f32" else "16bit"]
    # each build pairs one dose candidate with one price candidate, then the
    # shared knobs vary around the first pair
    builds: List[dict] = []
    for i in range(max(len(dose_c), len(PRICE_CANDIDATES))):
        builds.append({**dose_c[i % len(dose_c)], **PRICE_CANDIDATES[i % len(PRICE_CANDIDATES)],
                       **SHARED_CANDIDATES[0]})
    for sh in SHARED_CANDIDATES[1:]:
        builds.append({**dose_c[0], **PRICE_CANDIDATES[0], **sh})
    results = []
    for opts in builds:
        t0 = time.perf_counter()
        ddc = dvmat.DDC(row, col, val, n_vox, n_bl, storage=storage, **grids, **opts)
        ddc.autotune(reps=3, obj=obj, nrhs=nrhs)
        td, tp = _time_products(ddc, obj, nrhs, reps)
        info = ddc.info
        results.append(dict(options=opts, dose_ms=round(td, 4), price_ms=round(tp, 4),
                            dose_layout=int(info.dose_layout), price_layout=int(info.price_layout)))
        log(f"[tune] {opts}: dose {td:.4f} ms, price {tp:.4f} ms ({time.perf_counter() - t0:.1f} s)")
        del ddc
        torch.cuda.empty_cache()
    best_d = min(results, key=lambda r: r["dose_ms"])
    best_p = min(results, key=lambda r: r["price_ms"])
    best_s = min(results, key=lambda r: r["dose_ms"] + r["price_ms"])
    chosen = {k: v for k, v in best_d["options"].items() if k.startswith("dose_")}
    chosen.update({k: v for k, v in best_p["options"].items() if k.startswith("price_")})
    chosen.update({k: best_s["options"][k] for k in ("panel_cols", "part_entries")})
    sig = signature(n_vox, n_bl, len(val), storage, grids, nrhs)
    path = path or cache_path()
    cache = _load(path)
    cache[sig] = dict(options=chosen, dose_ms=best_d["dose_ms"], price_ms=best_p["price_ms"],
                      candidates=results, tuned=time.strftime("%Y-%m-%d"))
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    log(f"[tune] chose {chosen} -> {path}")
    return chosen
