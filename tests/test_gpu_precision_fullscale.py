"""Error of the storage forms against the FP64 oracle at full size, per structure.

The full-scale single-arc workload (180 control points x 40x40 beamlets, 128^3
voxels, ~5e8 non-zeros) in the sliced panel layout the benchmark times, with values
stored as FP32, FP16 and BF16 (16-bit forms: per-beamlet FP32 scale, FP32
accumulation).  Reference: COO products in FP64 over the whole matrix.
Reported (run with -s): the largest dose error over the voxels of each
structure relative to the maximum dose, and the largest price error relative to
the price's no-cancellation scale max_j (D^T|g|)_j.  Bounds: FP32 1e-5; FP16
2e-3 (its unit roundoff 2^-11 on the non-negative dose terms); BF16 2^-8 (the
worst case of its rounding).
"""
import numpy as np
import pytest
import torch

from oracle import products as oprod
from paper_1503_01721_amd import synth

pytestmark = pytest.mark.gpu
PLAN = synth.PLANS["cp180_bl40x40_vox128"]
NAMES = {synth.S_OUTSIDE: "outside", synth.S_BODY: "body", synth.S_OAR_A: "OAR A", synth.S_OAR_B: "OAR B"}
BOUND = {"f32": 1e-5, "f16": 2e-3, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module")
def reference():
    assert torch.cuda.is_available()
    d = synth.generate_ddc(PLAN)
    sid, _ = synth.structures(PLAN)
    x, g = synth.bench_vectors(PLAN.n_bl, PLAN.n_vox, 1004)
    x = x * 3.0
    z64 = oprod.dose(d["row"], d["col"], d["val"], x, PLAN.n_vox)
    p64 = oprod.price(d["row"], d["col"], d["val"], g, PLAN.n_bl)
    pscale = oprod.price(d["row"], d["col"], d["val"], np.abs(g), PLAN.n_bl).max()
    return d, sid, x, g, z64, p64, pscale


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_fullscale_error_per_structure(reference, storage):
    from paper_1503_01721_amd import dvmat
    d, sid, x, g, z64, p64, pscale = reference
    ddc = dvmat.DDC(d["row"], d["col"], d["val"], PLAN.n_vox, PLAN.n_bl, storage=storage, **PLAN.grids)
    assert ddc.info.dose_layout == 2 and ddc.info.price_layout == 2       # the default with grids: sliced panels
    z = ddc.dose(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    p = ddc.price(torch.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    del ddc
    torch.cuda.empty_cache()
    zmax = z64.max()
    ez = np.abs(z - z64) / zmax
    per = {}
    for s in np.unique(sid):
        name = NAMES.get(int(s), f"PTV {int(s) - synth.S_PTV0}")
        per[name] = float(ez[sid == s].max())
    ep = float(np.abs(p - p64).max() / pscale)
    ep_max = float(np.abs(p - p64).max() / np.abs(p64).max())
    print(f"\n{storage}: dose error / max dose: " + ", ".join(f"{k} {v:.2e}" for k, v in per.items())
          + f"; price error / max D^T|g|: {ep:.2e} (/ max|p|: {ep_max:.2e})")
    assert max(per.values()) <= BOUND[storage]
    assert ep <= BOUND[storage]
