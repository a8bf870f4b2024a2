"""The truncation study of Sec. 2.4 (S1) and Sec. 3 on the GPU: column
generation on a matrix truncated by a cone about each beamlet axis, the plan
then re-evaluated on the complete matrix ("actual dose"), both checked
against the FP64 oracle from the GPU's own iterates."""
import numpy as np
import pytest
import torch

from oracle import bb as obb
from oracle import objective as oobj
from oracle import products as oprod
from paper_1503_01721_amd import synth

pytestmark = pytest.mark.gpu

PLAN = synth.PLANS["cp20_bl20x20_vox32"]
CONE_MM = 4.5


def test_truncated_plan_reevaluated_on_the_complete_matrix_matches_oracle():
    assert torch.cuda.is_available()
    from paper_1503_01721_amd import dvmat
    from paper_1503_01721_amd.colgen import ColumnGeneration
    full = synth.generate_ddc(PLAN)
    tr = synth.generate_ddc(PLAN, cone_mm=CONE_MM)
    sid, table = synth.structures(PLAN)
    ddc_full = dvmat.DDC(full["row"], full["col"], full["val"], PLAN.n_vox, PLAN.n_bl, **PLAN.grids)
    ddc_tr = dvmat.DDC(tr["row"], tr["col"], tr["val"], PLAN.n_vox, PLAN.n_bl, **PLAN.grids)
    assert ddc_tr.info.nnz == len(tr["val"]) < ddc_full.info.nnz
    obj = dvmat.Objective(sid, table)
    cg = ColumnGeneration(ddc_tr, obj, PLAN.n_cp, PLAN.n_rows, PLAN.n_cols, bb_steps=50, eps_f=0.0, eps_step=0.0)
    cg.start()
    apset = obb.ApertureSet(PLAN.n_cp, PLAN.n_rows, PLAN.n_cols)
    y = np.zeros(0)
    for it in range(6):
        # the prices the selection sees are the truncated matrix's
        z = oprod.dose(tr["row"], tr["col"], tr["val"], apset.expand(y), PLAN.n_vox)
        gz = oobj.gradient(z, sid, table)
        p_ref = oprod.price(tr["row"], tr["col"], tr["val"], gz, PLAN.n_bl)
        scale = oprod.price(tr["row"], tr["col"], tr["val"], np.abs(gz), PLAN.n_bl).max()
        assert np.abs(cg.p.cpu().numpy() - p_ref).max() <= 1e-4 * scale, it
        rec = cg.iteration()
        assert rec is not None
        apset.add(rec.cp, cg.sel.L.cpu().numpy()[rec.cp], cg.sel.R.cpu().numpy()[rec.cp])
        y = cg.bb.y().cpu().numpy().astype(np.float64)
        z_opt = oprod.dose(tr["row"], tr["col"], tr["val"], apset.expand(y), PLAN.n_vox)
        assert rec.F == pytest.approx(oobj.objective(z_opt, sid, table), rel=1e-5), it
    # the final fluence on both matrices: optimised (truncated) and actual (complete) dose
    x = cg.x.cpu().numpy().astype(np.float64)
    assert np.array_equal(x, apset.expand(y))
    z_opt_gpu = cg.z.cpu().numpy()
    z_act_gpu = ddc_full.dose(cg.x).cpu().numpy()
    z_opt = oprod.dose(tr["row"], tr["col"], tr["val"], x, PLAN.n_vox)
    z_act = oprod.dose(full["row"], full["col"], full["val"], x, PLAN.n_vox)
    assert np.abs(z_opt_gpu - z_opt).max() <= 1e-5 * z_opt.max()
    assert np.abs(z_act_gpu - z_act).max() <= 1e-5 * z_act.max()
    # the study's finding: the actual target dose exceeds the optimised one
    ptv = sid == synth.S_PTV0
    shift = z_act[ptv].mean() / z_opt[ptv].mean() - 1.0
    shift_gpu = z_act_gpu[ptv].mean() / z_opt_gpu[ptv].mean() - 1.0
    assert shift > 0.05 and shift_gpu == pytest.approx(shift, abs=1e-5)
    assert np.all(z_act_gpu >= z_opt_gpu - 1e-5 * z_opt.max())
