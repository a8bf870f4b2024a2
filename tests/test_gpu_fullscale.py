"""Parity at full size, in the launch configuration the benchmark times.

The full-scale single-arc workload (180 control points x 40x40 beamlets,
128^3 voxels, ~5e8 non-zeros) is built in the layout the benchmark uses (the
tuner's cached choice), in the panel and in the CSR layout, and autotuned
exactly as bench.py does.  The FP64 oracle cannot run the whole
products quickly, so it checks sampled outputs one by one: each sampled
dose row and price row is formed from the generator's pointwise definition of
D_ij (independent of the COO arrays and of the library), plus properties that
hold at any size (adjoint identity, the objective of the returned dose,
optimality of the selected aperture).
"""
import numpy as np
import pytest
import torch

from oracle import aperture as oap
from oracle import objective as oobj
from paper_1503_01721_amd import synth

pytestmark = pytest.mark.gpu
PLAN = synth.PLANS["cp180_bl40x40_vox128"]
TOL = 1e-5


@pytest.fixture(scope="module", params=["bench", "panel", "csr"])
def full(request):
    assert torch.cuda.is_available()
    from paper_1503_01721_amd import dvmat, tuner
    d = synth.generate_ddc(PLAN)
    sid, table = synth.structures(PLAN)
    obj = dvmat.Objective(sid, table)
    if request.param == "bench":
        layout = dict(PLAN.grids, **(tuner.layout_for(tuner.signature(PLAN.n_vox, PLAN.n_bl, len(d["val"]), "f32",
                                                                      PLAN.grids, 1)) or {}))
    elif request.param == "panel":
        layout = dict(PLAN.grids, dose_layout="panel", price_layout="panel")
    else:
        layout = {}
    ddc = dvmat.DDC(d["row"], d["col"], d["val"], PLAN.n_vox, PLAN.n_bl, **layout)
    assert (ddc.info.dose_layout == 0) == (request.param == "csr")
    nnz = len(d["val"])
    del d
    if request.param == "csr":
        ddc.autotune(reps=3)
    else:
        ddc.autotune(reps=3, obj=obj)
    return dvmat, ddc, obj, sid, table, nnz


def _sample_rows(rng, n, k, must=()):
    return np.unique(np.concatenate([rng.choice(n, k, replace=False), np.asarray(must, np.int64)]))


def test_fullscale_dose_rows_and_objective(full):
    dvmat, ddc, obj, sid, table, nnz = full
    assert ddc.info.nnz == nnz
    x, _ = synth.bench_vectors(PLAN.n_bl, PLAN.n_vox, 1002)
    x = x * 3.0
    z, g, F = ddc.dose(torch.from_numpy(x).cuda(), obj, with_grad=True)
    z = z.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(11)
    N = PLAN.n_grid
    centre = ((N // 2) * N + N // 2) * N + N // 2
    rows = _sample_rows(rng, PLAN.n_vox, 40, must=[0, centre, centre + 1, PLAN.n_vox - 1])
    all_bl = np.arange(PLAN.n_bl)
    zmax = 0.0
    for i in rows:
        Di = synth.ddc_entries(PLAN, np.full(PLAN.n_bl, i), all_bl).astype(np.float64)
        zi = float(Di @ x)
        zmax = max(zmax, zi)
        assert abs(z[i] - zi) <= TOL * max(zi, 1.0), (i, z[i], zi)
    assert zmax > 0
    # the objective and gradient of the returned dose (Eq. 1), in FP64
    F_ref = oobj.objective(z, sid, table)
    assert abs(float(F.cpu()[0]) - F_ref) <= 1e-5 * F_ref
    g_ref = oobj.gradient(z, sid, table)
    assert np.allclose(g.cpu().numpy(), g_ref, rtol=1e-5, atol=1e-4)


def test_fullscale_price_rows_and_adjoint(full):
    dvmat, ddc, obj, sid, table, nnz = full
    x, g = synth.bench_vectors(PLAN.n_bl, PLAN.n_vox, 1003)
    p = ddc.price(torch.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(12)
    cols = _sample_rows(rng, PLAN.n_bl, 24, must=[0, PLAN.n_bl // 2 + 20, PLAN.n_bl - 1])
    all_vox = np.arange(PLAN.n_vox)
    for j in cols:
        Dj = synth.ddc_entries(PLAN, all_vox, np.full(PLAN.n_vox, j)).astype(np.float64)
        pj = float(Dj @ g)
        scale = float(Dj @ np.abs(g))
        assert abs(p[j] - pj) <= TOL * max(scale, 1e-30), (j, p[j], pj)
    # adjoint identity over the whole matrix, from the two products
    z = ddc.dose(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    lhs, rhs = float(z @ g), float(x @ p)
    assert abs(lhs - rhs) <= 1e-5 * float(np.abs(z) @ np.abs(g))


def test_fullscale_aperture_selection(full):
    dvmat, ddc, obj, sid, table, nnz = full
    z, g, F = ddc.dose(torch.zeros(PLAN.n_bl, device="cuda"), obj, with_grad=True)
    p = ddc.price(g)
    out = dvmat.aperture_select(p, PLAN.n_cp, PLAN.n_rows, PLAN.n_cols)
    p64 = p.cpu().numpy().astype(np.float64)
    ref = oap.select(p64, PLAN.n_cp, PLAN.n_rows, PLAN.n_cols, np.zeros(PLAN.n_cp, bool))
    P = p64.reshape(PLAN.n_cp, PLAN.n_rows, PLAN.n_cols)
    L, R = out["L"].cpu().numpy(), out["R"].cpu().numpy()
    bound = 64 * 2.0 ** -24 * np.abs(P).sum(axis=2)
    chosen = np.array([[P[k, r, L[k, r]:R[k, r]].sum() for r in range(PLAN.n_rows)] for k in range(PLAN.n_cp)])
    best_rows = np.array([[P[k, r, ref["L"][k, r]:ref["R"][k, r]].sum() for r in range(PLAN.n_rows)]
                          for k in range(PLAN.n_cp)])
    assert np.all(np.abs(chosen - best_rows) <= bound)
    b = int(out["best"].cpu()[0])
    assert b >= 0 and abs(ref["cp_price"][b] - ref["best_price"]) <= bound.sum(axis=1).max()
