"""Differentiation form: dose as an autograd Function whose backward is the
price kernel, checked against the FP64 oracle and central finite differences
(h = 1e-3) evaluated in the oracle on the dequantised FP16 matrix."""
import numpy as np
import pytest
import torch

from oracle import bb as obb
from oracle import objective as oobj
from oracle import products as oprod
from paper_1503_01721_amd import synth

pytestmark = pytest.mark.gpu

PLAN = synth.PLANS["cp64_bl12x12_vox40"]


@pytest.fixture(scope="module", params=["csr", "panel", "sliced"])
def setup(request):
    assert torch.cuda.is_available()
    from paper_1503_01721_amd import dvmat
    d = synth.generate_ddc(PLAN)
    sid, table = synth.structures(PLAN)
    layout = {} if request.param == "csr" else dict(PLAN.grids, dose_layout=request.param,
                                                            price_layout=request.param)
    ddc = dvmat.DDC(d["row"], d["col"], d["val"], PLAN.n_vox, PLAN.n_bl, storage="f16", **layout)
    assert ddc.info.dose_layout == {"csr": 0, "panel": 1, "sliced": 2}[request.param]
    obj = dvmat.Objective(sid, table)
    cps, L, R = synth.random_apertures(PLAN, 64, 2004)
    aps = dvmat.Apertures(PLAN.n_cp, PLAN.n_rows, PLAN.n_cols, cps, L, R)
    # dequantised matrix, computed here independently of the library
    s = np.zeros(PLAN.n_bl, np.float32)
    np.maximum.at(s, d["col"], np.abs(d["val"]))
    s[s == 0] = 1.0
    deq = (d["val"] / s[d["col"]]).astype(np.float16).astype(np.float64) * s[d["col"]]
    apset = obb.ApertureSet(PLAN.n_cp, PLAN.n_rows, PLAN.n_cols)
    for k in range(64):
        apset.add(cps[k], L[k], R[k])
    # aperture DDC vectors DA_k (Eq. 5) of the dequantised matrix, one pass over COO
    own = apset.owner[d["col"]]
    sel = own >= 0
    DA = np.bincount(own[sel] * PLAN.n_vox + d["row"][sel], weights=deq[sel],
                     minlength=64 * PLAN.n_vox).reshape(64, PLAN.n_vox)
    return dvmat, d, sid, table, ddc, obj, aps, apset, deq, DA


def _y(seed):
    # rates scaled so the mean PTV dose is about the prescription at y = 1
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 1.5, 64)


def test_gradient_matches_oracle_and_finite_differences(setup):
    from paper_1503_01721_amd.autograd import plan_objective
    dvmat, d, sid, table, ddc, obj, aps, apset, deq, DA = setup
    ptv = sid == synth.S_PTV0
    z1 = DA.sum(axis=0)
    scale = 70.0 / z1[ptv].mean()
    y = _y(5) * scale
    yt = torch.tensor(y, dtype=torch.float32, device="cuda", requires_grad=True)
    F = plan_objective(yt, aps, ddc, obj)
    F.backward()
    G = yt.grad.cpu().numpy().astype(np.float64)
    y32 = yt.detach().cpu().numpy().astype(np.float64)
    z = DA.T @ y32
    F_ref = oobj.objective(z, sid, table)
    assert float(F.detach().cpu()[0]) == pytest.approx(F_ref, rel=1e-5)
    # exact gradient in the oracle: G_k = <DA_k, dF/dz>
    G_ref = DA @ oobj.gradient(z, sid, table)
    assert np.abs(G - G_ref).max() <= 1e-4 * np.abs(G_ref).max()
    # central differences, h = 1e-3, z(y +- h e_k) = z +- h DA_k
    h = 1e-3
    G_fd = np.array([(oobj.objective(z + h * DA[k], sid, table) - oobj.objective(z - h * DA[k], sid, table)) / (2 * h)
                     for k in range(64)])
    # on this case the central differences of the FP64 objective match its exact
    # gradient to about 2e-12 (h = 1e-3), so the bound is the exact gradient's
    assert np.abs(G - G_fd).max() <= 1e-4 * np.abs(G_fd).max()


def test_dose_fn_backward_is_price(setup):
    from paper_1503_01721_amd.autograd import DoseFn
    dvmat, d, sid, table, ddc, obj, aps, apset, deq, DA = setup
    x, g = synth.bench_vectors(PLAN.n_bl, PLAN.n_vox, 2005)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    z = DoseFn.apply(xt, ddc)
    z.backward(torch.tensor(g, device="cuda"))
    p_ref = oprod.price(d["row"], d["col"], deq, g, PLAN.n_bl)
    scale = oprod.price(d["row"], d["col"], deq, np.abs(g), PLAN.n_bl).max()
    assert np.abs(xt.grad.cpu().numpy() - p_ref).max() <= 1e-5 * scale
    z_ref = oprod.dose(d["row"], d["col"], deq, x, PLAN.n_vox)
    assert np.abs(z.detach().cpu().numpy() - z_ref).max() <= 1e-5 * z_ref.max()


def test_aperture_maps(setup):
    dvmat, d, sid, table, ddc, obj, aps, apset, deq, DA = setup
    y = _y(6).astype(np.float32)
    x = torch.empty(PLAN.n_bl, device="cuda")
    aps.expand_(torch.tensor(y, device="cuda"), x)
    assert np.array_equal(x.cpu().numpy(), apset.expand(y).astype(np.float32))
    p = np.random.default_rng(7).standard_normal(PLAN.n_bl).astype(np.float32)
    G = torch.empty(64, device="cuda")
    aps.gather_(torch.tensor(p, device="cuda"), G)
    G_ref = apset.gather(p)
    assert np.allclose(G.cpu().numpy(), G_ref, rtol=1e-5, atol=1e-5 * np.abs(p).sum() / 64)


def test_autograd_bb_equals_price_driven_bb(setup):
    from paper_1503_01721_amd.autograd import solve_master_problem
    dvmat, d, sid, table, ddc, obj, aps, apset, deq, DA = setup
    y0 = torch.zeros(64, device="cuda")
    y_a, F_a, flags_a = solve_master_problem(aps, ddc, obj, y0, steps=20, eps_f=0.0, eps_step=0.0)
    # the same solve through the price-driven entry points
    bb = dvmat.BB(PLAN.n_cp, PLAN.n_rows, PLAN.n_cols, 64, max_iter=20, eps_f=0.0, eps_step=0.0)
    for k in range(64):
        bb.add_aperture(int(aps.cps[k]), aps.L[k], aps.R[k], 0.0, float("inf"))
    x = torch.zeros(PLAN.n_bl, device="cuda")
    xd = torch.zeros_like(x)
    z = torch.empty(PLAN.n_vox, device="cuda")
    g = torch.empty_like(z)
    p = torch.empty(PLAN.n_bl, device="cuda")
    F = torch.empty(1, device="cuda")
    curv = torch.empty(1, dtype=torch.float64, device="cuda")
    bb.expand_(x)
    ddc.dose_(x, z, obj, g, F)
    ddc.price_(g, p)
    bb.begin()
    bb.direction_(p, xd)
    ddc.curvature_(xd, obj, z, curv)
    for _ in range(20):
        bb.step_(p, F, curv, x)
        ddc.dose_(x, z, obj, g, F)
        ddc.price_(g, p)
    assert torch.allclose(y_a, bb.y(), rtol=1e-5, atol=1e-6)
    assert flags_a & dvmat.BB_MAX_ITER
    # and the objective went down from y = 0
    F0 = oobj.objective(np.zeros(PLAN.n_vox), sid, table)
    assert float(F_a.cpu()[0]) < F0
