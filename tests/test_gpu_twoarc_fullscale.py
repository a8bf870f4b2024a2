"""Parity past 2^31 stored entries: the two-arc workload (360 control points x
60x60 beamlets of 3.3 mm, 160^3 voxels of 2 mm, 4.35e9 non-zeros) in FP16
storage and the default sliced panel layout, the differentiation form's
configuration.

Slice offsets, panel offsets and slice starts beyond 2^31 are exercised by
the rows and columns sampled at the end of each orientation.  The FP64 oracle
cannot hold the products of a matrix this size quickly, so it checks sampled
outputs one by one from the generator's pointwise definition of D_ij
(independent of the COO arrays and of the library), dequantised exactly as
the storage form defines it (v = fp16(D_ij / s_j) * s_j with s_j the largest
entry of beamlet j), plus properties that hold at any size (adjoint identity,
the objective of the returned dose) and the gradient dF/dy that automatic
differentiation returns for apertures of the 64 random ones."""
import math

import numpy as np
import pytest
import torch

from oracle import objective as oobj
from paper_1503_01721_amd import synth

pytestmark = pytest.mark.gpu
PLAN = synth.PLANS["cp360_bl60x60_vox160"]
TOL = 1e-5
REACH_MM = 11.2          # the 1e-3 cut-off reaches 11.15 mm from a beamlet axis


@pytest.fixture(scope="module")
def twoarc():
    assert torch.cuda.is_available()
    import time
    from paper_1503_01721_amd import dvmat
    t0 = time.perf_counter()
    d = synth.generate_ddc(PLAN)
    nnz = len(d["val"])
    print(f"\n[two-arc] generated {nnz} entries in {time.perf_counter() - t0:.0f} s", flush=True)
    # per-beamlet scale s_j = max_i D_ij: the COO is sorted by beamlet
    starts = np.flatnonzero(np.r_[True, np.diff(d["col"]) != 0])
    s = np.zeros(PLAN.n_bl, np.float32)
    s[d["col"][starts]] = np.maximum.reduceat(d["val"], starts)
    ddc = dvmat.DDC(d["row"], d["col"], d["val"], PLAN.n_vox, PLAN.n_bl, storage="f16", **PLAN.grids)
    del d, starts
    print(f"[two-arc] built and uploaded in {time.perf_counter() - t0:.0f} s", flush=True)
    ddc.autotune(reps=2)
    sid, table = synth.structures(PLAN)
    obj = dvmat.Objective(sid, table)
    return dvmat, ddc, obj, sid, table, nnz, s


def _deq(val, s):
    """FP16 storage of val / s, scaled back, in FP64."""
    q = (val.astype(np.float32) / s.astype(np.float32)).astype(np.float16)
    return q.astype(np.float64) * s.astype(np.float64)


def _column(j, body=synth.body_xy(PLAN)):
    """(voxels, D_ij) of beamlet j: only voxels within reach of its axis are
    evaluated (outside it every entry is below the cut-off)."""
    px, py, pidx = body
    n, nr = PLAN.n_cols, PLAN.n_rows
    c, r, a = j % n, (j // n) % nr, j // (n * nr)
    u_c = (c - (n - 1) / 2.0) * PLAN.bl_mm
    v_r = (r - (nr - 1) / 2.0) * PLAN.bl_mm
    th = synth.cp_angle(PLAN, a)
    pu = px * math.cos(th) + py * math.sin(th)
    strip = pidx[np.abs(pu - u_c) <= REACH_MM]
    zc = synth.axis_centres(PLAN.n_grid, PLAN.vox_mm)
    slices = np.flatnonzero(np.abs(zc - v_r) <= REACH_MM)
    N = PLAN.n_grid
    vox = (slices[:, None] * (N * N) + strip[None, :]).ravel()
    val = synth.ddc_entries(PLAN, vox, np.full(len(vox), j))
    keep = val != 0
    return vox[keep], val[keep]


def test_twoarc_layout_is_past_2_31(twoarc):
    dvmat, ddc, obj, sid, table, nnz, s = twoarc
    info = ddc.info
    assert info.nnz == nnz and nnz > 2 ** 31
    assert info.dose_layout == 2 and info.price_layout == 2 and info.storage == dvmat.F16     # sliced panels
    assert info.nnz_pad_dose > 2 ** 31 and info.nnz_pad_price > 2 ** 31


def test_twoarc_dose_rows_and_objective(twoarc):
    dvmat, ddc, obj, sid, table, nnz, s = twoarc
    x, _ = synth.bench_vectors(PLAN.n_bl, PLAN.n_vox, 1004)
    z, g, F = ddc.dose(torch.from_numpy(x).cuda(), obj, with_grad=True)
    z = z.cpu().numpy().astype(np.float64)
    N = PLAN.n_grid
    centre = ((N // 2) * N + N // 2) * N + N // 2
    rng = np.random.default_rng(21)
    body = np.flatnonzero(sid != synth.S_OUTSIDE)
    last_slab = body[body >= (N - 12) * N * N]         # rows stored at the end of the dose layout
    rows = np.unique(np.r_[rng.choice(body, 10, replace=False), rng.choice(last_slab, 6, replace=False),
                           centre, body[-1], PLAN.n_vox - 1])
    all_bl = np.arange(PLAN.n_bl)
    zmax = 0.0
    for i in rows:
        Di = synth.ddc_entries(PLAN, np.full(PLAN.n_bl, i), all_bl)
        nz = Di != 0
        zi = float(_deq(Di[nz], s[all_bl[nz]]) @ x[nz])
        zi_exact = float(Di[nz].astype(np.float64) @ x[nz])
        zmax = max(zmax, zi)
        assert abs(z[i] - zi) <= TOL * max(zi, 1.0), (i, z[i], zi)         # arithmetic on the stored values
        assert abs(z[i] - zi_exact) <= 2e-3 * max(zi_exact, 1.0), (i, z[i], zi_exact)   # storage
    assert zmax > 0
    F_ref = oobj.objective(z, sid, table)
    assert abs(float(F.cpu()[0]) - F_ref) <= 1e-5 * F_ref
    assert np.allclose(g.cpu().numpy(), oobj.gradient(z, sid, table), rtol=1e-5, atol=1e-4)


def test_twoarc_price_columns_and_adjoint(twoarc):
    dvmat, ddc, obj, sid, table, nnz, s = twoarc
    x, g = synth.bench_vectors(PLAN.n_bl, PLAN.n_vox, 1005)
    p = ddc.price(torch.from_numpy(g).cuda()).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(22)
    per_cp = PLAN.n_rows * PLAN.n_cols
    cols = np.unique(np.r_[rng.choice(PLAN.n_bl, 8, replace=False),
                           rng.integers((PLAN.n_cp - 4) * per_cp, PLAN.n_bl, 6),
                           PLAN.n_bl // 2 + PLAN.n_cols // 2, PLAN.n_bl - 1 - PLAN.n_cols // 2])
    checked = 0
    for j in cols:
        vox, Dj = _column(int(j))
        if len(vox) == 0:
            assert p[j] == 0.0
            continue
        dq = _deq(Dj, np.full(len(Dj), s[j]))
        pj = float(dq @ g[vox])
        scale = float(dq @ np.abs(g[vox]))
        assert abs(p[j] - pj) <= TOL * scale, (j, p[j], pj)
        checked += 1
    assert checked >= 8
    z = ddc.dose(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    lhs, rhs = float(z @ g), float(x.astype(np.float64) @ p)
    assert abs(lhs - rhs) <= 1e-5 * float(np.abs(z) @ np.abs(g))


def test_twoarc_autograd_gradient(twoarc):
    """dF/dy from automatic differentiation (dose forward, price backward) for
    64 random apertures, checked for several of them against
    G_k = sum_{j in A_k} sum_i D_ij dF/dz_i with every column from the
    pointwise definition and dF/dz of the returned dose in FP64."""
    from paper_1503_01721_amd.autograd import plan_objective
    dvmat, ddc, obj, sid, table, nnz, s = twoarc
    cps, L, R = synth.random_apertures(PLAN, 64, 2004)
    aps = dvmat.Apertures(PLAN.n_cp, PLAN.n_rows, PLAN.n_cols, cps, L, R)
    x1 = torch.empty(PLAN.n_bl, device="cuda")
    aps.expand_(torch.ones(64, device="cuda"), x1)
    z1 = ddc.dose(x1).cpu().numpy()
    scale = 70.0 / float(z1[sid == synth.S_PTV0].mean())
    rng = np.random.default_rng(2004)
    y = torch.tensor(rng.uniform(0.5, 1.5, 64) * scale, dtype=torch.float32, device="cuda", requires_grad=True)
    F = plan_objective(y, aps, ddc, obj)
    F.backward()
    G = y.grad.cpu().numpy().astype(np.float64)
    x = torch.empty(PLAN.n_bl, device="cuda")
    aps.expand_(y.detach(), x)
    z = ddc.dose(x).cpu().numpy().astype(np.float64)
    gz = oobj.gradient(z, sid, table)
    assert float(F.detach().cpu()[0]) == pytest.approx(oobj.objective(z, sid, table), rel=1e-5)
    n = PLAN.n_cols
    for k in (0, 31, 63):
        Gk, Sk = 0.0, 0.0
        for r in range(PLAN.n_rows):
            for c in range(int(L[k, r]), int(R[k, r])):
                j = (int(cps[k]) * PLAN.n_rows + r) * n + c
                vox, Dj = _column(j)
                dq = _deq(Dj, np.full(len(Dj), s[j]))
                Gk += float(dq @ gz[vox])
                Sk += float(dq @ np.abs(gz[vox]))
        assert abs(G[k] - Gk) <= 1e-4 * Sk, (k, G[k], Gk, Sk)
