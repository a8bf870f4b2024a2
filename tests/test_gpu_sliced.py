"""Parity of the sliced-panel layout (rows of a panel sorted by length, run in
slices of 64 / W rows with W lanes per row) with the FP64 oracle, through the
C ABI.  Tolerances as in test_gpu_parity.py: dose within 1e-5 of the largest
dose, price within 1e-5 of max (D^T |g|), F within 1e-5 relative, the
curvature within 3e-5 relative; 16-bit storage is compared with the oracle on
the dequantised values."""
import numpy as np
import pytest
import torch

from oracle import objective as oobj
from oracle import products as oprod
from paper_1503_01721_amd import synth

pytestmark = pytest.mark.gpu

PLAN1 = synth.PLANS["cp20_bl20x20_vox32"]
TOL = 1e-5


@pytest.fixture(scope="module")
def dv():
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_1503_01721_amd import dvmat
    return dvmat


@pytest.fixture(scope="module")
def plan1(dv):
    d = synth.generate_ddc(PLAN1)
    sid, table = synth.structures(PLAN1)
    return d, sid, table, dv.Objective(sid, table)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bf16_round(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def _dequantised(d, storage, n_bl):
    val = d["val"].astype(np.float64)
    if storage == "f32":
        return val
    s = np.zeros(n_bl, np.float32)
    np.maximum.at(s, d["col"], np.abs(d["val"]))
    s[s == 0] = 1.0
    q = d["val"] / s[d["col"]]
    q = q.astype(np.float16).astype(np.float32) if storage == "f16" else _bf16_round(q)
    return q.astype(np.float64) * s[d["col"]]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("W", [4, 8, 16])
@pytest.mark.parametrize("price_layout,part", [("panel", 131072), ("sliced", 20000)])
def test_sliced_layout_plain_method_workload(dv, plan1, storage, W, price_layout, part):
    """Dose with the objective epilogue, price, curvature, 1, 3 and 8
    right-hand sides (8 in chunks that fit LDS), bitwise repeatability."""
    d, sid, table, obj = plan1
    ddc = dv.DDC(d["row"], d["col"], d["val"], PLAN1.n_vox, PLAN1.n_bl, storage=storage, dose_layout="sliced",
                 price_layout=price_layout, slice_lanes=W, part_entries=part, **PLAN1.grids)
    info = ddc.info
    assert info.dose_layout == 2 and info.dose_slice_lanes == W and info.dose_kernel == 3
    assert info.price_layout == (2 if price_layout == "sliced" else 1)
    val = _dequantised(d, storage, PLAN1.n_bl)
    x = synth.bench_vectors(PLAN1.n_bl, PLAN1.n_vox, 410 + W)[0] * 4.0
    z_ref = oprod.dose(d["row"], d["col"], val, x, PLAN1.n_vox)
    z, g, F = ddc.dose(cuda(x), obj, with_grad=True)
    assert np.abs(z.cpu().numpy() - z_ref).max() <= TOL * z_ref.max()
    F_ref = oobj.objective(z_ref, sid, table)
    assert abs(float(F.cpu()[0]) - F_ref) <= 1e-5 * F_ref
    assert np.allclose(g.cpu().numpy(), oobj.gradient(z.cpu().numpy().astype(np.float64), sid, table),
                       rtol=1e-5, atol=1e-4)
    gz = g.cpu().numpy().astype(np.float64)
    p_ref = oprod.price(d["row"], d["col"], val, gz, PLAN1.n_bl)
    p = ddc.price(g).cpu().numpy()
    assert np.abs(p - p_ref).max() <= TOL * oprod.price(d["row"], d["col"], np.abs(val), np.abs(gz), PLAN1.n_bl).max()
    curv = torch.zeros(1, dtype=torch.float64, device="cuda")
    ddc.curvature_(cuda(x), obj, z, curv)
    c_ref = oobj.curvature(z_ref, z.cpu().numpy().astype(np.float64), sid, table)
    assert abs(float(curv.cpu()[0]) - c_ref) <= 3e-5 * c_ref
    rng = np.random.default_rng(W)
    for nrhs in (3, 8):
        X = rng.random((PLAN1.n_bl, nrhs)).astype(np.float32)
        Z_ref = oprod.dose(d["row"], d["col"], val, X, PLAN1.n_vox)
        assert np.abs(ddc.dose(cuda(X)).cpu().numpy() - Z_ref).max() <= TOL * Z_ref.max()
        G = rng.standard_normal((PLAN1.n_vox, nrhs)).astype(np.float32)
        P_ref = oprod.price(d["row"], d["col"], val, G, PLAN1.n_bl)
        scale = oprod.price(d["row"], d["col"], np.abs(val), np.abs(G), PLAN1.n_bl).max()
        assert np.abs(ddc.price(cuda(G)).cpu().numpy() - P_ref).max() <= TOL * scale
        Zo, Go, Fo = ddc.dose(cuda(X), obj, with_grad=True)
        Fo_ref = np.array([oobj.objective(Z_ref[:, h], sid, table) for h in range(nrhs)])
        assert np.all(np.abs(Fo.cpu().numpy() - Fo_ref) <= 1e-5 * Fo_ref)
    a = ddc.dose(cuda(x), obj, with_grad=True)
    assert torch.equal(a[0], z) and torch.equal(a[1], g) and torch.equal(a[2], F)
    assert torch.equal(ddc.price(g), ddc.price(g))


@pytest.mark.parametrize("wg", [8, 100, 8192])
@pytest.mark.parametrize("W", [4, 16])
def test_sliced_layout_unstructured(dv, wg, W):
    """Greedy panels over a ragged matrix (no grid): empty rows (more than a
    slice of them), a band of long rows, rows of every length near the step
    boundaries 4W, duplicates summed; small parts."""
    rng = np.random.default_rng(95)
    n_vox, n_bl = 2500, 3100
    mask = rng.random((n_vox, n_bl)) < 0.01
    mask[100:140] = rng.random((40, n_bl)) < 0.3
    mask[2000:2300] = False
    mask[:, 50:80] = False
    for i, n in enumerate(range(1, 4 * W * 3 + 2)):     # row 2300 + i: exactly n entries
        mask[2300 + i] = False
        mask[2300 + i, rng.choice(n_bl, n, replace=False)] = True
    r, c = np.nonzero(mask)
    r = np.concatenate([r, r[:100]])
    c = np.concatenate([c, c[:100]])
    v = rng.uniform(0.001, 1, len(r)).astype(np.float32)
    for cap, part in ((2048, 131072), (4096, 3000)):
        ddc = dv.DDC(r, c, v, n_vox, n_bl, dose_layout="sliced", price_layout="sliced", slice_lanes=W,
                     panel_cols=cap, part_entries=part)
        assert (ddc.info.dose_layout, ddc.info.price_layout) == (2, 2)
        ddc.set_kernel("dose", "panel", wg)
        ddc.set_kernel("price", "panel", wg)
        for nrhs in (1, 2, 5):
            X = rng.random((n_bl, nrhs)).astype(np.float32)
            G = rng.standard_normal((n_vox, nrhs)).astype(np.float32)
            x, g = (X[:, 0].copy(), G[:, 0].copy()) if nrhs == 1 else (X, G)
            z_ref = oprod.dose(r, c, v, x, n_vox)
            p_ref = oprod.price(r, c, v, g, n_bl)
            z = ddc.dose(cuda(x)).cpu().numpy()
            assert np.abs(z - z_ref).max() <= TOL * np.abs(z_ref).max()
            assert np.all(z[2000:2300] == 0)
            p = ddc.price(cuda(g)).cpu().numpy()
            assert np.abs(p - p_ref).max() <= TOL * oprod.price(r, c, v, np.abs(g), n_bl).max()


def test_sliced_layout_edges_and_batch_lanes(dv, plan1):
    # an empty matrix, and a single entry
    for r, c, v in ((np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32)),
                    (np.array([7], np.int32), np.array([3], np.int32), np.array([0.5], np.float32))):
        ddc = dv.DDC(r, c, v, 100, 30, dose_layout="sliced", price_layout="sliced")
        z = ddc.dose(torch.ones(30, device="cuda")).cpu().numpy()
        p = ddc.price(torch.ones(100, device="cuda")).cpu().numpy()
        assert np.array_equal(z, oprod.dose(r, c, v, np.ones(30), 100).astype(np.float32))
        assert np.array_equal(p, oprod.price(r, c, v, np.ones(100), 30).astype(np.float32))
    d, _, _, _ = plan1
    sl = dv.DDC(d["row"], d["col"], d["val"], PLAN1.n_vox, PLAN1.n_bl, dose_layout="sliced", price_layout="sliced",
                slice_lanes=8, **PLAN1.grids)
    sl4 = dv.DDC(d["row"], d["col"], d["val"], PLAN1.n_vox, PLAN1.n_bl, dose_layout="sliced", price_layout="sliced",
                 slice_lanes=4, **PLAN1.grids)
    with pytest.raises(dv.DvmatError):                  # a batch's sliced plans share their lanes per row
        dv.Batch([sl, sl4])
    dv.Batch([sl, sl])
    with pytest.raises(dv.DvmatError):
        sl.set_kernel("dose", "row", 1024)
