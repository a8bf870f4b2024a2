"""Invariants of the synthetic workload generator (inputs for both sides)."""
import numpy as np
import pytest

from paper_1503_01721_amd import synth


@pytest.mark.parametrize("name", ["tiny_cp4_bl3x4_vox8", "small_cp8_bl6x6_vox16", "cp20_bl20x20_vox32"])
def test_generator_layout_and_values(name):
    plan = synth.PLANS[name]
    d = synth.generate_ddc(plan)
    row, col, val = d["row"], d["col"], d["val"]
    assert row.dtype == np.int32 and col.dtype == np.int32 and val.dtype == np.float32
    assert row.min() >= 0 and row.max() < plan.n_vox
    assert col.min() >= 0 and col.max() < plan.n_bl
    # kept entries respect the cut and the kernel maximum of 1
    assert val.min() >= np.float32(synth.CUTOFF) and val.max() <= 1.0
    # unique pairs, sorted by (beamlet, voxel)
    key = col.astype(np.int64) * plan.n_vox + row
    assert np.all(np.diff(key) > 0)
    # pointwise definition reproduces every stored value (and zeros elsewhere)
    assert np.array_equal(synth.ddc_entries(plan, row, col), val)
    rng = np.random.default_rng(0)
    vox = rng.integers(0, plan.n_vox, 2000)
    bl = rng.integers(0, plan.n_bl, 2000)
    dense_pick = synth.ddc_entries(plan, vox, bl)
    stored = dict(zip(key.tolist(), val.tolist()))
    for v, b, e in zip(vox.tolist(), bl.tolist(), dense_pick.tolist()):
        assert stored.get(b * plan.n_vox + v, 0.0) == e
    # no entries outside the body cylinder
    sid, table = synth.structures(plan)
    assert np.all(sid[row] != synth.S_OUTSIDE)


def test_plain_method_workload_size():
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    d = synth.generate_ddc(plan)
    assert plan.n_vox == 32768 and plan.n_bl == 8000
    assert 4.5e6 < len(d["val"]) < 5.5e6       # ~5.07 M under this generator


def test_structures_priority_and_table():
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    sid, table = synth.structures(plan)
    counts = np.bincount(sid, minlength=5)
    assert counts[synth.S_PTV0] > 0 and counts[synth.S_OAR_A] > 0 and counts[synth.S_OAR_B] > 0
    assert table.shape == (5, 3)
    assert table[synth.S_PTV0].tolist() == [70.0, 1.0, 1.0]
    assert table[synth.S_OUTSIDE].tolist() == [0.0, 0.0, 0.0]
    # OAR weights: one-sided (no under-dose penalty)
    assert table[synth.S_OAR_A, 2] == 0 and table[synth.S_BODY, 2] == 0


def test_full_scale_control_point_is_reachable():
    # One control point of the 180-angle, 128^3 workload reaches the PTV centre.
    plan = synth.PLANS["cp180_bl40x40_vox128"]
    r, c, v = synth.generate_cp(plan, 45)
    N = plan.n_grid
    centre = ((N // 2) * N + N // 2) * N + N // 2
    assert np.any(r == centre)
    assert 2.0e6 < len(v) < 3.5e6


def test_random_apertures_and_boxes():
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    cps, L, R = synth.random_apertures(plan, 8, 5)
    assert len(set(cps.tolist())) == 8
    assert np.all(L >= 0) and np.all(R <= plan.n_cols) and np.all(L < R)
    lo, hi = synth.random_boxes(8, 5)
    assert np.all(lo >= 0) and np.all(hi > lo)


def test_z_slab_is_the_full_matrix_restricted_to_the_slab():
    """The share of one GPU in a split by voxel rows: generating only slices
    z0 <= iz < z1 gives exactly the full matrix's entries in those rows."""
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    full = synth.generate_ddc(plan)
    N = plan.n_grid
    for z0, z1 in ((8, 12), (0, 4), (28, 32)):
        sl = synth.generate_ddc(plan, z_slab=(z0, z1))
        keep = (full["row"] >= z0 * N * N) & (full["row"] < z1 * N * N)
        for k in ("row", "col", "val"):
            assert np.array_equal(sl[k], full[k][keep]), (z0, k)


def test_slice_counts_and_balanced_slabs():
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    d = synth.generate_ddc(plan)
    N = plan.n_grid
    c = synth.slice_counts(plan)
    assert np.array_equal(c, np.bincount(d["row"] // (N * N), minlength=N))
    for G in (1, 3, 4, 7):
        slabs = synth.balanced_slabs(plan, G, c)
        assert slabs[0][0] == 0 and slabs[-1][1] == N and all(a < b for a, b in slabs)
        assert all(slabs[k][1] == slabs[k + 1][0] for k in range(G - 1))
        share = [c[a:b].sum() for a, b in slabs]
        assert max(share) <= c.sum() / G + c.max()             # within one slice of the ideal


def _lateral_mm(plan, vox, bl):
    """Distance from voxel centres to beamlet central axes, computed here
    from the geometry (beam direction (sin, -cos, 0), u = (cos, sin, 0),
    v = z), independently of the generator's factorisation."""
    N, h = plan.n_grid, plan.vox_mm
    ix, iy, iz = vox % N, (vox // N) % N, vox // (N * N)
    P = np.stack([(ix - (N - 1) / 2) * h, (iy - (N - 1) / 2) * h, (iz - (N - 1) / 2) * h], axis=1)
    c, r, a = bl % plan.n_cols, (bl // plan.n_cols) % plan.n_rows, bl // (plan.n_cols * plan.n_rows)
    th = 2 * np.pi * a / plan.n_cp
    axis_point = np.stack([((c - (plan.n_cols - 1) / 2) * plan.bl_mm) * np.cos(th),
                           ((c - (plan.n_cols - 1) / 2) * plan.bl_mm) * np.sin(th),
                           (r - (plan.n_rows - 1) / 2) * plan.bl_mm], axis=1)
    d = np.stack([np.sin(th), -np.cos(th), np.zeros_like(th)], axis=1)
    w = P - axis_point
    along = (w * d).sum(axis=1)
    return np.linalg.norm(w - along[:, None] * d, axis=1)


@pytest.mark.parametrize("cone", [4.5, 6.0, 7.5])
def test_cone_truncation_keeps_the_complete_entries_within_the_cone(cone):
    """Sec. 2.4 S1: the truncated matrix holds exactly the complete matrix's
    entries of voxels within the cone radius of the beamlet axis, with the
    same values; the pointwise form agrees."""
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    full = synth.generate_ddc(plan)
    tr = synth.generate_ddc(plan, cone_mm=cone)
    dist = _lateral_mm(plan, full["row"].astype(np.int64), full["col"].astype(np.int64))
    inside = dist <= cone
    # margin: entries within 1e-9 mm of the cone surface could round either way
    assert not np.any(np.abs(dist - cone) < 1e-9)
    for k in ("row", "col", "val"):
        assert np.array_equal(tr[k], full[k][inside]), k
    assert 0 < len(tr["val"]) < len(full["val"])
    assert np.array_equal(synth.ddc_entries(plan, tr["row"], tr["col"], cone_mm=cone), tr["val"])
    out = ~inside
    assert not np.any(synth.ddc_entries(plan, full["row"][out], full["col"][out], cone_mm=cone))


def test_cone_wider_than_the_cutoff_reach_changes_nothing():
    """At depth 0 the 1e-3 cut-off reaches sqrt(2 sigma^2 ln 1000) = 11.15 mm
    from the axis: a cone of 11.2 mm drops nothing, and a higher value
    cut-off drops exactly the entries below it."""
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    full = synth.generate_ddc(plan)
    assert np.sqrt(2 * synth.SIGMA_MM ** 2 * np.log(1e3)) == pytest.approx(11.15, abs=0.01)
    wide = synth.generate_ddc(plan, cone_mm=11.2)
    for k in ("row", "col", "val"):
        assert np.array_equal(wide[k], full[k])
    hi = synth.generate_ddc(plan, cutoff=1e-2)
    keep = full["val"] >= np.float32(1e-2)
    # stored values are float32 roundings of the float64 entries tested against the cut
    assert abs(len(hi["val"]) - int(keep.sum())) <= 8
    assert hi["val"].min() >= np.float32(1e-2) * (1 - 1e-6)
