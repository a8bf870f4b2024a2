"""The device layouts as built on the host, checked on the CPU.

The library builds both orientations of D (CSR or panels, block rows, row
order, entry interleaving, panel column lists with 16-bit local indices, work
units) before any device memory is touched.  These tests copy the host-side
arrays out with dvmat_ddc_layout_array, rebuild the dense matrix from them in
NumPy and compare it with the COO input (duplicates summed), and check the
structural invariants the kernels rely on.
"""
import ctypes

import numpy as np
import pytest

from paper_1503_01721_amd import synth

P = ctypes.c_void_p


@pytest.fixture(scope="module")
def dv():
    from paper_1503_01721_amd import dvmat
    return dvmat


def _array(dv, h, orient, which, dtype):
    n = ctypes.c_size_t()
    assert dv.lib.dvmat_ddc_layout_array(h, orient, which, None, 0, ctypes.byref(n)) == 0
    out = np.empty(n.value // np.dtype(dtype).itemsize, dtype)
    if n.value:
        assert dv.lib.dvmat_ddc_layout_array(h, orient, which, out.ctypes.data_as(P), n.value, ctypes.byref(n)) == 0
    return out


def _create(dv, row, col, val, n_vox, n_bl, opts, storage=0):
    row = np.ascontiguousarray(row, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float32)
    h = ctypes.c_void_p()
    code = dv.lib.dvmat_ddc_create_ex(n_vox, n_bl, len(val), row.ctypes.data_as(P), col.ctypes.data_as(P),
                                      val.ctypes.data_as(P), storage, ctypes.byref(opts), ctypes.byref(h))
    assert code == 0, dv.lib.dvmat_last_error()
    info = dv.DdcInfo()
    assert dv.lib.dvmat_ddc_info(h, ctypes.byref(info)) == 0
    return h, info


def _rebuild_sliced(dv, h, info, orient, n_rows, n_cols, scale=None):
    """Dense matrix of a sliced-panel orientation (layout 2) from its arrays,
    plus the invariants the slice kernel relies on."""
    W = info.dose_slice_lanes if orient == 0 else info.price_slice_lanes
    assert W in (4, 8, 16)
    C = 64 // W
    E = 16 // info.value_bytes                            # entries per lane and step
    sptr = _array(dv, h, orient, 0, np.int64)
    col16 = _array(dv, h, orient, 1, np.uint16)
    vals = _array(dv, h, orient, 2, np.float32 if info.value_bytes == 4 else np.uint16)
    first = _array(dv, h, orient, 3, np.int32)
    perm = _array(dv, h, orient, 4, np.int32)
    ulist = _array(dv, h, orient, 5, np.int32)
    pu = _array(dv, h, orient, 6, np.int64)
    pslices = _array(dv, h, orient, 7, np.int32)
    parts = _array(dv, h, orient, 8, np.int32)
    ppan = _array(dv, h, orient, 9, np.int32)
    n_sl = len(sptr) - 1
    assert len(first) == n_sl + 1 and first[0] == 0 and first[-1] == n_rows and np.all(np.diff(first) >= 1)
    assert sptr[0] == 0 and np.all(np.diff(sptr) >= 0) and len(col16) == len(vals) == sptr[-1]
    assert np.array_equal(np.sort(perm), np.arange(n_rows))
    assert pslices[0] == 0 and pslices[-1] == n_sl and np.all(np.diff(pslices) >= 0)
    assert parts[0] == 0 and parts[-1] == n_sl and np.all(np.diff(ppan) >= 0)
    assert np.all(parts[:-1] >= pslices[ppan]) and np.all(parts[1:] <= pslices[ppan + 1])
    D = np.zeros((n_rows, n_cols), np.float64)
    lens = np.zeros(n_rows, np.int64)                     # stored non-zeros per row, for the order checks
    part_start = set(parts[:-1].tolist())
    for p in range(len(pu) - 1):
        u = ulist[pu[p]:pu[p + 1]]
        assert np.all(np.diff(u) > 0)
        prev = None
        for q in range(pslices[p], pslices[p + 1]):
            if q in part_start:
                prev = None                               # rows are sorted within each part
            nr = first[q + 1] - first[q]
            k0, k1 = sptr[q], sptr[q + 1]
            if k1 == k0:
                assert nr <= 64
                continue
            assert nr <= C and (k1 - k0) % (nr * W * E) == 0
            S = (k1 - k0) // (nr * W * E)
            k = np.arange(k1 - k0)
            i = (k // E // W) % nr
            t, w, qq = k // (E * W * nr), (k // E) % W, k % E
            sidx = E * W * t + qq * W + w                 # sorted entry of the row held at k
            rows = perm[first[q] + i]
            loc = col16[k0:k1].astype(np.int64)
            assert len(u) == 0 or np.all(loc < len(u))
            v = vals[k0:k1]
            if info.value_bytes == 2:                     # FP16 codes of D_ij / s_j (beamlet scale s_j)
                v = v.view(np.float16).astype(np.float64) * scale[u[loc] if orient == 0 else rows]
            np.add.at(D, (rows, u[loc] if len(u) else loc), v)
            # a row's columns increase along its sorted entries
            for r in range(nr):
                m = (i == r) & (v != 0)
                order = np.argsort(sidx[m])
                assert np.all(np.diff(u[loc[m]][order]) > 0)
                lens[perm[first[q] + r]] = m.sum()
            # the step count is the longest row's
            longest = max(lens[perm[first[q]:first[q + 1]]])
            assert S == -(-(-(-longest // E)) // W)
            # rows sorted by length, longest first, within the part
            ls = lens[perm[first[q]:first[q + 1]]]
            assert np.all(np.diff(ls) <= 0) and (prev is None or ls[0] <= prev)
            prev = ls[-1]
    return D, 2


def _rebuild(dv, h, info, orient, n_rows, n_cols):
    """Dense matrix of one orientation from its layout arrays, plus invariants."""
    B = info.dose_block_rows if orient == 0 else info.price_block_rows
    layout = info.dose_layout if orient == 0 else info.price_layout
    if layout == 2:
        return _rebuild_sliced(dv, h, info, orient, n_rows, n_cols)
    rowptr = _array(dv, h, orient, 0, np.int64)
    vals = _array(dv, h, orient, 2, np.float32)
    units = _array(dv, h, orient, 3, np.int32)
    perm = _array(dv, h, orient, 4, np.int32)
    n_br = (n_rows + B - 1) // B
    assert len(rowptr) == n_br + 1 and rowptr[0] == 0 and np.all(np.diff(rowptr) % 4 == 0)
    n_pos = rowptr[-1]
    assert len(vals) == n_pos * B
    # work units cover the block rows in order, at most 64 block rows each
    assert units[0] == 0 and units[-1] == n_br and np.all(np.diff(units) >= 1) and np.all(np.diff(units) <= 64)
    if len(perm):
        assert np.array_equal(np.sort(perm), np.arange(n_rows))
    natural = perm if len(perm) else np.arange(n_rows)
    if layout == 1:
        col16 = _array(dv, h, orient, 1, np.uint16)
        ulist = _array(dv, h, orient, 5, np.int32)
        pu = _array(dv, h, orient, 6, np.int64)
        punits = _array(dv, h, orient, 7, np.int32)
        n_pan = len(pu) - 1
        assert n_pan == (info.dose_panels if orient == 0 else info.price_panels)
        assert punits[0] == 0 and punits[-1] == len(units) - 1 and np.all(np.diff(punits) >= 0)
        # parts: runs of units inside one panel, covering every panel in order
        parts = _array(dv, h, orient, 8, np.int32)
        ppan = _array(dv, h, orient, 9, np.int32)
        assert len(parts) == len(ppan) + 1 == (info.dose_panel_parts if orient == 0 else info.price_panel_parts) + 1
        assert parts[0] == 0 and parts[-1] == len(units) - 1 and np.all(np.diff(parts) >= 0)
        assert np.all(np.diff(ppan) >= 0) and np.array_equal(np.unique(ppan), np.arange(n_pan))
        assert np.all(parts[:-1] >= punits[ppan]) and np.all(parts[1:] <= punits[ppan + 1])
        gcol = np.empty(n_pos, np.int64)
        sizes = np.diff(pu)
        assert sizes.max(initial=0) == (info.dose_panel_cols if orient == 0 else info.price_panel_cols)
        for p in range(n_pan):
            u = ulist[pu[p]:pu[p + 1]]
            assert np.all(np.diff(u) > 0) and (len(u) == 0 or (u[0] >= 0 and u[-1] < n_cols))
            k0, k1 = rowptr[units[punits[p]]], rowptr[units[punits[p + 1]]]
            loc = col16[k0:k1].astype(np.int64)
            assert np.all(loc < len(u))
            gcol[k0:k1] = u[loc]
            # every listed column is used by the panel
            assert len(np.unique(gcol[k0:k1])) == len(u)
    else:
        gcol = _array(dv, h, orient, 1, np.int32).astype(np.int64)
        assert len(gcol) == n_pos and (n_pos == 0 or (gcol.min() >= 0 and gcol.max() < n_cols))
    D = np.zeros((n_rows, n_cols), np.float64)
    br_of_pos = np.repeat(np.arange(n_br), np.diff(rowptr))
    for b in range(B):
        stored = br_of_pos * B + b
        ok = stored < n_rows
        np.add.at(D, (natural[stored[ok]], gcol[ok]), vals[np.nonzero(ok)[0] * B + b])
    return D, layout


def _dense(row, col, val, n_vox, n_bl):
    D = np.zeros((n_vox, n_bl), np.float64)
    np.add.at(D, (row, col), val.astype(np.float32).astype(np.float64))
    return D


def _opts(dv, B=(1, 1), layout=(0, 0), grids=None, tiles=None, panel_cols=8192, order=(0, 0), interleave=1,
          part_entries=131072, unit_entries=0, slice_lanes=0):
    o = dv.BuildOpts()
    assert dv.lib.dvmat_ddc_default_opts(0, ctypes.byref(o)) == 0
    o.dose_block_rows, o.price_block_rows = B
    o.dose_layout, o.price_layout = layout
    o.dose_row_order, o.price_row_order = order
    o.interleave = interleave
    o.panel_cols = panel_cols
    o.part_entries = part_entries
    o.unit_entries = unit_entries
    o.dose_slice_lanes = o.price_slice_lanes = slice_lanes
    if grids is not None:
        o.dose_grid[:] = grids["dose_grid"]
        o.price_grid[:] = grids["price_grid"]
        o.dose_tile[:] = tiles[0]
        o.price_tile[:] = tiles[1]
    return o


def _check_both(dv, row, col, val, n_vox, n_bl, opts):
    h, info = _create(dv, row, col, val, n_vox, n_bl, opts)
    try:
        ref = _dense(row, col, val, n_vox, n_bl)
        Dd, lay_d = _rebuild(dv, h, info, 0, n_vox, n_bl)
        Dp, lay_p = _rebuild(dv, h, info, 1, n_bl, n_vox)
        assert np.array_equal(Dd.astype(np.float32), ref.astype(np.float32))
        assert np.array_equal(Dp.astype(np.float32), ref.T.astype(np.float32))
        return info, lay_d, lay_p
    finally:
        dv.lib.dvmat_ddc_destroy(h)


PLAN = synth.PLANS["small_cp8_bl6x6_vox16"]


@pytest.fixture(scope="module")
def small():
    d = synth.generate_ddc(PLAN)
    return d["row"], d["col"], d["val"]


@pytest.mark.parametrize("B", [(1, 1), (2, 2), (4, 2), (2, 4)])
def test_panel_layout_rebuilds_the_matrix(dv, small, B):
    row, col, val = small
    info, ld, lp = _check_both(dv, row, col, val, PLAN.n_vox, PLAN.n_bl,
                               _opts(dv, B, (1, 1), PLAN.grids, (dv.DOSE_TILE, dv.PRICE_TILE)))
    assert (ld, lp) == (1, 1)
    # at least one panel per tile, none wider than the budget
    tiles = np.prod([-(-g // t) for g, t in zip(PLAN.grids["dose_grid"], dv.DOSE_TILE)])
    assert info.dose_panels >= tiles and 0 < info.dose_panel_cols <= 8192
    assert info.price_panels >= 1 and info.price_panel_cols <= 8192


def test_panel_budget_splits_tiles(dv, small):
    row, col, val = small
    info, ld, lp = _check_both(dv, row, col, val, PLAN.n_vox, PLAN.n_bl,
                               _opts(dv, (2, 1), (1, 1), PLAN.grids, (dv.DOSE_TILE, dv.PRICE_TILE), panel_cols=900,
                                     part_entries=2000, unit_entries=256))
    assert (ld, lp) == (1, 1)
    assert info.dose_panel_parts > info.dose_panels and info.price_panel_parts > info.price_panels
    assert info.dose_panel_cols <= 900 and info.price_panel_cols <= 900
    # the default tiles give 6 price panels here; the budget splits them
    assert info.price_panels > 6


def test_ragged_tiles_and_csr(dv, small):
    row, col, val = small
    # tiles that do not divide the grid, price rows in first-column order as CSR
    info, ld, lp = _check_both(dv, row, col, val, PLAN.n_vox, PLAN.n_bl,
                               _opts(dv, (2, 1), (1, 0), PLAN.grids, ((6, 5, 3), (4, 4, 4)), order=(0, 1)))
    assert (ld, lp) == (1, 0)
    info, ld, lp = _check_both(dv, row, col, val, PLAN.n_vox, PLAN.n_bl, _opts(dv, (4, 2), (0, 0), interleave=0))
    assert (ld, lp) == (0, 0)


def test_unstructured_greedy_panels_and_fallback(dv):
    rng = np.random.default_rng(90)
    n_vox, n_bl = 700, 900
    mask = rng.random((n_vox, n_bl)) < 0.02
    mask[100:110] = rng.random((10, n_bl)) < 0.9          # rows of ~800 entries
    mask[400:450] = False                                 # empty rows
    r, c = np.nonzero(mask)
    r = np.concatenate([r, r[:50]])                       # duplicate pairs are summed
    c = np.concatenate([c, c[:50]])
    v = rng.uniform(0.001, 1, len(r)).astype(np.float32)
    info, ld, lp = _check_both(dv, r, c, v, n_vox, n_bl, _opts(dv, (2, 1), (1, 1), panel_cols=1024))
    assert (ld, lp) == (1, 1)
    # a dense row wider than the budget keeps that orientation in CSR
    info, ld, lp = _check_both(dv, r, c, v, n_vox, n_bl, _opts(dv, (1, 1), (1, 1), panel_cols=500))
    assert ld == 0 and info.dose_panels == 0


@pytest.mark.parametrize("W", [4, 8, 16])
def test_sliced_panels_rebuild_the_matrix(dv, small, W):
    row, col, val = small
    info, ld, lp = _check_both(dv, row, col, val, PLAN.n_vox, PLAN.n_bl,
                               _opts(dv, (1, 1), (2, 2), PLAN.grids, (dv.DOSE_TILE, dv.PRICE_TILE), slice_lanes=W,
                                     part_entries=3000))
    assert (ld, lp) == (2, 2) and info.dose_slice_lanes == W and info.price_slice_lanes == W
    assert info.dose_panel_parts > info.dose_panels
    # ragged tiles, a small budget, sliced dose with a panel-layout price
    info, ld, lp = _check_both(dv, row, col, val, PLAN.n_vox, PLAN.n_bl,
                               _opts(dv, (1, 2), (2, 1), PLAN.grids, ((6, 5, 3), (4, 4, 4)), panel_cols=2000,
                                     slice_lanes=W))
    assert (ld, lp) == (2, 1) and info.price_slice_lanes == 0


@pytest.mark.parametrize("W", [4, 16])
def test_sliced_panels_16bit_codes(dv, small, W):
    """At 16-bit storage a lane's step holds 8 entries (16 bytes of codes);
    every stored code is the FP16 rounding of D_ij / s_j."""
    row, col, val = small
    o = _opts(dv, (1, 1), (2, 2), PLAN.grids, (dv.DOSE_TILE, dv.PRICE_TILE), slice_lanes=W, part_entries=3000)
    h, info = _create(dv, row, col, val, PLAN.n_vox, PLAN.n_bl, o, storage=1)
    try:
        assert (info.dose_layout, info.price_layout, info.value_bytes) == (2, 2, 2)
        ref = _dense(row, col, val, PLAN.n_vox, PLAN.n_bl).astype(np.float32)
        s = np.abs(ref).max(axis=0)
        s[s == 0] = 1.0
        q = (ref / s[None, :]).astype(np.float16).astype(np.float64) * s[None, :].astype(np.float64)
        Dd, _ = _rebuild_sliced(dv, h, info, 0, PLAN.n_vox, PLAN.n_bl, scale=s.astype(np.float64))
        Dp, _ = _rebuild_sliced(dv, h, info, 1, PLAN.n_bl, PLAN.n_vox, scale=s.astype(np.float64))
        assert np.array_equal(Dd, q) and np.array_equal(Dp, q.T)
    finally:
        dv.lib.dvmat_ddc_destroy(h)


def test_sliced_panels_unstructured_and_options(dv):
    rng = np.random.default_rng(91)
    n_vox, n_bl = 500, 600
    mask = rng.random((n_vox, n_bl)) < 0.03
    mask[50:60] = rng.random((10, n_bl)) < 0.8            # long rows
    mask[200:290] = False                                 # more empty rows than one slice holds
    r, c = np.nonzero(mask)
    v = rng.uniform(0.001, 1, len(r)).astype(np.float32)
    info, ld, lp = _check_both(dv, r, c, v, n_vox, n_bl, _opts(dv, (1, 1), (2, 2), panel_cols=1024, slice_lanes=8))
    assert (ld, lp) == (2, 2)
    # block rows other than 1 and unknown lane counts are refused
    for o in (_opts(dv, (2, 1), (2, 0)), _opts(dv, (1, 1), (2, 0), slice_lanes=3)):
        h = ctypes.c_void_p()
        rr = np.ascontiguousarray(r, np.int32); cc = np.ascontiguousarray(c, np.int32)
        assert dv.lib.dvmat_ddc_create_ex(n_vox, n_bl, len(v), rr.ctypes.data_as(P), cc.ctypes.data_as(P),
                                          v.ctypes.data_as(P), 0, ctypes.byref(o), ctypes.byref(h)) == -1


@pytest.mark.parametrize("row_len,storage,want", [(100, 0, 4), (900, 0, 8), (1800, 0, 16), (900, 1, 4),
                                                  (1800, 1, 8), (4000, 1, 16)])
def test_sliced_lanes_follow_the_mean_row_length(dv, row_len, storage, want):
    """Lanes left open: the W in {4, 8, 16} whose slices need closest to 32
    steps of W lanes x E entries (E = 4 at FP32, 8 at 16 bits) for a row of
    the mean non-empty length."""
    rng = np.random.default_rng(row_len)
    n_rows, n_cols = 40, 5000
    r = np.repeat(np.arange(n_rows), row_len)
    c = np.concatenate([rng.choice(n_cols, row_len, replace=False) for _ in range(n_rows)])
    v = rng.uniform(0.1, 1.0, len(r)).astype(np.float32)
    o = _opts(dv, (1, 1), (2, 0), panel_cols=8192)
    h, info = _create(dv, r, c, v, n_rows, n_cols, o, storage=storage)
    try:
        assert info.dose_layout == 2 and info.dose_slice_lanes == want
    finally:
        dv.lib.dvmat_ddc_destroy(h)


def test_grid_must_match_rows(dv, small):
    row, col, val = small
    o = _opts(dv, (2, 1), (1, 1), {"dose_grid": (16, 16, 15), "price_grid": PLAN.grids["price_grid"]},
              (dv.DOSE_TILE, dv.PRICE_TILE))
    h = ctypes.c_void_p()
    row = np.ascontiguousarray(row, np.int32); col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float32)
    assert dv.lib.dvmat_ddc_create_ex(PLAN.n_vox, PLAN.n_bl, len(val), row.ctypes.data_as(P), col.ctypes.data_as(P),
                                      val.ctypes.data_as(P), 0, ctypes.byref(o), ctypes.byref(h)) == -1
    o = _opts(dv, (2, 1), (1, 1), PLAN.grids, ((7, 8, 8), dv.PRICE_TILE))      # 7 is not a multiple of B = 2
    assert dv.lib.dvmat_ddc_create_ex(PLAN.n_vox, PLAN.n_bl, len(val), row.ctypes.data_as(P), col.ctypes.data_as(P),
                                      val.ctypes.data_as(P), 0, ctypes.byref(o), ctypes.byref(h)) == -1
