"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point of include/dvmat.h, and validates COO input in
dvmat_ddc_create (which runs on the host only)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dvmat.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dvmat_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def dv():
    from paper_1503_01721_amd import dvmat
    return dvmat


def test_library_exports_every_header_symbol(dv):
    names = header_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(dv.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares exactly the header's functions
    assert sorted(dv.exported_symbols()) == names


def test_version(dv):
    assert dv.lib.dvmat_version() == 0x000100


def _create(dv, n_vox, n_bl, row, col, val, storage=0):
    row = np.ascontiguousarray(row, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float32)
    h = ctypes.c_void_p()
    code = dv.lib.dvmat_ddc_create(n_vox, n_bl, len(val), row.ctypes.data_as(ctypes.c_void_p),
                                   col.ctypes.data_as(ctypes.c_void_p), val.ctypes.data_as(ctypes.c_void_p),
                                   storage, ctypes.byref(h))
    return code, h


def test_create_rejects_out_of_range_index(dv):
    code, h = _create(dv, 4, 3, [0, 4], [0, 1], [1.0, 2.0])
    assert code == -3 and not h.value
    assert b"outside" in dv.lib.dvmat_last_error()
    code, h = _create(dv, 4, 3, [0, 1], [0, -1], [1.0, 2.0])
    assert code == -3


def test_create_rejects_non_finite_and_bad_sizes(dv):
    code, _ = _create(dv, 4, 3, [0, 1], [0, 1], [1.0, np.nan])
    assert code == -1
    code, _ = _create(dv, 4, 3, [0, 1], [0, 1], [np.inf, 1.0])
    assert code == -1
    code, _ = _create(dv, 0, 3, [], [], [])
    assert code == -1
    code, _ = _create(dv, 4, 3, [0], [0], [1.0], storage=7)
    assert code == -1
    h = ctypes.c_void_p()
    assert dv.lib.dvmat_ddc_create(4, 3, 2, None, None, None, 0, ctypes.byref(h)) == -1


def test_create_merges_duplicates_and_pads_rows(dv):
    # voxel 0: beamlets 2, 0, 2 (duplicate, unsorted); voxel 2: beamlet 1; voxel 1 empty
    code, h = _create(dv, 3, 3, [0, 0, 2, 0], [2, 0, 1, 2], [1.0, 2.0, 3.0, 4.0])
    assert code == 0
    info = dv.DdcInfo()
    assert dv.lib.dvmat_ddc_info(h, ctypes.byref(info)) == 0
    assert info.nnz == 3                       # (0,0), (0,2) merged, (2,1)
    assert info.nnz_pad_dose % 4 == 0 and info.nnz_pad_price % 4 == 0
    assert info.nonempty_rows_dose == 2 and info.nonempty_rows_price == 3
    assert info.value_bytes == 4 and info.workspace_bytes > 0
    dv.lib.dvmat_ddc_destroy(h)


def test_create_empty_matrix_and_16bit_storage(dv):
    h = ctypes.c_void_p()
    assert dv.lib.dvmat_ddc_create(5, 7, 0, None, None, None, 1, ctypes.byref(h)) == 0
    info = dv.DdcInfo()
    dv.lib.dvmat_ddc_info(h, ctypes.byref(info))
    assert info.nnz == 0 and info.nnz_pad_dose == 0 and info.value_bytes == 2
    dv.lib.dvmat_ddc_destroy(h)


def test_row_blocks_cover_rows(dv):
    from paper_1503_01721_amd import synth
    plan = synth.PLANS["small_cp8_bl6x6_vox16"]
    d = synth.generate_ddc(plan)
    code, h = _create(dv, plan.n_vox, plan.n_bl, d["row"], d["col"], d["val"])
    assert code == 0
    info = dv.DdcInfo()
    dv.lib.dvmat_ddc_info(h, ctypes.byref(info))
    assert info.nnz == len(d["val"])
    assert info.n_blocks_dose >= 1 and info.n_blocks_price >= 1
    # with one row per block row, padding adds fewer than 4 entries per non-empty row
    assert info.price_block_rows == 1
    assert info.nnz <= info.nnz_pad_price < info.nnz + 4 * info.nonempty_rows_price
    assert info.nnz_pad_dose >= info.nnz
    dv.lib.dvmat_ddc_destroy(h)


def test_bb_and_select_argument_checks(dv):
    g = dv.Geom(4, 3, 5)
    n = ctypes.c_size_t()
    assert dv.lib.dvmat_bb_workspace_size(g, 5, ctypes.byref(n)) == -1      # more apertures than CPs
    assert dv.lib.dvmat_bb_workspace_size(g, 4, ctypes.byref(n)) == 0 and n.value > 0
    assert dv.lib.dvmat_bb_workspace_size(dv.Geom(0, 3, 5), 1, ctypes.byref(n)) == -2
    big = dv.Geom(2, 200, 200)
    assert dv.lib.dvmat_aperture_select(big, None, None, None, None, None, None, None, None, None) == -2
    assert dv.lib.dvmat_aperture_select(g, None, None, None, None, None, None, None, None, None) == -1
    assert dv.lib.dvmat_leaf_windows(g, None, None, None, 1, None, None) == -1
    assert dv.lib.dvmat_leaf_windows(dv.Geom(0, 3, 5), None, None, None, 1, None, None) == -2
    assert dv.lib.dvmat_aperture_select_ws_size(dv.Geom(4, 3, 5), ctypes.byref(n)) == 0
    assert n.value == 4 * 3 * (6 * 7 // 2) * 4                  # one FP32 value per row state
    assert dv.lib.dvmat_aperture_select_ws_size(dv.Geom(4, 3, 97), ctypes.byref(n)) == -2
    assert dv.lib.dvmat_aperture_select_interdigitated(g, None, None, None, None, None, None, None, None, None,
                                                       0, None) == -1
    assert dv.lib.dvmat_obj_workspace_size(0, ctypes.byref(n)) == -1
    assert dv.lib.dvmat_obj_workspace_size(5, ctypes.byref(n)) == 0
    assert dv.lib.dvmat_bb_count(None) == -1


def test_build_options(dv):
    from paper_1503_01721_amd import synth
    opts = dv.BuildOpts()
    for storage in (0, 1, 2):
        assert dv.lib.dvmat_ddc_default_opts(storage, ctypes.byref(opts)) == 0
        assert opts.dose_block_rows in (0, 1, 2, 4) and opts.price_block_rows in (0, 1, 2, 4)
        assert opts.interleave in (0, 1)
    assert dv.lib.dvmat_ddc_default_opts(7, ctypes.byref(opts)) == -1
    plan = synth.PLANS["small_cp8_bl6x6_vox16"]
    d = synth.generate_ddc(plan)
    row = np.ascontiguousarray(d["row"]); col = np.ascontiguousarray(d["col"]); val = np.ascontiguousarray(d["val"])
    P = ctypes.c_void_p
    # 0 = the default for the layout and storage (CSR, FP32 here: dose 2, price 1)
    for bd, bp in ((1, 1), (2, 4), (4, 2), (3, 1), (1, 8), (0, 0)):
        o = dv.BuildOpts()
        assert dv.lib.dvmat_ddc_default_opts(0, ctypes.byref(o)) == 0
        o.dose_block_rows, o.price_block_rows, o.price_row_order = bd, bp, 1
        h = ctypes.c_void_p()
        code = dv.lib.dvmat_ddc_create_ex(plan.n_vox, plan.n_bl, len(val), row.ctypes.data_as(P), col.ctypes.data_as(P),
                                          val.ctypes.data_as(P), 0, ctypes.byref(o), ctypes.byref(h))
        if bd not in (0, 1, 2, 4) or bp not in (0, 1, 2, 4):
            assert code == -1
            continue
        assert code == 0
        bd, bp = bd or 2, bp or 1
        info = dv.DdcInfo()
        dv.lib.dvmat_ddc_info(h, ctypes.byref(info))
        assert info.nnz == len(val) and info.dose_block_rows == bd and info.price_block_rows == bp
        # stored value slots: at least the non-zeros, block rows hold B values per stored column
        assert info.nnz_pad_dose >= info.nnz and info.nnz_pad_dose % bd == 0
        assert info.nnz_pad_price >= info.nnz and info.nnz_pad_price % bp == 0
        dv.lib.dvmat_ddc_destroy(h)


def test_machine_leaf_travel_and_argument_checks(dv):
    """The leaf travel is host arithmetic: checked against the oracle here."""
    import math

    from oracle import machine as omach
    cases = [(2.0, 1.0, 6.0, 1.0, 2.0, 10.0, 3.0, 8), (2.0, 1.0, 6.0, 1.0, 2.0, 10.0, 3.0, 4),
             (1.0, 0.0, 4.0, 0.5, 0.0, 1.0, 2.0, 20), (1.0, 0.5, 4.0, 0.5, 0.0, 1.0, math.inf, 20),
             (0.75, 0.5, 4.0, 0.25, 1.0, 2.0, 1.25, 40), (3.0, 0.25, math.inf, math.inf, 0.0, math.inf, 0.5, 100)]
    for *vals, n_cols in cases:
        m = dv.Machine(*vals)
        assert dv.machine_leaf_travel(m, n_cols) == omach.leaf_travel(omach.Machine(*vals), n_cols)
    t = ctypes.c_int32()
    bad = [(0.0, 1, 2, 1, 0, 1, 1), (1, -1, 2, 1, 0, 1, 1), (1, 3, 2, 1, 0, 1, 1), (1, 1, 2, -1, 0, 1, 1),
           (1, 1, 2, 1, 2, 1, 1), (1, 1, 2, 1, 0, 1, 0), (1, 1, 2, 1, math.nan, 1, 1), (1, 1, 2, 1, math.inf, math.inf, 1)]
    for vals in bad:
        assert dv.lib.dvmat_machine_leaf_travel(ctypes.byref(dv.Machine(*vals)), 10, ctypes.byref(t)) == -1, vals
    good = dv.Machine(2, 1, 6, 1, 2, 10, 3)
    assert dv.lib.dvmat_machine_leaf_travel(None, 10, ctypes.byref(t)) == -1
    assert dv.lib.dvmat_machine_leaf_travel(ctypes.byref(good), 0, ctypes.byref(t)) == -1
    g = dv.Geom(4, 3, 5)
    assert dv.lib.dvmat_machine_boxes(g, ctypes.byref(good), None, None, None, None, None, None, None) == -1
    assert dv.lib.dvmat_machine_boxes(g, ctypes.byref(dv.Machine(*bad[0])), None, None, None, None, None, None,
                                      None) == -1
    assert dv.lib.dvmat_machine_boxes(dv.Geom(8193, 3, 5), ctypes.byref(good), None, None, None, None, None, None,
                                      None) == -2
    assert dv.lib.dvmat_bb_set_boxes(None, None, None, None) == -1


def test_select_noalloc_rejects_before_touching_a_device(dv):
    """The no-allocation selection checks its arguments and the scratch limit
    on the host before it looks up the device array or enqueues anything."""
    f = dv.lib.dvmat_aperture_select_interdigitated_noalloc
    dummy = ctypes.c_void_p(256)          # never dereferenced: the call returns first
    args = [dummy] * 5 + [None]          # L, R, cp_price, best, best_price; null stream
    # 96 columns: 4,753 states x 4 bytes per row; 1,765 rows exceed 32 MiB
    assert f(dv.Geom(1765, 1, 96), dummy, None, None, *args) == -4
    assert b"limit" in dv.lib.dvmat_last_error()
    assert f(dv.Geom(1, 1, 97), dummy, None, None, *args) == -2      # DP limited to 96 columns
    assert f(dv.Geom(0, 1, 8), dummy, None, None, *args) == -2
    assert f(dv.Geom(4, 2, 8), None, None, None, *args) == -1        # p is NULL
