"""ctypes binding of libdvmat (argument marshalling only).

Every step of the path runs in the HIP library; this module converts torch
tensors to device pointers, owns the device workspaces the library asks for,
and passes torch's current HIP stream.  If the library is not built the
import fails: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libdvmat.so")

F32, F16, BF16 = 0, 1, 2
STORAGE = {"f32": F32, "f16": F16, "bf16": BF16}
KERNEL_KINDS = ("row", "stream", "pipe", "panel")

BB_REL_F, BB_SMALL_STEP, BB_MAX_ITER, BB_FALLBACK, BB_CONVERGED, BB_NONFINITE = 1, 2, 4, 8, 16, 32
BB_STOP_MASK = BB_REL_F | BB_SMALL_STEP | BB_MAX_ITER | BB_CONVERGED | BB_NONFINITE

E_NAMES = {-1: "DVMAT_E_ARG", -2: "DVMAT_E_SHAPE", -3: "DVMAT_E_INDEX", -4: "DVMAT_E_NOMEM",
           -5: "DVMAT_E_HIP", -6: "DVMAT_E_STATE"}


class DvmatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{E_NAMES.get(code, code)}: {msg}")
        self.code = code


class DdcInfo(ctypes.Structure):
    _fields_ = [("n_vox", ctypes.c_int64), ("n_bl", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("nnz_pad_dose", ctypes.c_int64), ("nnz_pad_price", ctypes.c_int64),
                ("n_blocks_dose", ctypes.c_int64), ("n_blocks_price", ctypes.c_int64),
                ("nonempty_rows_dose", ctypes.c_int64), ("nonempty_rows_price", ctypes.c_int64),
                ("storage", ctypes.c_int32), ("value_bytes", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t),
                ("dose_kernel", ctypes.c_int32), ("dose_workgroups", ctypes.c_int32),
                ("price_kernel", ctypes.c_int32), ("price_workgroups", ctypes.c_int32),
                ("dose_tuned_ms", ctypes.c_float), ("price_tuned_ms", ctypes.c_float),
                ("dose_block_rows", ctypes.c_int32), ("price_block_rows", ctypes.c_int32),
                ("dose_row_order", ctypes.c_int32), ("price_row_order", ctypes.c_int32),
                ("dose_layout", ctypes.c_int32), ("price_layout", ctypes.c_int32),
                ("dose_panels", ctypes.c_int64), ("price_panels", ctypes.c_int64),
                ("dose_panel_cols", ctypes.c_int64), ("price_panel_cols", ctypes.c_int64),
                ("dose_panel_cols_total", ctypes.c_int64), ("price_panel_cols_total", ctypes.c_int64),
                ("dose_panel_parts", ctypes.c_int64), ("price_panel_parts", ctypes.c_int64),
                ("dose_slice_lanes", ctypes.c_int32), ("price_slice_lanes", ctypes.c_int32)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("dose_block_rows", ctypes.c_int32), ("price_block_rows", ctypes.c_int32),
                ("interleave", ctypes.c_int32), ("unit_entries", ctypes.c_int32),
                ("dose_row_order", ctypes.c_int32), ("price_row_order", ctypes.c_int32),
                ("dose_layout", ctypes.c_int32), ("price_layout", ctypes.c_int32),
                ("dose_grid", ctypes.c_int32 * 3), ("price_grid", ctypes.c_int32 * 3),
                ("dose_tile", ctypes.c_int32 * 3), ("price_tile", ctypes.c_int32 * 3),
                ("panel_cols", ctypes.c_int32), ("part_entries", ctypes.c_int32),
                ("dose_slice_lanes", ctypes.c_int32), ("price_slice_lanes", ctypes.c_int32)]


# Panel tiles used when the grids are known: 32x16x2 voxels for the dose at
# FP32 (rows of 32 voxels make whole 128-byte lines of the dose output),
# 16x8x8 at 16-bit storage (measured faster there, with two rows per block
# row, and for the batched launch's narrow panels); 4 beamlet columns x 2 MLC
# rows x 8 control points for the price.
DOSE_TILE = (32, 16, 2)
DOSE_TILE_16BIT = (16, 8, 8)
PRICE_TILE = (4, 2, 8)
LAYOUTS = {"csr": 0, "panel": 1, "sliced": 2}


class Geom(ctypes.Structure):
    _fields_ = [("n_cp", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32)]


class BBParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("eps_f", ctypes.c_float), ("eps_step", ctypes.c_float)]


class Machine(ctypes.Structure):
    """Machine parameters of Eq. (2) (dvmat_machine): gantry_step, speed_min,
    speed_max, speed_change, rate_min, rate_max, leaf_speed."""
    _fields_ = [(n, ctypes.c_float) for n in ("gantry_step", "speed_min", "speed_max", "speed_change", "rate_min",
                                              "rate_max", "leaf_speed")]


_P = ctypes.c_void_p
_I32, _I64, _SZ, _F = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float

# name -> (restype, argtypes); must match include/dvmat.h
_SIGNATURES = {
    "dvmat_last_error": (ctypes.c_char_p, []),
    "dvmat_version": (_I32, []),
    "dvmat_ddc_create": (_I32, [_I64, _I64, _I64, _P, _P, _P, _I32, ctypes.POINTER(_P)]),
    "dvmat_ddc_create_ex": (_I32, [_I64, _I64, _I64, _P, _P, _P, _I32, ctypes.POINTER(BuildOpts),
                                   ctypes.POINTER(_P)]),
    "dvmat_ddc_layout_array": (_I32, [_P, _I32, _I32, _P, _SZ, ctypes.POINTER(_SZ)]),
    "dvmat_ddc_default_opts": (_I32, [_I32, ctypes.POINTER(BuildOpts)]),
    "dvmat_ddc_info": (_I32, [_P, ctypes.POINTER(DdcInfo)]),
    "dvmat_ddc_bind": (_I32, [_P, _P, _SZ, _P]),
    "dvmat_ddc_destroy": (None, [_P]),
    "dvmat_obj_workspace_size": (_I32, [_I32, ctypes.POINTER(_SZ)]),
    "dvmat_obj_create": (_I32, [_I64, _I32, _P, _P, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "dvmat_obj_destroy": (None, [_P]),
    "dvmat_objective": (_I32, [_P, _P, _I32, _P, _P, _P]),
    "dvmat_dose": (_I32, [_P, _P, _I32, _P, _P, _P, _P, _P]),
    "dvmat_price": (_I32, [_P, _P, _I32, _P, _P]),
    "dvmat_dose_curvature": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "dvmat_ddc_autotune": (_I32, [_P, _P, _P, _P, _P, _I32, _P]),
    "dvmat_ddc_autotune_obj": (_I32, [_P, _P, _P, _I32, _P, _P, _P, _P, _I32, _P]),
    "dvmat_ddc_set_kernel": (_I32, [_P, _I32, _I32, _I32]),
    "dvmat_batch_workspace_size": (_I32, [_I32, ctypes.POINTER(_SZ)]),
    "dvmat_batch_create": (_I32, [ctypes.POINTER(_P), _I32, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "dvmat_batch_destroy": (None, [_P]),
    "dvmat_batch_dose": (_I32, [_P, ctypes.POINTER(_P), _I32, ctypes.POINTER(_P), _P]),
    "dvmat_batch_price": (_I32, [_P, ctypes.POINTER(_P), _I32, ctypes.POINTER(_P), _P]),
    "dvmat_batch_autotune": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                    ctypes.POINTER(_P), _I32, _I32, _P]),
    "dvmat_batch_set_kernel": (_I32, [_P, _I32, _I32, _I32]),
    "dvmat_batch_info": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    "dvmat_aperture_select": (_I32, [Geom, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dvmat_leaf_windows": (_I32, [Geom, _P, _P, _P, _I32, _P, _P]),
    "dvmat_aperture_select_ws_size": (_I32, [Geom, ctypes.POINTER(_SZ)]),
    "dvmat_machine_leaf_travel": (_I32, [ctypes.POINTER(Machine), _I32, ctypes.POINTER(_I32)]),
    "dvmat_machine_boxes": (_I32, [Geom, ctypes.POINTER(Machine), _P, _P, _P, _P, _P, _P, _P]),
    "dvmat_bb_set_boxes": (_I32, [_P, _P, _P, _P]),
    "dvmat_aperture_select_interdigitated": (_I32, [Geom, _P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "dvmat_aperture_select_interdigitated_noalloc": (_I32, [Geom, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dvmat_bb_workspace_size": (_I32, [Geom, _I32, ctypes.POINTER(_SZ)]),
    "dvmat_bb_create": (_I32, [Geom, _I32, BBParams, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "dvmat_bb_destroy": (None, [_P]),
    "dvmat_bb_count": (_I32, [_P]),
    "dvmat_bb_occupancy": (_I32, [_P, ctypes.POINTER(_P)]),
    "dvmat_bb_add_aperture": (_I32, [_P, _I32, _P, _P, _F, _F, _F, _P]),
    "dvmat_bb_begin": (_I32, [_P, _P]),
    "dvmat_bb_direction": (_I32, [_P, _P, _P, _P]),
    "dvmat_bb_step": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "dvmat_bb_direction_g": (_I32, [_P, _P, _P, _P]),
    "dvmat_bb_step_g": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "dvmat_bb_state": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "dvmat_da_workspace_size": (_I32, [_I64, _I32, ctypes.POINTER(_SZ)]),
    "dvmat_da_create": (_I32, [_I64, _I32, _P, _SZ, ctypes.POINTER(_P)]),
    "dvmat_da_destroy": (None, [_P]),
    "dvmat_da_count": (_I32, [_P]),
    "dvmat_da_append": (_I32, [_P, _P, _P, _P]),
    "dvmat_da_eval": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "dvmat_da_curvature": (_I32, [_P, _P, _P, _P, _P, _P]),
    "dvmat_da_bb_step": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "dvmat_da_set_support": (_I32, [_P, _P, ctypes.POINTER(_I64), _P]),
    "dvmat_da_column": (_I32, [_P, _I32, ctypes.POINTER(_P)]),
    "dvmat_aperture_expand": (_I32, [Geom, _I32, _P, _P, _P, _P, _P, _P]),
    "dvmat_aperture_gather": (_I32, [Geom, _I32, _P, _P, _P, _P, _P, _P]),
    "dvmat_bb_expand": (_I32, [_P, _P, _P]),
    "dvmat_bb_get_y": (_I32, [_P, _P, _P]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdvmat is not built ({LIB_PATH} missing); run __graft_entry__.build() "
                          "or python -m paper_1503_01721_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(code):
    if code != 0:
        raise DvmatError(code, lib.dvmat_last_error().decode(errors="replace"))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, numel, dtype=torch.float32, name="tensor", at_least=False):
    """Shape/dtype guard: raw pointers cross the ABI, so sizes are checked here."""
    if t is None:
        return
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if (t.numel() < numel) if at_least else (t.numel() != numel):
        raise ValueError(f"{name}: {t.numel()} elements, expected {'>= ' if at_least else ''}{numel}")


def _nrhs(t, n, name):
    nrhs = 1 if t.dim() == 1 else t.shape[1]
    if t.dim() > 2 or t.shape[0] != n or not 1 <= nrhs <= 8:
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected [{n}] or [{n}, nrhs<=8]")
    return nrhs


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


class DDC:
    """DDC matrix in both CSR orientations, resident in one GPU's memory."""

    def __init__(self, row, col, val, n_vox: int, n_bl: int, storage: str = "f32", device="cuda",
                 dose_block_rows=None, price_block_rows=None, interleave=None, unit_entries=None,
                 dose_row_order=None, price_row_order=None, dose_grid=None, price_grid=None,
                 dose_layout=None, price_layout=None, dose_tile=None, price_tile=None, panel_cols=None,
                 part_entries=None, slice_lanes=None, dose_slice_lanes=None, price_slice_lanes=None):
        """COO (row = voxel, col = beamlet) to the device layouts.

        dose_grid / price_grid: the voxel grid (nx, ny, nz) and the beamlet grid
        (columns, MLC rows, control points), fastest axis first.  With a grid
        the orientation defaults to the sliced panel layout, the fastest
        measured (tiles DOSE_TILE, or DOSE_TILE_16BIT at 16-bit storage, and
        PRICE_TILE), or to panels when block rows of several rows are asked
        for; without one, to CSR.  *_layout: "csr", "panel" or "sliced" (panels whose rows, sorted
        by length, run in slices of 64 / W rows with W lanes per row: W from
        dose_slice_lanes / price_slice_lanes, or slice_lanes for both)."""
        row = np.ascontiguousarray(row, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float32)
        if not (len(row) == len(col) == len(val)):
            raise ValueError("COO arrays differ in length")
        self.n_vox, self.n_bl = int(n_vox), int(n_bl)
        self.storage = storage
        opts = BuildOpts()
        _check(lib.dvmat_ddc_default_opts(STORAGE[storage], ctypes.byref(opts)))
        for name, v in (("dose_block_rows", dose_block_rows), ("price_block_rows", price_block_rows),
                        ("interleave", interleave), ("unit_entries", unit_entries),
                        ("dose_row_order", dose_row_order), ("price_row_order", price_row_order),
                        ("panel_cols", panel_cols), ("part_entries", part_entries),
                        ("dose_slice_lanes", dose_slice_lanes if dose_slice_lanes is not None else slice_lanes),
                        ("price_slice_lanes", price_slice_lanes if price_slice_lanes is not None else slice_lanes)):
            if v is not None:
                setattr(opts, name, int(v))
        dose_dflt = DOSE_TILE if storage == "f32" else DOSE_TILE_16BIT
        for side, grid, lay, tile, dflt, B in (
                ("dose", dose_grid, dose_layout, dose_tile, dose_dflt, dose_block_rows),
                ("price", price_grid, price_layout, price_tile, PRICE_TILE, price_block_rows)):
            if lay is None:
                # block rows of several rows exist in panels and CSR only
                lay = ("panel" if B is not None and B > 1 else "sliced") if grid is not None else "csr"
            setattr(opts, side + "_layout", LAYOUTS[lay])
            if grid is not None:
                getattr(opts, side + "_grid")[:] = [int(v) for v in grid]
                getattr(opts, side + "_tile")[:] = [int(v) for v in (tile if tile is not None else dflt)]
        h = _P()
        _check(lib.dvmat_ddc_create_ex(self.n_vox, self.n_bl, len(val),
                                       row.ctypes.data_as(_P) if len(val) else None,
                                       col.ctypes.data_as(_P) if len(val) else None,
                                       val.ctypes.data_as(_P) if len(val) else None,
                                       STORAGE[storage], ctypes.byref(opts), ctypes.byref(h)))
        self._destroy = lib.dvmat_ddc_destroy     # bound now: module globals may be gone at exit
        self._h = h
        info = DdcInfo()
        _check(lib.dvmat_ddc_info(h, ctypes.byref(info)))
        self.info = info
        self.device = torch.device(device)
        self.workspace = _workspace(info.workspace_bytes, self.device)
        _check(lib.dvmat_ddc_bind(h, _ptr(self.workspace), self.workspace.numel(), _stream()))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_destroy", None) is not None:
            self._destroy(h)
            self._h = None

    # -- products -----------------------------------------------------------
    def dose_(self, x, z, obj=None, g=None, F=None, stream=None):
        nrhs = _nrhs(x, self.n_bl, "x")
        _need(x, self.n_bl * nrhs, name="x")
        _need(z, self.n_vox * nrhs, name="z")
        _need(g, self.n_vox * nrhs, name="g")
        _need(F, nrhs, name="F", at_least=True)
        if obj is not None and obj.n_vox != self.n_vox:
            raise ValueError("objective and matrix differ in voxel count")
        _check(lib.dvmat_dose(self._h, _ptr(x), nrhs, _ptr(z), obj.handle if obj is not None else None,
                              _ptr(g), _ptr(F), _stream(stream)))

    def price_(self, g, p, stream=None):
        nrhs = _nrhs(g, self.n_vox, "g")
        _need(g, self.n_vox * nrhs, name="g")
        _need(p, self.n_bl * nrhs, name="p")
        _check(lib.dvmat_price(self._h, _ptr(g), nrhs, _ptr(p), _stream(stream)))

    def dose(self, x, obj=None, with_grad=False):
        """z = D x (x: [n_bl] or [n_bl, nrhs] float32 on the device).

        With obj: returns (z, g = dF/dz or None, F[nrhs])."""
        shape = (self.n_vox,) if x.dim() == 1 else (self.n_vox, x.shape[1])
        z = torch.empty(shape, dtype=torch.float32, device=x.device)
        if obj is None:
            self.dose_(x, z)
            return z
        nrhs = 1 if x.dim() == 1 else x.shape[1]
        g = torch.empty_like(z) if with_grad else None
        F = torch.empty(nrhs, dtype=torch.float32, device=x.device)
        self.dose_(x, z, obj, g, F)
        return z, g, F

    def price(self, g):
        """p = D^T g (g: [n_vox] or [n_vox, nrhs] float32 on the device)."""
        shape = (self.n_bl,) if g.dim() == 1 else (self.n_bl, g.shape[1])
        p = torch.empty(shape, dtype=torch.float32, device=g.device)
        self.price_(g, p)
        return p

    def refresh_info(self):
        _check(lib.dvmat_ddc_info(self._h, ctypes.byref(self.info)))
        return self.info

    def autotune(self, reps=5, seed=0, obj=None, nrhs=1):
        """Pick the fastest launch shape per orientation (times every candidate);
        with obj, the dose is timed with its objective epilogue and the price
        on the gradient it writes, nrhs right-hand sides."""
        gen = torch.Generator(device=self.device).manual_seed(seed)
        if obj is not None:
            if obj.n_vox != self.n_vox:
                raise ValueError("objective and matrix differ in voxel count")
            shape_x = (self.n_bl,) if nrhs == 1 else (self.n_bl, nrhs)
            shape_z = (self.n_vox,) if nrhs == 1 else (self.n_vox, nrhs)
            x = torch.rand(shape_x, device=self.device, generator=gen)
            z = torch.empty(shape_z, device=self.device)
            g = torch.empty(shape_z, device=self.device)
            F = torch.empty(nrhs, device=self.device)
            p = torch.empty(shape_x, device=self.device)
            _check(lib.dvmat_ddc_autotune_obj(self._h, obj.handle, _ptr(x), int(nrhs), _ptr(z), _ptr(g), _ptr(F),
                                              _ptr(p), int(reps), _stream()))
            return self.refresh_info()
        x = torch.rand(self.n_bl, device=self.device, generator=gen)
        g = torch.randn(self.n_vox, device=self.device, generator=gen)
        z = torch.empty(self.n_vox, device=self.device)
        p = torch.empty(self.n_bl, device=self.device)
        _check(lib.dvmat_ddc_autotune(self._h, _ptr(x), _ptr(z), _ptr(g), _ptr(p), int(reps), _stream()))
        return self.refresh_info()

    def set_kernel(self, orientation: str, kind: str, workgroups: int):
        _check(lib.dvmat_ddc_set_kernel(self._h, {"dose": 0, "price": 1}[orientation],
                                        KERNEL_KINDS.index(kind), int(workgroups)))
        return self.refresh_info()

    def curvature_(self, x_dir, obj, z_ref, curv, d_out=None, stream=None):
        _need(x_dir, self.n_bl, name="x_dir")
        _need(z_ref, self.n_vox, name="z_ref")
        _need(curv, 1, torch.float64, name="curv", at_least=True)
        _need(d_out, self.n_vox, name="d_out")
        if obj.n_vox != self.n_vox:
            raise ValueError("objective and matrix differ in voxel count")
        _check(lib.dvmat_dose_curvature(self._h, _ptr(x_dir), obj.handle, _ptr(z_ref), _ptr(d_out),
                                        _ptr(curv), _stream(stream)))


class Objective:
    """Per-voxel structure ids (device uint8) and the (T, w+, w-) table."""

    def __init__(self, struct_id, table, device="cuda"):
        table = np.ascontiguousarray(table, dtype=np.float32)
        if table.ndim != 2 or table.shape[1] != 3:
            raise ValueError("table must be [n_struct, 3]")
        self.device = torch.device(device)
        if isinstance(struct_id, np.ndarray):
            if len(struct_id) and int(struct_id.max()) >= table.shape[0]:
                raise ValueError("structure id beyond the table")
            struct_id = torch.from_numpy(np.ascontiguousarray(struct_id, dtype=np.uint8)).to(self.device)
        self.sid = struct_id.contiguous()
        self.n_vox = self.sid.numel()
        self.table = table
        nbytes = _SZ()
        _check(lib.dvmat_obj_workspace_size(table.shape[0], ctypes.byref(nbytes)))
        self.workspace = _workspace(nbytes.value, self.device)
        h = _P()
        _check(lib.dvmat_obj_create(self.n_vox, table.shape[0], _ptr(self.sid), table.ctypes.data_as(_P),
                                    _ptr(self.workspace), self.workspace.numel(), _stream(), ctypes.byref(h)))
        self._destroy = lib.dvmat_obj_destroy     # bound now: module globals may be gone at exit
        self._h = h

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_destroy", None) is not None:
            self._destroy(h)
            self._h = None

    def __call__(self, z, with_grad=True):
        """(F[nrhs], g = dF/dz) of an external dose z."""
        nrhs = _nrhs(z, self.n_vox, "z")
        _need(z, self.n_vox * nrhs, name="z")
        g = torch.empty_like(z) if with_grad else None
        F = torch.empty(nrhs, dtype=torch.float32, device=z.device)
        _check(lib.dvmat_objective(self._h, _ptr(z), nrhs, _ptr(g), _ptr(F), _stream()))
        return F, g


class ApertureSelector:
    """Aperture selection over control points (preallocated outputs); with
    interdigitated=True the leaf rows obey the interdigitation constraint."""

    def __init__(self, n_cp, n_rows, n_cols, device="cuda", interdigitated=False, best=None, best_price=None):
        """best, best_price: optional 1-element device tensors (int32, float32)
        that receive the choice, e.g. views into a caller's status record."""
        self.geom = Geom(n_cp, n_rows, n_cols)
        dev = torch.device(device)
        self.interdigitated = interdigitated
        self.ws = None
        if interdigitated:
            nbytes = _SZ()
            _check(lib.dvmat_aperture_select_ws_size(self.geom, ctypes.byref(nbytes)))
            self.ws = _workspace(nbytes.value, dev)
        self.L = torch.empty((n_cp, n_rows), dtype=torch.int32, device=dev)
        self.R = torch.empty((n_cp, n_rows), dtype=torch.int32, device=dev)
        self.cp_price = torch.empty(n_cp, dtype=torch.float32, device=dev)
        self.best = torch.empty(1, dtype=torch.int32, device=dev) if best is None else best
        self.best_price = torch.empty(1, dtype=torch.float32, device=dev) if best_price is None else best_price
        _need(self.best, 1, torch.int32, name="best")
        _need(self.best_price, 1, name="best_price")

    def __call__(self, p, occupied=None, stream=None, windows=None):
        """windows: device int32 [n_cp, n_rows, 4] leaf windows (Lmin, Lmax, Rmin, Rmax) or None."""
        g = self.geom
        _need(p, g.n_cp * g.n_rows * g.n_cols, name="p")
        if not isinstance(occupied, ctypes.c_void_p):
            _need(occupied, g.n_cp, torch.uint8, name="occupied")
        occ = occupied if isinstance(occupied, ctypes.c_void_p) else _ptr(occupied)
        _need(windows, g.n_cp * g.n_rows * 4, torch.int32, name="windows")
        win = _ptr(windows)
        if self.interdigitated:
            _check(lib.dvmat_aperture_select_interdigitated(
                self.geom, _ptr(p), occ, win, _ptr(self.L), _ptr(self.R), _ptr(self.cp_price), _ptr(self.best),
                _ptr(self.best_price), _ptr(self.ws), self.ws.numel(), _stream(stream)))
            return self
        _check(lib.dvmat_aperture_select(self.geom, _ptr(p), occ, win, _ptr(self.L), _ptr(self.R),
                                         _ptr(self.cp_price), _ptr(self.best), _ptr(self.best_price),
                                         _stream(stream)))
        return self


def aperture_select(p, n_cp, n_rows, n_cols, occupied=None, interdigitated=False, windows=None):
    sel = ApertureSelector(n_cp, n_rows, n_cols, device=p.device, interdigitated=interdigitated)
    sel(p, occupied, windows=windows)
    return dict(L=sel.L, R=sel.R, cp_price=sel.cp_price, best=sel.best, best_price=sel.best_price)


def leaf_windows(n_cp, n_rows, n_cols, occupied, L, R, travel, out=None, stream=None):
    """Leaf windows [n_cp, n_rows, 4] from the openings L, R [n_cp, n_rows] at
    the occupied control points (each leaf within travel beamlets of its
    position at the occupied neighbours)."""
    geom = Geom(n_cp, n_rows, n_cols)
    if not isinstance(occupied, ctypes.c_void_p):
        _need(occupied, n_cp, torch.uint8, name="occupied")
    occ = occupied if isinstance(occupied, ctypes.c_void_p) else _ptr(occupied)
    _need(L, n_cp * n_rows, torch.int32, name="L")
    _need(R, n_cp * n_rows, torch.int32, name="R")
    if out is None:
        out = torch.empty((n_cp, n_rows, 4), dtype=torch.int32, device=L.device)
    _need(out, n_cp * n_rows * 4, torch.int32, name="out")
    _check(lib.dvmat_leaf_windows(geom, occ, _ptr(L), _ptr(R), int(travel), _ptr(out), _stream(stream)))
    return out


def machine_leaf_travel(machine: Machine, n_cols: int) -> int:
    """Leaf travel that keeps a candidate reachable at the slowest gantry speed."""
    t = _I32()
    _check(lib.dvmat_machine_leaf_travel(ctypes.byref(machine), int(n_cols), ctypes.byref(t)))
    return t.value


def machine_boxes(n_cp, n_rows, n_cols, machine: Machine, occupied, L, R, out=None, stream=None):
    """(S^U_k, lo_k, hi_k) device float[n_cp] each: the rate boxes of Eq. (6)
    that the machine model of Eq. (2) gives the apertures L, R [n_cp, n_rows]
    at the occupied control points."""
    geom = Geom(n_cp, n_rows, n_cols)
    if not isinstance(occupied, ctypes.c_void_p):
        _need(occupied, n_cp, torch.uint8, name="occupied")
    occ = occupied if isinstance(occupied, ctypes.c_void_p) else _ptr(occupied)
    _need(L, n_cp * n_rows, torch.int32, name="L")
    _need(R, n_cp * n_rows, torch.int32, name="R")
    if out is None:
        out = tuple(torch.empty(n_cp, dtype=torch.float32, device=L.device) for _ in range(3))
    for t, name in zip(out, ("speed_hi", "lo", "hi")):
        _need(t, n_cp, name=name)
    _check(lib.dvmat_machine_boxes(geom, ctypes.byref(machine), occ, _ptr(L), _ptr(R), _ptr(out[0]), _ptr(out[1]),
                                   _ptr(out[2]), _stream(stream)))
    return out


class BB:
    """Device-resident master-problem state (aperture set, rates, BB history)."""

    def __init__(self, n_cp, n_rows, n_cols, max_apertures, max_iter=50, eps_f=1e-5, eps_step=1e-7, device="cuda"):
        self.geom = Geom(n_cp, n_rows, n_cols)
        self.n_bl = n_cp * n_rows * n_cols
        self.params = BBParams(max_iter, eps_f, eps_step)
        nbytes = _SZ()
        _check(lib.dvmat_bb_workspace_size(self.geom, max_apertures, ctypes.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = _workspace(nbytes.value, self.device)
        h = _P()
        _check(lib.dvmat_bb_create(self.geom, max_apertures, self.params, _ptr(self.workspace),
                                   self.workspace.numel(), _stream(), ctypes.byref(h)))
        self._destroy = lib.dvmat_bb_destroy     # bound now: module globals may be gone at exit
        self._h = h
        self.flags = torch.zeros(1, dtype=torch.int32, device=self.device)

    @property
    def handle(self):
        return self._h

    @property
    def count(self):
        return lib.dvmat_bb_count(self._h)

    def state_ptrs(self):
        """(y, masked gradient) device pointers inside the workspace."""
        y, gt = _P(), _P()
        _check(lib.dvmat_bb_state(self._h, ctypes.byref(y), ctypes.byref(gt)))
        return y, gt

    @property
    def occupied_ptr(self):
        """Device pointer of the control-point occupancy bytes (for aperture selection)."""
        out = _P()
        _check(lib.dvmat_bb_occupancy(self._h, ctypes.byref(out)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_destroy", None) is not None:
            self._destroy(h)
            self._h = None

    def add_aperture(self, cp, L_row, R_row, lo=0.0, hi=float("inf"), y0=None, stream=None):
        y0 = lo if y0 is None else y0
        _need(L_row, self.geom.n_rows, torch.int32, name="L")
        _need(R_row, self.geom.n_rows, torch.int32, name="R")
        _check(lib.dvmat_bb_add_aperture(self._h, int(cp), _ptr(L_row), _ptr(R_row), float(lo), float(hi),
                                         float(y0), _stream(stream)))

    def set_boxes(self, lo_cp, hi_cp, stream=None):
        """Every aperture takes the box of its control point (device float[n_cp])."""
        _need(lo_cp, self.geom.n_cp, name="lo_cp")
        _need(hi_cp, self.geom.n_cp, name="hi_cp")
        _check(lib.dvmat_bb_set_boxes(self._h, _ptr(lo_cp), _ptr(hi_cp), _stream(stream)))

    def begin(self, stream=None):
        _check(lib.dvmat_bb_begin(self._h, _stream(stream)))

    def direction_(self, p, x_dir, stream=None):
        _need(p, self.n_bl, name="p")
        _need(x_dir, self.n_bl, name="x_dir")
        _check(lib.dvmat_bb_direction(self._h, _ptr(p), _ptr(x_dir), _stream(stream)))

    def step_(self, p, F, curv, x_next, stream=None):
        _need(p, self.n_bl, name="p")
        _need(F, 1, name="F", at_least=True)
        _need(curv, 1, torch.float64, name="curv", at_least=True)
        _need(x_next, self.n_bl, name="x_next")
        _check(lib.dvmat_bb_step(self._h, _ptr(p), _ptr(F), _ptr(curv), _ptr(x_next), _ptr(self.flags),
                                 _stream(stream)))

    def direction_g_(self, G, x_dir, stream=None):
        _need(G, self.count, name="G", at_least=True)
        _need(x_dir, self.n_bl, name="x_dir")
        _check(lib.dvmat_bb_direction_g(self._h, _ptr(G), _ptr(x_dir), _stream(stream)))

    def step_g_(self, G, F, curv, x_next, stream=None):
        _need(G, self.count, name="G", at_least=True)
        _need(F, 1, name="F", at_least=True)
        _need(curv, 1, torch.float64, name="curv", at_least=True)
        _need(x_next, self.n_bl, name="x_next")
        _check(lib.dvmat_bb_step_g(self._h, _ptr(G), _ptr(F), _ptr(curv), _ptr(x_next), _ptr(self.flags),
                                   _stream(stream)))

    def expand_(self, x, stream=None):
        _need(x, self.n_bl, name="x")
        _check(lib.dvmat_bb_expand(self._h, _ptr(x), _stream(stream)))

    def y(self):
        out = torch.empty(max(self.count, 1), dtype=torch.float32, device=self.device)
        _check(lib.dvmat_bb_get_y(self._h, _ptr(out), _stream()))
        return out[:self.count]


class DAColumns:
    """Dense aperture dose vectors DA_k (Eq. 5) for the DA-form master problem.
    With obj, the columns keep only the rows of the objective's support
    (dvmat_da_set_support): eval then writes z and dF/dz at those voxels only."""

    def __init__(self, n_vox, max_apertures, device="cuda", obj=None):
        self.n_vox = int(n_vox)
        nbytes = _SZ()
        _check(lib.dvmat_da_workspace_size(self.n_vox, int(max_apertures), ctypes.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = _workspace(nbytes.value, self.device)
        h = _P()
        _check(lib.dvmat_da_create(self.n_vox, int(max_apertures), _ptr(self.workspace), self.workspace.numel(),
                                   ctypes.byref(h)))
        self._destroy = lib.dvmat_da_destroy     # bound now: module globals may be gone at exit
        self._h = h
        self.n_rows = self.n_vox
        if obj is not None:
            if obj.n_vox != self.n_vox:
                raise ValueError("objective and columns differ in voxel count")
            n = _I64()
            _check(lib.dvmat_da_set_support(h, obj.handle, ctypes.byref(n), _stream()))
            self.n_rows = n.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_destroy", None) is not None:
            self._destroy(h)
            self._h = None

    @property
    def count(self):
        return lib.dvmat_da_count(self._h)

    def append_(self, ddc, x_ind, stream=None):
        _need(x_ind, ddc.n_bl, name="x_ind")
        _check(lib.dvmat_da_append(self._h, ddc.handle, _ptr(x_ind), _stream(stream)))

    def eval_(self, obj, y, G, z=None, g=None, F=None, stream=None):
        """y, G: device pointers (c_void_p) or tensors of count floats."""
        yp = y if isinstance(y, ctypes.c_void_p) else _ptr(y)
        if not isinstance(y, ctypes.c_void_p):
            _need(y, self.count, name="y", at_least=True)
        _need(G, self.count, name="G", at_least=True)
        _need(z, self.n_vox, name="z")
        _need(g, self.n_vox, name="g")
        _need(F, 1, name="F", at_least=True)
        _check(lib.dvmat_da_eval(self._h, obj.handle, yp, _ptr(z), _ptr(g), _ptr(G), _ptr(F), _stream(stream)))

    def bb_step_(self, bb, obj, G, F, curv, stream=None):
        """One BB iteration on the columns in one launch (dvmat_da_bb_step):
        G, F at bb's current rates, then its step; flags go to bb.flags."""
        _need(G, self.count, name="G", at_least=True)
        _need(F, 1, name="F", at_least=True)
        _need(curv, 1, torch.float64, name="curv", at_least=True)
        _check(lib.dvmat_da_bb_step(self._h, bb.handle, obj.handle, _ptr(G), _ptr(F), _ptr(curv), _ptr(bb.flags),
                                    _stream(stream)))

    def curvature_(self, obj, direction, z_ref, curv, stream=None):
        dp = direction if isinstance(direction, ctypes.c_void_p) else _ptr(direction)
        _need(z_ref, self.n_vox, name="z_ref")
        _need(curv, 1, torch.float64, name="curv", at_least=True)
        _check(lib.dvmat_da_curvature(self._h, obj.handle, dp, _ptr(z_ref), _ptr(curv), _stream(stream)))

    def column(self, k):
        p = _P()
        _check(lib.dvmat_da_column(self._h, int(k), ctypes.byref(p)))
        return p


class Apertures:
    """An explicit list of apertures (distinct control points) on the device,
    with the fluence map x = B y and its adjoint G = B^T p."""

    def __init__(self, n_cp, n_rows, n_cols, cps, L, R, device="cuda"):
        self.geom = Geom(n_cp, n_rows, n_cols)
        self.n_bl = n_cp * n_rows * n_cols
        dev = torch.device(device)
        cps = np.ascontiguousarray(cps, np.int32)
        if len(set(cps.tolist())) != len(cps) or (len(cps) and (cps.min() < 0 or cps.max() >= n_cp)):
            raise ValueError("apertures must sit at distinct control points in range")
        L = np.ascontiguousarray(L, np.int32).reshape(len(cps), n_rows)
        R = np.ascontiguousarray(R, np.int32).reshape(len(cps), n_rows)
        if np.any(L < 0) or np.any(R > n_cols) or np.any(L > R):
            raise ValueError("openings must satisfy 0 <= L <= R <= n_cols")
        self.m = len(cps)
        self.cps = torch.from_numpy(cps).to(dev)
        self.L = torch.from_numpy(L).to(dev)
        self.R = torch.from_numpy(R).to(dev)

    def expand_(self, y, x, stream=None):
        _need(y, self.m, name="y")
        _need(x, self.n_bl, name="x")
        _check(lib.dvmat_aperture_expand(self.geom, self.m, _ptr(self.cps), _ptr(self.L), _ptr(self.R), _ptr(y),
                                         _ptr(x), _stream(stream)))

    def gather_(self, p, G, stream=None):
        _need(p, self.n_bl, name="p")
        _need(G, self.m, name="G")
        _check(lib.dvmat_aperture_gather(self.geom, self.m, _ptr(self.cps), _ptr(self.L), _ptr(self.R), _ptr(p),
                                         _ptr(G), _stream(stream)))


class Batch:
    """Several plans' products in one launch each (dose, price)."""

    def __init__(self, ddcs, device="cuda"):
        self.ddcs = list(ddcs)
        n = len(self.ddcs)
        nbytes = _SZ()
        _check(lib.dvmat_batch_workspace_size(n, ctypes.byref(nbytes)))
        self.device = torch.device(device)
        self.workspace = _workspace(nbytes.value, self.device)
        arr = (_P * n)(*[d.handle.value for d in self.ddcs])
        h = _P()
        _check(lib.dvmat_batch_create(arr, n, _ptr(self.workspace), self.workspace.numel(), _stream(),
                                      ctypes.byref(h)))
        self._destroy = lib.dvmat_batch_destroy     # bound now: module globals may be gone at exit
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_destroy", None) is not None:
            self._destroy(h)
            self._h = None

    def _ptrs(self, ts, sizes, name):
        if len(ts) != len(self.ddcs):
            raise ValueError(f"{name}: {len(ts)} tensors for {len(self.ddcs)} plans")
        nrhs = 1 if ts[0].dim() == 1 else ts[0].shape[1]
        for t, n in zip(ts, sizes):
            _need(t, n * nrhs, name=name)
            if (1 if t.dim() == 1 else t.shape[1]) != nrhs:
                raise ValueError(f"{name}: mixed nrhs")
        return (_P * len(ts))(*[t.data_ptr() for t in ts]), nrhs

    def dose_(self, xs, zs, stream=None):
        px, nrhs = self._ptrs(xs, [d.n_bl for d in self.ddcs], "x")
        pz, _ = self._ptrs(zs, [d.n_vox for d in self.ddcs], "z")
        _check(lib.dvmat_batch_dose(self._h, px, nrhs, pz, _stream(stream)))

    def price_(self, gs, ps, stream=None):
        pg, nrhs = self._ptrs(gs, [d.n_vox for d in self.ddcs], "g")
        pp, _ = self._ptrs(ps, [d.n_bl for d in self.ddcs], "p")
        _check(lib.dvmat_batch_price(self._h, pg, nrhs, pp, _stream(stream)))

    def autotune(self, xs, zs, gs, ps, reps=3):
        px, nrhs = self._ptrs(xs, [d.n_bl for d in self.ddcs], "x")
        pz, _ = self._ptrs(zs, [d.n_vox for d in self.ddcs], "z")
        pg, _ = self._ptrs(gs, [d.n_vox for d in self.ddcs], "g")
        pp, _ = self._ptrs(ps, [d.n_bl for d in self.ddcs], "p")
        _check(lib.dvmat_batch_autotune(self._h, px, pz, pg, pp, nrhs, int(reps), _stream()))
        return self.info()

    def set_kernel(self, orientation: str, kind: str, workgroups: int):
        _check(lib.dvmat_batch_set_kernel(self._h, {"dose": 0, "price": 1}[orientation],
                                          KERNEL_KINDS.index(kind), int(workgroups)))
        return self.info()

    def info(self):
        nd, npb = _I64(), _I64()
        cfg = (_I32 * 4)()
        _check(lib.dvmat_batch_info(self._h, ctypes.byref(nd), ctypes.byref(npb), cfg))
        return dict(dose_blocks=nd.value, price_blocks=npb.value, dose_kernel=cfg[0], dose_workgroups=cfg[1],
                    price_kernel=cfg[2], price_workgroups=cfg[3])


def exported_symbols():
    """Names this binding binds (all entry points of include/dvmat.h)."""
    return sorted(_SIGNATURES)
