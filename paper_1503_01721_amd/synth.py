"""Seeded synthetic VMAT workloads: pencil-beam dose-deposition (DDC) matrices,
structure maps and benchmark vectors.

This module produces INPUTS only.  It holds none of the optimiser's arithmetic
(no dose/price products, no objective, no aperture selection, no step rule);
the FP64 oracle and the HIP library both consume the arrays it returns, and
neither of them is imported here.

The paper's DDC comes from a finite-size pencil-beam engine on patient CT
(Section 2.4) that is not available; these matrices stand in for it with the
same shape: voxels x beamlets, one beamlet grid per control point (beam
angle), entries non-negative, each beamlet touching a narrow tilted cylinder
of voxels, small entries dropped (the same effect as the truncation of
Section 2.4, method S1).

Geometry (all workloads)
------------------------
* Cube of N^3 voxels of pitch h; voxel centre along each axis is
  (i - (N-1)/2) * h, voxel index (iz*N + iy)*N + ix (x fastest).
* Gantry axis = z.  Control point a has angle theta_a = a * 360deg / n_cp,
  beam direction d = (sin, -cos, 0), beam's-eye axes u = (cos, sin, 0) and
  v = (0, 0, 1).  Parallel beams.
* Beamlet (r, c) of an n_rows x n_cols grid of pitch b sits at
  u_c = (c - (n_cols-1)/2) b, v_r = (r - (n_rows-1)/2) b; an MLC leaf row is
  one r (leaves move along u).  Beamlet index j = (a*n_rows + r)*n_cols + c.
* Body: cylinder along z of radius R_b = min(0.45 N h, 115 mm); voxels
  outside it get no entries and no objective.
* Entry for voxel P and beamlet j:
      t     = P.d,  depth = max(0, t + sqrt(max(R_b^2 - u_c^2, 0)))
      f_u   = exp(-mu depth) * exp(-(P.u - u_c)^2 / (2 sigma^2))
      f_v   = exp(-(P.v - v_r)^2 / (2 sigma^2))
      D_ij  = f_u * f_v   (float64), kept iff D_ij >= 1e-3, stored float32
  with mu = 0.05 / mm and sigma = 3 mm, so the kernel's maximum is 1.
* Structures (priority PTV > OAR > body): PTV sphere(s); OAR_a (cord-like)
  sphere at (0, 0.75 R_b, 0) radius 0.2 R_b; OAR_b (parotid-like) sphere at
  (0.6 R_b, -0.35 R_b, 0) radius 0.15 R_b; body.  Per-structure table rows
  are (T, w_over, w_under) in the notation of the objective, Eq. (1).
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Tuple

import numpy as np

MU_PER_MM = 0.05
SIGMA_MM = 3.0
CUTOFF = 1e-3

# structure ids
S_OUTSIDE, S_BODY, S_OAR_A, S_OAR_B, S_PTV0 = 0, 1, 2, 3, 4


@dataclasses.dataclass(frozen=True)
class Plan:
    """Geometry of one synthetic plan."""
    name: str
    n_cp: int          # control points (beam angles)
    n_rows: int        # MLC leaf rows per control point
    n_cols: int        # beamlets per leaf row
    bl_mm: float       # beamlet pitch
    n_grid: int        # voxel cube side N
    vox_mm: float      # voxel pitch h
    # PTVs: (cx, cy, cz, radius, prescription); None -> one 20 mm sphere at 70 Gy
    ptvs: Optional[Tuple[Tuple[float, float, float, float, float], ...]] = None

    @property
    def n_vox(self) -> int:
        return self.n_grid ** 3

    @property
    def n_bl(self) -> int:
        return self.n_cp * self.n_rows * self.n_cols

    @property
    def grids(self) -> dict:
        """Row grids of the two orientations, fastest axis first: voxels
        (x, y, z) and beamlets (column, MLC row, control point)."""
        return {"dose_grid": (self.n_grid, self.n_grid, self.n_grid),
                "price_grid": (self.n_cols, self.n_rows, self.n_cp)}

    @property
    def body_radius(self) -> float:
        return min(0.45 * self.n_grid * self.vox_mm, 115.0)

    def ptv_list(self):
        if self.ptvs is not None:
            return list(self.ptvs)
        return [(0.0, 0.0, 0.0, min(20.0, 0.5 * self.body_radius), 70.0)]


# Named workloads (sizes in the name).  The first three are the plain-method,
# full-scale and two-arc shapes; "tiny" is for dense brute force.
PLANS: Dict[str, Plan] = {
    "tiny_cp4_bl3x4_vox8": Plan("tiny_cp4_bl3x4_vox8", 4, 3, 4, 5.0, 8, 5.0,
                                ((0.0, 0.0, 0.0, 8.0, 70.0),)),
    "small_cp8_bl6x6_vox16": Plan("small_cp8_bl6x6_vox16", 8, 6, 6, 5.0, 16, 2.5,
                                  ((0.0, 0.0, 0.0, 8.0, 70.0),)),
    "cp20_bl20x20_vox32": Plan("cp20_bl20x20_vox32", 20, 20, 20, 5.0, 32, 2.5),
    "cp180_bl40x40_vox128": Plan("cp180_bl40x40_vox128", 180, 40, 40, 5.0, 128, 2.5),
    "cp360_bl60x60_vox160": Plan("cp360_bl60x60_vox160", 360, 60, 60, 3.3, 160, 2.0),
    # two-arc pitches (3.3 mm beamlets, 2 mm voxels) at a size the oracle finishes quickly
    "cp64_bl12x12_vox40": Plan("cp64_bl12x12_vox40", 64, 12, 12, 3.3, 40, 2.0,
                               ((0.0, 0.0, 0.0, 12.0, 70.0),)),
}


def batched_plans(n: int = 48, seed: int = 2005, max_cp: int = 180, max_grid: int = 40, max_vox: int = 128):
    """n independent plans of uneven size: angles U{60..max_cp}, beamlet grids
    U{20..max_grid} square at 5 mm, voxel cubes U{48..max_vox} at 2.5 mm, 1-3
    non-overlapping spherical PTVs of radius U[12, 20] mm centred within
    0.4 R_b, prescriptions drawn from {70, 59.4, 54} Gy (the three PTV levels
    of the paper's head-and-neck case, Sec. 2.4)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        n_cp = int(rng.integers(60, max_cp + 1))
        grid = int(rng.integers(20, max_grid + 1))
        nv = int(rng.integers(48, max_vox + 1))
        R = min(0.45 * nv * 2.5, 115.0)
        ptvs = []
        want = int(rng.integers(1, 4))
        tries = 0
        while len(ptvs) < want and tries < 1000:
            tries += 1
            rad = float(rng.uniform(12.0, 20.0))
            c = rng.uniform(-0.4 * R, 0.4 * R, 3)
            if np.linalg.norm(c) > 0.4 * R:
                continue
            if all(np.linalg.norm(c - np.array(q[:3])) > rad + q[3] for q in ptvs):
                ptvs.append((float(c[0]), float(c[1]), float(c[2]), rad, float(rng.choice([70.0, 59.4, 54.0]))))
        out.append(Plan(f"batch{i:02d}_cp{n_cp}_bl{grid}x{grid}_vox{nv}", n_cp, grid, grid, 5.0, nv, 2.5, tuple(ptvs)))
    return out


def axis_centres(n: int, pitch: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * pitch


def beamlet_offsets(plan: Plan) -> Tuple[np.ndarray, np.ndarray]:
    """(u_c for c in cols, v_r for r in rows) in mm."""
    return axis_centres(plan.n_cols, plan.bl_mm), axis_centres(plan.n_rows, plan.bl_mm)


def cp_angle(plan: Plan, a: int) -> float:
    return 2.0 * math.pi * a / plan.n_cp


def body_xy(plan: Plan) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Body cross-section points in raster order: (x, y, iy*N+ix)."""
    N, h, R = plan.n_grid, plan.vox_mm, plan.body_radius
    c = axis_centres(N, h)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    inside = (xx * xx + yy * yy) <= R * R
    idx = np.nonzero(inside.ravel())[0]
    return xx.ravel()[idx], yy.ravel()[idx], idx.astype(np.int64)


def _angle_factors(plan: Plan, a: int, px, py, u_c, with_lateral: bool = False):
    """f_u[c, p] for every beamlet column c and body cross-section point p
    (and, with_lateral, the squared distance along u to the beamlet axis)."""
    th = cp_angle(plan, a)
    s, co = math.sin(th), math.cos(th)
    t = px * s - py * co
    pu = px * co + py * s
    R = plan.body_radius
    entry = np.sqrt(np.maximum(R * R - u_c * u_c, 0.0))
    depth = np.maximum(0.0, t[None, :] + entry[:, None])
    lat = pu[None, :] - u_c[:, None]
    fu = np.exp(-MU_PER_MM * depth) * np.exp(-(lat * lat) / (2.0 * SIGMA_MM ** 2))
    return (fu, lat * lat) if with_lateral else fu


def _v_factors(plan: Plan, v_r):
    z = axis_centres(plan.n_grid, plan.vox_mm)
    dz = z[None, :] - v_r[:, None]
    return np.exp(-(dz * dz) / (2.0 * SIGMA_MM ** 2))     # [n_rows, N]


def generate_cp(plan: Plan, a: int, xy=None, z_slab: Optional[Tuple[int, int]] = None,
                cutoff: float = CUTOFF, cone_mm: Optional[float] = None):
    """All entries of control point a, sorted by beamlet then voxel index;
    with z_slab = (z0, z1) only the voxels of slices z0 <= iz < z1.
    cutoff: entries below it are dropped; cone_mm: entries of voxels farther
    than this from the beamlet's central axis are dropped too (the truncation
    by a cone about each beamlet axis of Sec. 2.4; the beams here are
    parallel, so the cone is a cylinder of that radius).

    Returns (row_vox int32, col_bl int32, val float32)."""
    px, py, pidx = xy if xy is not None else body_xy(plan)
    N = plan.n_grid
    u_c, v_r = beamlet_offsets(plan)
    fu, lat2_u = _angle_factors(plan, a, px, py, u_c, with_lateral=True)   # [C, P]
    fv = _v_factors(plan, v_r)                            # [R, N]
    lat2_v = (axis_centres(N, plan.vox_mm)[None, :] - v_r[:, None]) ** 2
    if z_slab is not None:
        fv[:, :z_slab[0]] = 0.0
        fv[:, z_slab[1]:] = 0.0
    r2max = np.inf if cone_mm is None else float(cone_mm) ** 2
    # Only points/slices that can pass the cut (the other factor is <= 1,
    # the other squared distance >= 0).
    # Padded per-column point lists keep the (r, c, iz, p) order of np.nonzero.
    keep_u = (fu >= cutoff) & (lat2_u <= r2max)
    cnt_u = keep_u.sum(axis=1)
    Pm = max(int(cnt_u.max()), 1)
    order_u = np.argsort(~keep_u, axis=1, kind="stable")[:, :Pm]   # kept first, raster order
    fu_pad = np.take_along_axis(fu, order_u, axis=1)
    fu_pad[np.arange(Pm)[None, :] >= cnt_u[:, None]] = 0.0
    keep_v = (fv >= cutoff) & (lat2_v <= r2max)
    cnt_v = keep_v.sum(axis=1)
    Km = max(int(cnt_v.max()), 1)
    order_v = np.argsort(~keep_v, axis=1, kind="stable")[:, :Km]
    fv_pad = np.take_along_axis(fv, order_v, axis=1)
    fv_pad[np.arange(Km)[None, :] >= cnt_v[:, None]] = 0.0
    if cone_mm is not None:
        l2u_pad = np.take_along_axis(lat2_u, order_u, axis=1)
        l2v_pad = np.take_along_axis(lat2_v, order_v, axis=1)
    rows_out, cols_out, vals_out = [], [], []
    # chunk over leaf rows to bound memory
    R, C = plan.n_rows, plan.n_cols
    chunk = max(1, int(2.0e7 // max(1, C * Km * Pm)))
    for r0 in range(0, R, chunk):
        r1 = min(R, r0 + chunk)
        prod = fv_pad[r0:r1, None, :, None] * fu_pad[None, :, None, :]   # [r, c, k, p]
        keep = prod >= cutoff
        if cone_mm is not None:
            keep &= (l2v_pad[r0:r1, None, :, None] + l2u_pad[None, :, None, :]) <= r2max
        rr, cc, kk, pp = np.nonzero(keep)
        vals = prod[rr, cc, kk, pp]
        iz = order_v[rr + r0, kk]
        p = order_u[cc, pp]
        rows_out.append((iz.astype(np.int64) * (N * N) + pidx[p]).astype(np.int32))
        cols_out.append((((a * R) + (rr + r0)) * C + cc).astype(np.int32))
        vals_out.append(vals.astype(np.float32))
    return (np.concatenate(rows_out), np.concatenate(cols_out), np.concatenate(vals_out))


def _threads() -> int:
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, min(n, 16))


def generate_ddc(plan: Plan, cps: Optional[List[int]] = None, threads: Optional[int] = None,
                 z_slab: Optional[Tuple[int, int]] = None, cutoff: float = CUTOFF,
                 cone_mm: Optional[float] = None):
    """COO of D (voxels x beamlets), sorted by (beamlet, voxel); unique pairs.
    z_slab = (z0, z1): only the rows of voxel slices z0 <= iz < z1 (global
    voxel indices), the share of one GPU in a split by voxel rows.
    cutoff, cone_mm: the truncation (generate_cp); the defaults give the
    complete matrix, and any truncation keeps a subset of its entries with
    the same values.

    Control points are generated on a thread pool (NumPy releases the GIL in
    its array loops); the result does not depend on the thread count.
    Returns dict(row=int32[nnz] voxel, col=int32[nnz] beamlet, val=float32[nnz])."""
    xy = body_xy(plan)
    cps = list(range(plan.n_cp) if cps is None else cps)
    nt = threads or _threads()
    if nt > 1 and len(cps) > 1:
        with ThreadPoolExecutor(nt) as ex:
            parts = list(ex.map(lambda a: generate_cp(plan, a, xy, z_slab, cutoff, cone_mm), cps))
    else:
        parts = [generate_cp(plan, a, xy, z_slab, cutoff, cone_mm) for a in cps]
    nnz = sum(len(p[0]) for p in parts)
    row = np.empty(nnz, np.int32)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float32)
    o = 0
    # copy part by part and drop each part once copied: the output's pages are
    # committed as they are written, so the peak stays near one copy
    parts.reverse()
    while parts:
        r_, c_, v_ = parts.pop()
        n = len(r_)
        row[o:o + n], col[o:o + n], val[o:o + n] = r_, c_, v_
        o += n
        del r_, c_, v_
    return dict(row=row, col=col, val=val)


def slice_counts(plan: Plan, threads: Optional[int] = None) -> np.ndarray:
    """Approximate number of stored entries in each voxel slice iz (int64[N]),
    without generating them: an entry is kept where f_v[r, iz] * f_u[c, p] >=
    CUTOFF, counted per (r, iz) by a search in the sorted f_u of each control
    point (threshold CUTOFF / f_v; rounding can move an entry at the edge).
    Used to cut balanced voxel slabs."""
    xy = body_xy(plan)
    px, py, _ = xy
    u_c, v_r = beamlet_offsets(plan)
    fv = _v_factors(plan, v_r)                                        # [R, N]
    with np.errstate(divide="ignore", over="ignore"):
        thr = np.where(fv > 0, CUTOFF / fv, np.inf)

    def one(a):
        fs = np.sort(_angle_factors(plan, a, px, py, u_c).ravel())
        return (len(fs) - np.searchsorted(fs, thr, side="left")).sum(axis=0)

    nt = threads or _threads()
    with ThreadPoolExecutor(nt) as ex:
        return np.sum(list(ex.map(one, range(plan.n_cp))), axis=0).astype(np.int64)


def balanced_slabs(plan: Plan, G: int, counts: Optional[np.ndarray] = None) -> List[Tuple[int, int]]:
    """G contiguous voxel-slice ranges with about equal entry counts."""
    c = slice_counts(plan) if counts is None else counts
    cum = np.concatenate([[0], np.cumsum(c)])
    cuts = [0]
    for k in range(1, G):
        z = int(np.searchsorted(cum, cum[-1] * k / G))
        cuts.append(min(max(z, cuts[-1] + 1), plan.n_grid - (G - k)))
    cuts.append(plan.n_grid)
    return [(cuts[k], cuts[k + 1]) for k in range(G)]


def ddc_entries(plan: Plan, vox: np.ndarray, bl: np.ndarray, cutoff: float = CUTOFF,
                cone_mm: Optional[float] = None) -> np.ndarray:
    """D_ij (float32, 0 where dropped) for explicit (voxel, beamlet) pairs.

    Same definition as generate_ddc, evaluated pointwise; used to sample rows
    or columns of matrices too large to hold on the host."""
    N, h = plan.n_grid, plan.vox_mm
    vox = np.asarray(vox, np.int64)
    bl = np.asarray(bl, np.int64)
    ix, iy, iz = vox % N, (vox // N) % N, vox // (N * N)
    px = (ix - (N - 1) / 2.0) * h
    py = (iy - (N - 1) / 2.0) * h
    pz = (iz - (N - 1) / 2.0) * h
    c = bl % plan.n_cols
    r = (bl // plan.n_cols) % plan.n_rows
    a = bl // (plan.n_cols * plan.n_rows)
    u_c = (c - (plan.n_cols - 1) / 2.0) * plan.bl_mm
    v_r = (r - (plan.n_rows - 1) / 2.0) * plan.bl_mm
    sin_t = np.array([math.sin(cp_angle(plan, k)) for k in range(plan.n_cp)])
    cos_t = np.array([math.cos(cp_angle(plan, k)) for k in range(plan.n_cp)])
    s, co = sin_t[a], cos_t[a]
    t = px * s - py * co
    pu = px * co + py * s
    R = plan.body_radius
    depth = np.maximum(0.0, t + np.sqrt(np.maximum(R * R - u_c * u_c, 0.0)))
    fu = np.exp(-MU_PER_MM * depth) * np.exp(-((pu - u_c) ** 2) / (2.0 * SIGMA_MM ** 2))
    fv = np.exp(-((pz - v_r) ** 2) / (2.0 * SIGMA_MM ** 2))
    d = fu * fv
    inside = (px * px + py * py) <= R * R
    keep = inside & (d >= cutoff)
    if cone_mm is not None:
        keep &= ((pu - u_c) ** 2 + (pz - v_r) ** 2) <= float(cone_mm) ** 2
    return np.where(keep, d, 0.0).astype(np.float32)


def structures(plan: Plan):
    """(struct_id uint8[n_vox], table float32[n_struct, 3] of (T, w_over, w_under))."""
    N, h, R = plan.n_grid, plan.vox_mm, plan.body_radius
    c = axis_centres(N, h)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    sid = np.zeros((N, N, N), np.uint8)
    sid[(xx * xx + yy * yy) <= R * R] = S_BODY
    body = sid == S_BODY

    def sphere(cx, cy, cz, rad):
        return ((xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2) <= rad * rad

    sid[body & sphere(0.0, 0.75 * R, 0.0, 0.2 * R)] = S_OAR_A
    sid[body & sphere(0.6 * R, -0.35 * R, 0.0, 0.15 * R)] = S_OAR_B
    table = [(0.0, 0.0, 0.0), (42.0, 0.1, 0.0), (45.0, 0.5, 0.0), (26.0, 0.5, 0.0)]
    for k, (cx, cy, cz, rad, T) in enumerate(plan.ptv_list()):
        sid[body & sphere(cx, cy, cz, rad)] = S_PTV0 + k
        table.append((T, 1.0, 1.0))
    return sid.ravel(), np.asarray(table, np.float32)


def bench_vectors(n_bl: int, n_vox: int, seed: int):
    """x ~ U[0,1) (fluence-like, non-negative) and g ~ N(0,1) (gradient-like)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random(n_bl, dtype=np.float64).astype(np.float32)
    g = rng.standard_normal(n_vox, dtype=np.float64).astype(np.float32)
    return x, g


def random_boxes(m: int, seed: int):
    """Finite per-aperture boxes [lo, hi] with 0 <= lo < hi."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = rng.uniform(0.0, 0.2, m)
    hi = lo + rng.uniform(0.05, 1.0, m)
    return lo.astype(np.float32), hi.astype(np.float32)


def random_apertures(plan: Plan, m: int, seed: int):
    """m apertures at distinct control points, each leaf row a uniform
    non-empty half-open interval [L, R).  Returns (cps int32[m],
    L int32[m, n_rows], R int32[m, n_rows])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cps = np.sort(rng.choice(plan.n_cp, size=m, replace=False)).astype(np.int32)
    n = plan.n_cols
    a = rng.integers(0, n, size=(m, plan.n_rows))
    b = rng.integers(0, n, size=(m, plan.n_rows))
    L = np.minimum(a, b).astype(np.int32)
    R = (np.maximum(a, b) + 1).astype(np.int32)
    return cps, L, R


def random_sparse(n_rows: int, n_cols: int, density: float, seed: int,
                  empty_rows: int = 0, empty_cols: int = 0):
    """Unstructured non-negative COO with some empty rows/columns (edge cases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = rng.random((n_rows, n_cols)) < density
    if empty_rows:
        mask[rng.choice(n_rows, size=min(empty_rows, n_rows), replace=False)] = False
    if empty_cols:
        mask[:, rng.choice(n_cols, size=min(empty_cols, n_cols), replace=False)] = False
    c, r = np.nonzero(mask.T)            # sorted by (col, row), like the DDC generator
    v = rng.uniform(1e-3, 1.0, size=len(r))
    return dict(row=r.astype(np.int32), col=c.astype(np.int32), val=v.astype(np.float32))
