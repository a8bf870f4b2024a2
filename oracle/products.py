"""Sparse DDC products over COO, in float64.  Test infrastructure only.

D is voxels x beamlets, given as COO triplets (row = voxel, col = beamlet,
val); duplicate pairs are summed, as COO semantics imply.

* dose:  z_i = sum_j D_ij x_j          (the dose of Sec. 2.1, z = sum_k DA(A_k) y_k
                                        written per beamlet)
* price: p_j = sum_i D_ij g_i          (Eq. 3; the paper's price is pi = D^T (-grad F))
* aperture_ddc: DA_i(A) = sum_{j in A} D_ij   (Eq. 5)
"""
from __future__ import annotations

import numpy as np

_CHUNK = 1 << 26


def _spmv(out_idx, in_idx, val, vec, n_out):
    vec = np.asarray(vec, dtype=np.float64)
    if vec.ndim == 1:
        out = np.zeros(n_out, np.float64)
        for s in range(0, len(val), _CHUNK):
            e = s + _CHUNK
            out += np.bincount(out_idx[s:e],
                               weights=val[s:e].astype(np.float64) * vec[in_idx[s:e]],
                               minlength=n_out)
        return out
    return np.stack([_spmv(out_idx, in_idx, val, vec[:, k], n_out)
                     for k in range(vec.shape[1])], axis=1)


def dose(row, col, val, x, n_vox):
    """z = D x.  x is [n_bl] or [n_bl, nrhs]; returns float64 of matching shape."""
    return _spmv(row, col, val, x, n_vox)


def price(row, col, val, g, n_bl):
    """p = D^T g (Eq. 3 with g the objective gradient; pi = -p).  g is [n_vox] or [n_vox, nrhs]."""
    return _spmv(col, row, val, g, n_bl)


def aperture_ddc(row, col, val, member, n_vox):
    """DA(A) = sum of the columns of D whose beamlets are in A (Eq. 5).

    member: bool[n_bl] beamlet membership of the aperture."""
    sel = np.asarray(member, bool)[col]
    return np.bincount(row[sel], weights=val[sel].astype(np.float64), minlength=n_vox)


def dose_rows(row, col, val, x, rows):
    """z_i for the listed voxel rows only (sampled parity on large matrices)."""
    rows = np.asarray(rows, np.int64)
    pos = {int(r): k for k, r in enumerate(rows)}
    sel = np.isin(row, rows)
    out = np.zeros(len(rows), np.float64)
    r, c, v = row[sel], col[sel], val[sel].astype(np.float64)
    idx = np.array([pos[int(t)] for t in r], np.int64) if len(r) else np.zeros(0, np.int64)
    np.add.at(out, idx, v * np.asarray(x, np.float64)[c])
    return out


def dense(row, col, val, n_vox, n_bl):
    """Dense float64 D (tiny matrices only)."""
    d = np.zeros((n_vox, n_bl), np.float64)
    np.add.at(d, (row, col), val.astype(np.float64))
    return d
