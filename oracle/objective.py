"""Voxel-wise one-sided quadratic objective, in float64.  Test infrastructure only.

Eq. (1):  F(z) = sum_i w+_i max(0, z_i - T_i)^2 + w-_i max(0, T_i - z_i)^2
with w+ the over-dose weight and w- the under-dose weight (the reading of
Eq. (1) and the sentence after it; one later sentence in Sec. 2.2.2 swaps the
two names).  Per-voxel parameters come from a structure id and a table of
(T, w+, w-) rows, the replicated "structure indices" of Sec. 2.2.2.

Eq. (4) defines g = -grad F; this module returns grad F itself:
    dF/dz_i = 2 w+_i max(0, z_i - T_i) - 2 w-_i max(0, T_i - z_i).
"""
from __future__ import annotations

import numpy as np


def voxel_params(sid, table):
    t = np.asarray(table, np.float64)
    sid = np.asarray(sid, np.int64)
    return t[sid, 0], t[sid, 1], t[sid, 2]


def objective(z, sid, table):
    """F(z) of Eq. (1).  z is [n_vox] or [n_vox, nrhs] (then F is [nrhs])."""
    T, wo, wu = voxel_params(sid, table)
    z = np.asarray(z, np.float64)
    if z.ndim == 2:
        T, wo, wu = T[:, None], wo[:, None], wu[:, None]
    over = np.maximum(0.0, z - T)
    under = np.maximum(0.0, T - z)
    return np.sum(wo * over * over + wu * under * under, axis=0)


def gradient(z, sid, table):
    """grad F(z) (= -g of Eq. (4))."""
    T, wo, wu = voxel_params(sid, table)
    z = np.asarray(z, np.float64)
    if z.ndim == 2:
        T, wo, wu = T[:, None], wo[:, None], wu[:, None]
    return 2.0 * wo * np.maximum(0.0, z - T) - 2.0 * wu * np.maximum(0.0, T - z)


def curvature(d, z, sid, table):
    """sum_i w_i(z) d_i^2, w_i = w+ where z_i > T_i, w- where z_i < T_i, 0 at z_i = T_i.

    Half the second derivative of F(z + a d) in a on the quadratic piece that
    contains z; the first BB step length of the master problem uses it."""
    T, wo, wu = voxel_params(sid, table)
    z = np.asarray(z, np.float64)
    w = np.where(z > T, wo, np.where(z < T, wu, 0.0))
    d = np.asarray(d, np.float64)
    return float(np.sum(w * d * d))
