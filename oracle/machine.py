"""Machine constraints of Eq. (2) turned into the rate boxes of Eq. (6), in
float64.  Test infrastructure only.

The delivery model of Eq. (2): the gantry turns through control points
k = 0 .. K-1, a fixed angle apart, with speed s_k in [S^L, S^U], a speed
change |s_k - s_{k+1}| <= dS between consecutive points, a dose rate r_k in
[R^L, R^U], and s_k small enough for the MLC to move from aperture A_k to
A_{k+1} in the time the gantry takes to cross the gap (S^U_{k,k+1}).  The
master problem (Eq. 6) bounds the fluence rate of aperture k by
y_k in [R^L / S^U_k, R^U / S^L_k], with S^U_k, S^L_k the speed bounds at k that
the apertures already chosen at other control points leave.

Readings where the paper is silent (its constants come from references that
are not part of it):
* parameters: gantry_step (angle between control points), speed_min/max
  (S^L, S^U), speed_change (dS), rate_min/max (R^L, R^U), leaf_speed (the
  leaves' maximum speed, in beamlet widths per unit time);
* s_k is the speed on the arc from point k to k+1, so the leaf motion from
  A_k to A_{k+1} bounds s_k only, and only when both points hold apertures:
  with d the largest position change of any leaf (both leaves of every row,
  in beamlet widths, a closed row's leaves where the selection placed them),
  S^U_{k,k+1} = leaf_speed * gantry_step / d, or no bound when d = 0;
* S^U_k is the largest speed at k of any profile meeting the speed range, the
  leaf-motion bounds and the speed-change bound along the whole arc (the
  gantry also crosses the unoccupied points); upper bounds never raise a lower
  one, so S^L_k = S^L; with S^L = 0 the rate has no upper bound;
* a candidate aperture must be reachable from the apertures at occupied
  neighbouring points even at the slowest gantry speed: each leaf within
  floor(leaf_speed * gantry_step / S^L) beamlets of its position there (the
  leaf windows of aperture.py), which keeps every S^U_k >= S^L and every box
  non-empty.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Machine:
    gantry_step: float
    speed_min: float
    speed_max: float
    speed_change: float
    rate_min: float
    rate_max: float
    leaf_speed: float


def leaf_move(L0, R0, L1, R1):
    """Largest leaf position change between two apertures (beamlet widths)."""
    L0, R0, L1, R1 = (np.asarray(a, np.int64) for a in (L0, R0, L1, R1))
    return int(max(np.abs(L0 - L1).max(initial=0), np.abs(R0 - R1).max(initial=0)))


def pair_speed_bound(m: Machine, d):
    """S^U_{k,k+1} of Eq. (2) for a leaf move of d beamlet widths."""
    return math.inf if d == 0 else m.leaf_speed * m.gantry_step / d


def speed_upper(m: Machine, occupied, L, R):
    """S^U_k for every control point: start from S^U and the leaf-motion
    bounds, then lower each point to its neighbours' bound plus dS until no
    bound changes (the largest profile with |s_k - s_{k+1}| <= dS)."""
    occ = np.asarray(occupied, bool)
    K = len(occ)
    s = np.full(K, float(m.speed_max))
    for k in range(K - 1):
        if occ[k] and occ[k + 1]:
            s[k] = min(s[k], pair_speed_bound(m, leaf_move(L[k], R[k], L[k + 1], R[k + 1])))
    changed = True
    while changed:
        changed = False
        for k in range(K):
            for nb in (k - 1, k + 1):
                if 0 <= nb < K and s[nb] + m.speed_change < s[k]:
                    s[k] = s[nb] + m.speed_change
                    changed = True
    return s


def boxes(m: Machine, occupied, L, R):
    """(S^U_k, lo_k, hi_k) for every control point: the rate box of Eq. (6)."""
    s_hi = speed_upper(m, occupied, L, R)
    with np.errstate(divide="ignore"):
        lo = m.rate_min / s_hi
    hi = np.full(len(s_hi), math.inf if m.speed_min == 0 else m.rate_max / m.speed_min)
    return s_hi, lo, hi


def leaf_travel(m: Machine, n_cols):
    """Leaf travel of a candidate aperture from an occupied neighbour (beamlets)."""
    if m.speed_min == 0 or math.isinf(m.leaf_speed):
        return int(n_cols)
    return int(min(n_cols, math.floor(m.leaf_speed * m.gantry_step / m.speed_min)))
