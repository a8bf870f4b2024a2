"""Aperture selection by exhaustive enumeration, in float64.  Test infrastructure only.

Sec. 2.1 and Sec. 2.2.2: from the beamlet prices, pick at an unoccupied
control point the deliverable aperture with the best price.  Without the
interdigitation constraint the MLC leaf rows are independent, so the best
aperture is the best opening per row; the aperture price is the sum over rows
and the chosen control point is the best over the unoccupied ones.

Sign: the paper maximises the price pi = D^T(-grad F) (Eqs. 3-4).  Here the
input is p = D^T grad F = -pi, so the best opening MINIMISES the sum of p.

Readings where the paper is silent:
* an opening of leaf row r is a half-open beamlet interval [L, R),
  0 <= L <= R <= n_cols; the closed row is the empty interval, written (0, 0),
  with sum 0;
* ties: smallest sum, then shortest interval, then leftmost L; between
  control points: smallest price, then lowest index;
* an occupied control point gets L = R = 0 and price +inf;
* there is no improving aperture (the column generation stops) when the best
  price is >= 0; the selected index is then -1.
"""
from __future__ import annotations

import itertools

import numpy as np


def all_intervals(n):
    """Every opening of an n-beamlet row: the empty one first, then all [L, R)."""
    out = [(0, 0)]
    out += [(L, R) for L in range(n) for R in range(L + 1, n + 1)]
    return out


def best_intervals(rows):
    """Best opening of each row of prices.  rows: [m, n].  Returns (L, R, sum)."""
    rows = np.asarray(rows, np.float64)
    m, n = rows.shape
    ivs = all_intervals(n)
    Ls = np.array([a for a, _ in ivs])
    Rs = np.array([b for _, b in ivs])
    cs = np.concatenate([np.zeros((m, 1)), np.cumsum(rows, axis=1)], axis=1)
    sums = cs[:, Rs] - cs[:, Ls]                         # [m, n_int]
    sums[:, 0] = 0.0                                     # the closed row
    length = Rs - Ls
    # lexicographic (sum, length, L): smallest wins
    best = np.empty(m, np.int64)
    for i in range(m):
        order = np.lexsort((Ls, length, sums[i]))
        best[i] = order[0]
    return Ls[best].astype(np.int32), Rs[best].astype(np.int32), sums[np.arange(m), best]


def select(p, n_cp, n_rows, n_cols, occupied):
    """Aperture selection over all unoccupied control points.

    p: [n_cp*n_rows*n_cols] beamlet prices (j = (k*n_rows + r)*n_cols + c).
    Returns dict(L, R [n_cp, n_rows] int32, cp_price [n_cp] float64, best int,
    best_price float)."""
    P = np.asarray(p, np.float64).reshape(n_cp * n_rows, n_cols)
    L, R, S = best_intervals(P)
    L = L.reshape(n_cp, n_rows)
    R = R.reshape(n_cp, n_rows)
    cp_price = S.reshape(n_cp, n_rows).sum(axis=1)
    occ = np.asarray(occupied, bool)
    L[occ] = 0
    R[occ] = 0
    cp_price[occ] = np.inf
    best = -1
    best_price = np.inf
    for k in range(n_cp):
        if not occ[k] and cp_price[k] < best_price:
            best, best_price = k, cp_price[k]
    if best >= 0 and not best_price < 0.0:
        best = -1
    return dict(L=L, R=R, cp_price=cp_price, best=best, best_price=best_price)


# ---------------------------------------------------------------- leaf windows
#
# Sec. 2.1: candidate apertures must be deliverable from the apertures already
# chosen at the neighbouring control points (the leaves travel a bounded
# distance between control points).  Readings: the bound is a maximum leaf
# travel of `travel` beamlets per control-point step; it gives each leaf row a
# window (Lmin, Lmax, Rmin, Rmax) of allowed leaf positions, intersected over
# the occupied neighbours k-1 and k+1; an opening [L, R) is allowed iff
# Lmin <= L <= Lmax and Rmin <= R <= Rmax; a closed row parks both leaves at
# one allowed position p (L = R = p, sum 0).  Ties as above: smallest sum,
# then shortest, then smallest L (so a closed row parks at the smallest
# allowed p; with the full window that is (0, 0)).  A row with no allowed
# opening makes its control point infeasible: price +inf, L = R = 0.

def full_windows(n_cp, n_rows, n_cols):
    w = np.zeros((n_cp, n_rows, 4), np.int32)
    w[..., 1] = n_cols
    w[..., 3] = n_cols
    return w


def leaf_windows(n_cp, n_rows, n_cols, occupied, L, R, travel):
    """Windows [n_cp, n_rows, 4] (Lmin, Lmax, Rmin, Rmax) from the openings L, R
    [n_cp, n_rows] of the occupied control points."""
    occ = np.asarray(occupied, bool)
    w = full_windows(n_cp, n_rows, n_cols)
    for k in range(n_cp):
        for nb in (k - 1, k + 1):
            if 0 <= nb < n_cp and occ[nb]:
                for r in range(n_rows):
                    w[k, r, 0] = max(w[k, r, 0], L[nb][r] - travel)
                    w[k, r, 1] = min(w[k, r, 1], L[nb][r] + travel)
                    w[k, r, 2] = max(w[k, r, 2], R[nb][r] - travel)
                    w[k, r, 3] = min(w[k, r, 3], R[nb][r] + travel)
    return w


def allowed(state, win):
    (a, b), (lmin, lmax, rmin, rmax) = state, win
    return lmin <= a <= lmax and rmin <= b <= rmax


def best_row_windowed(row, win):
    """Best allowed opening of one row by enumeration: (L, R, sum) or None."""
    row = np.asarray(row, np.float64)
    best = None
    for (a, b) in states(len(row)):
        if not allowed((a, b), win):
            continue
        key = (row[a:b].sum(), b - a, a)
        if best is None or key < best[0]:
            best = (key, a, b)
    if best is None:
        return None
    return best[1], best[2], best[0][0]


def select_windowed(p, n_cp, n_rows, n_cols, occupied, windows):
    """Aperture selection with leaf windows [n_cp, n_rows, 4] (rows independent)."""
    P = np.asarray(p, np.float64).reshape(n_cp, n_rows, n_cols)
    occ = np.asarray(occupied, bool)
    L = np.zeros((n_cp, n_rows), np.int32)
    R = np.zeros((n_cp, n_rows), np.int32)
    cp_price = np.full(n_cp, np.inf)
    for k in range(n_cp):
        if occ[k]:
            continue
        rows = [best_row_windowed(P[k, r], windows[k][r]) for r in range(n_rows)]
        if any(x is None for x in rows):
            continue
        L[k] = [x[0] for x in rows]
        R[k] = [x[1] for x in rows]
        cp_price[k] = sum(x[2] for x in rows)
    return _pick(L, R, cp_price, occ)


def _pick(L, R, cp_price, occ):
    best, best_price = -1, np.inf
    for k in range(len(cp_price)):
        if not occ[k] and cp_price[k] < best_price:
            best, best_price = k, cp_price[k]
    if best >= 0 and not best_price < 0.0:
        best = -1
    return dict(L=L, R=R, cp_price=cp_price, best=best, best_price=best_price)


def best_aperture_bruteforce(p_cp):
    """Best whole aperture of one control point by enumerating the Cartesian
    product of every row's openings (tiny grids only).  p_cp: [n_rows, n_cols].

    Returns (price, openings tuple).  Independent of the row decomposition,
    so it checks that decomposition."""
    p_cp = np.asarray(p_cp, np.float64)
    n_rows, n_cols = p_cp.shape
    ivs = all_intervals(n_cols)
    row_sums = [[p_cp[r, a:b].sum() if b > a else 0.0 for (a, b) in ivs] for r in range(n_rows)]
    best, arg = np.inf, None
    for combo in itertools.product(range(len(ivs)), repeat=n_rows):
        s = sum(row_sums[r][combo[r]] for r in range(n_rows))
        if s < best:
            best, arg = s, tuple(ivs[c] for c in combo)
    return best, arg


def aperture_members(cp, L, R, n_cp, n_rows, n_cols):
    """bool[n_bl] membership of the aperture with openings [L_r, R_r) at control point cp."""
    m = np.zeros((n_cp, n_rows, n_cols), bool)
    for r in range(n_rows):
        m[cp, r, int(L[r]):int(R[r])] = True
    return m.ravel()


# ---------------------------------------------------------------- interdigitation
#
# Sec. 2.2.2: with the interdigitation constraint L_r <= min(R_{r-1}, R_{r+1})
# the leaf rows are coupled; the paper enumerates the combinations of row
# openings per control point.  Readings: for adjacent rows the constraint is
# L_r <= R_{r+1} and L_{r+1} <= R_r; a closed row may park its leaves at any
# position p (L = R = p, sum 0), and where it parks matters for its
# neighbours.  The best aperture minimises the sum of p over its openings.

def states(n):
    """All openings (L, R), 0 <= L <= R <= n, closed rows included."""
    return [(L, R) for L in range(n + 1) for R in range(L, n + 1)]


def compatible(a, b):
    """Interdigitation between adjacent rows with openings a and b."""
    return a[0] <= b[1] and b[0] <= a[1]


def best_aperture_interdigitated_bruteforce(p_cp, windows=None):
    """Exhaustive search over the Cartesian product of row openings (tiny grids)."""
    p_cp = np.asarray(p_cp, np.float64)
    n_rows, n = p_cp.shape
    st = states(n)
    sums = [[p_cp[r, a:b].sum() for (a, b) in st] for r in range(n_rows)]
    best, arg = np.inf, None
    for combo in itertools.product(range(len(st)), repeat=n_rows):
        if windows is not None and any(not allowed(st[combo[r]], windows[r]) for r in range(n_rows)):
            continue
        if any(not compatible(st[combo[r]], st[combo[r + 1]]) for r in range(n_rows - 1)):
            continue
        s = sum(sums[r][combo[r]] for r in range(n_rows))
        if s < best:
            best, arg = s, tuple(st[c] for c in combo)
    return best, arg


def best_aperture_interdigitated(p_cp, windows=None):
    """Best aperture of one control point under interdigitation, by dynamic
    programming over the leaf rows: value[r][s] = rowsum_r(s) + min over
    states s' of row r-1 compatible with s of value[r-1][s'] (states outside
    a row's leaf window cost +inf).
    Returns (price, openings [(L, R)] per row); price +inf if infeasible."""
    p_cp = np.asarray(p_cp, np.float64)
    n_rows, n = p_cp.shape
    st = states(n)
    cs = np.concatenate([np.zeros((n_rows, 1)), np.cumsum(p_cp, axis=1)], axis=1)
    rowsum = np.array([[cs[r, b] - cs[r, a] for (a, b) in st] for r in range(n_rows)])
    if windows is not None:
        for r in range(n_rows):
            rowsum[r, [not allowed(x, windows[r]) for x in st]] = np.inf
    value = [rowsum[0].copy()]
    choice = []
    comp = np.array([[compatible(s1, s2) for s2 in st] for s1 in st])   # [prev, cur]
    for r in range(1, n_rows):
        prev = value[-1]
        cand = np.where(comp, prev[:, None], np.inf)                     # [prev, cur]
        arg = np.argmin(cand, axis=0)
        value.append(rowsum[r] + cand[arg, np.arange(len(st))])
        choice.append(arg)
    last = int(np.argmin(value[-1]))
    path = [last]
    for r in range(n_rows - 1, 0, -1):
        path.append(int(choice[r - 1][path[-1]]))
    path.reverse()
    return float(value[-1][last]), [st[i] for i in path]


def select_interdigitated(p, n_cp, n_rows, n_cols, occupied, windows=None):
    """Aperture selection under interdigitation over the unoccupied control
    points (optionally within leaf windows [n_cp, n_rows, 4])."""
    P = np.asarray(p, np.float64).reshape(n_cp, n_rows, n_cols)
    occ = np.asarray(occupied, bool)
    L = np.zeros((n_cp, n_rows), np.int32)
    R = np.zeros((n_cp, n_rows), np.int32)
    cp_price = np.full(n_cp, np.inf)
    for k in range(n_cp):
        if occ[k]:
            continue
        v, path = best_aperture_interdigitated(P[k], None if windows is None else windows[k])
        if not np.isfinite(v):
            continue
        cp_price[k] = v
        L[k] = [a for a, _ in path]
        R[k] = [b for _, b in path]
    best, best_price = -1, np.inf
    for k in range(n_cp):
        if not occ[k] and cp_price[k] < best_price:
            best, best_price = k, cp_price[k]
    if best >= 0 and not best_price < 0.0:
        best = -1
    return dict(L=L, R=R, cp_price=cp_price, best=best, best_price=best_price)
