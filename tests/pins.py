"""Independent references that pin the oracle (no code shared with it).

* ``brute_force_hull`` -- the strictly convex hull from its definition: a
  directed pair (i, j) is a clockwise hull edge iff every point is right of or
  on i->j and every point on the line lies in the closed segment [i, j].  Exact
  integer arithmetic, O(u^3) for u distinct points.
* ``andrew_hull`` -- Andrew's monotone chain (cited in the paper's Section 1)
  with an exact integer cross product.
* ``exact_orient`` / ``rounded_orient`` -- the orientation value in exact
  rational arithmetic, and the binary64 value of the fixed formula computed by
  exact rationals plus correct rounding of each operation (``float(Fraction)``
  rounds to nearest even), i.e. without touching the host FPU.

All reference hulls use the same output convention as the method: strictly
convex vertices, each coordinate represented by its lowest index, clockwise
(y up) starting at the lexicographically smallest point.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact_orient(a, b, c) -> Fraction:
    ax, ay, bx, by, cx, cy = (Fraction(v) for v in (*a, *b, *c))
    return (ax - cx) * (by - cy) - (ay - cy) * (bx - cx)


def _rn(q: Fraction) -> float:
    return float(q)


def rounded_orient(a, b, c) -> float:
    """binary64 value of (a.x-c.x)*(b.y-c.y) - (a.y-c.y)*(b.x-c.x), each operation rounded."""
    F = Fraction
    t1 = _rn(F(a[0]) - F(c[0]))
    t2 = _rn(F(b[1]) - F(c[1]))
    t3 = _rn(F(a[1]) - F(c[1]))
    t4 = _rn(F(b[0]) - F(c[0]))
    m1 = _rn(F(t1) * F(t2))
    m2 = _rn(F(t3) * F(t4))
    return _rn(F(m1) - F(m2))


def _unique_lowest(x, y):
    """Distinct coordinates with the lowest index of each (dict keeps first)."""
    first = {}
    for i, (a, b) in enumerate(zip(x.tolist(), y.tolist())):
        key = (a + 0.0, b + 0.0)  # -0.0 and +0.0 are one coordinate
        if key not in first:
            first[key] = i
    return first


def _lexmin_lexmax(coords):
    pts = sorted(coords)
    return pts[0], pts[-1]


def brute_force_hull(x, y) -> list[int]:
    """Exact strictly convex hull of integer-valued inputs (|c| < 2^20)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    if n == 0:
        return []
    first = _unique_lowest(x, y)
    coords = list(first.keys())
    idx = [first[c] for c in coords]
    u = len(coords)
    if u == 1:
        return [idx[0]]
    X = np.array([int(c[0]) for c in coords], dtype=np.int64)
    Y = np.array([int(c[1]) for c in coords], dtype=np.int64)
    assert np.all(X == np.array([c[0] for c in coords])) and np.all(np.abs(X) < 2**20), "integer inputs only"
    assert np.all(Y == np.array([c[1] for c in coords])) and np.all(np.abs(Y) < 2**20), "integer inputs only"
    # O[i, j, k] = orient(P_i, P_j, P_k)
    Xi, Xj, Xk = X[:, None, None], X[None, :, None], X[None, None, :]
    Yi, Yj, Yk = Y[:, None, None], Y[None, :, None], Y[None, None, :]
    O = (Xi - Xk) * (Yj - Yk) - (Yi - Yk) * (Xj - Xk)
    lo, hi = _lexmin_lexmax(coords)
    if not np.any(O):  # every point on one line
        return [first[lo], first[hi]]
    right_or_on = np.all(O <= 0, axis=2)
    # collinear k must lie in the closed segment [i, j]
    dot_i = (Xk - Xi) * (Xj - Xi) + (Yk - Yi) * (Yj - Yi)
    dot_j = (Xk - Xj) * (Xi - Xj) + (Yk - Yj) * (Yi - Yj)
    inseg = (dot_i >= 0) & (dot_j >= 0)
    ok = right_or_on & np.all((O != 0) | inseg, axis=2)
    np.fill_diagonal(ok, False)
    succ = {}
    for i, j in zip(*np.nonzero(ok)):
        assert i not in succ, "a hull vertex has two outgoing hull edges"
        succ[int(i)] = int(j)
    start = coords.index(lo)
    out = [start]
    while True:
        nxt = succ[out[-1]]
        if nxt == start:
            break
        out.append(nxt)
        assert len(out) <= u
    assert len(out) == len(succ)
    return [idx[k] for k in out]


def andrew_hull(x, y) -> list[int]:
    """Andrew's monotone chain with exact integer arithmetic (integer-valued inputs)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if len(x) == 0:
        return []
    first = _unique_lowest(x, y)
    pts = sorted(first.keys())
    if len(pts) == 1:
        return [first[pts[0]]]
    P = [(int(a), int(b)) for a, b in pts]
    assert all(float(a) == c[0] and float(b) == c[1] for (a, b), c in zip(P, pts)), "integer inputs only"

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower = []
    for p in P:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    upper = []
    for p in reversed(P):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    ccw = lower[:-1] + upper[:-1]  # counterclockwise from the lexmin point
    if len(ccw) == 2 and ccw[0] == ccw[1]:
        ccw = ccw[:1]
    cw = [ccw[0]] + ccw[1:][::-1]
    lookup = {(int(a), int(b)): first[(a, b)] for a, b in pts}
    return [lookup[p] for p in cw]


def exact_hull_fraction(x, y) -> list[int]:
    """Exact strictly convex hull for arbitrary finite float inputs (Fractions), small n only."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    first = _unique_lowest(x, y)
    coords = list(first.keys())
    if not coords:
        return []
    if len(coords) == 1:
        return [first[coords[0]]]
    F = [(Fraction(a), Fraction(b)) for a, b in coords]
    lo, hi = _lexmin_lexmax(coords)
    # Andrew's chain in exact rationals
    order = sorted(range(len(coords)), key=lambda k: coords[k])

    def cross(o, a, b):
        return (F[a][0] - F[o][0]) * (F[b][1] - F[o][1]) - (F[a][1] - F[o][1]) * (F[b][0] - F[o][0])

    lower, upper = [], []
    for k in order:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], k) <= 0:
            lower.pop()
        lower.append(k)
    for k in reversed(order):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], k) <= 0:
            upper.pop()
        upper.append(k)
    ccw = lower[:-1] + upper[:-1]
    cw = [ccw[0]] + ccw[1:][::-1]
    assert coords[cw[0]] == lo
    return [first[coords[k]] for k in cw]
