"""Brute-force Voronoi diagram for n <= 8 -- TEST INFRASTRUCTURE ONLY.

Pins the oracle to something other than itself.  A vertex of a cell restricted to X is the
meeting point of two of its boundary lines, so it is one of: a corner of X, the point where
the bisector of two sites meets a side of X, or the circumcentre of three sites (the centre of
an empty circle).  The cell of site k is the convex hull of every such candidate point of X
whose nearest sites include k.  The label of a hull edge is the line that contains both of its
endpoints: a side of X, or the bisector of k and a site j equidistant from both endpoints.
Exact rationals throughout.
"""
from __future__ import annotations

from fractions import Fraction as F
from itertools import combinations

from . import region as _region


def _meet(l1, l2):
    """Intersection of two lines N.v = c, or None when parallel."""
    (ax, ay, ac), (bx, by, bc) = l1, l2
    d = ax * by - ay * bx
    if d == 0:
        return None
    return (F(ac * by - bc * ay, d), F(ax * bc - bx * ac, d))


def _candidates(x, y, sides, corners):
    pts = {(F(a), F(b)) for a, b in corners}
    n = len(x)
    # bisector of (i, j) meets every side line
    for i, j in combinations(range(n), 2):
        bis = (2 * (x[j] - x[i]), 2 * (y[j] - y[i]),
               (x[j] ** 2 + y[j] ** 2) - (x[i] ** 2 + y[i] ** 2))
        for sl in sides:
            p = _meet(bis, sl)
            if p is not None:
                pts.add(p)
    # circumcentres of non-collinear triples
    for i, j, k in combinations(range(n), 3):
        ax, ay, bx, by, cx, cy = x[i], y[i], x[j], y[j], x[k], y[k]
        d = 2 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
        if d == 0:
            continue
        a2, b2, c2 = ax * ax + ay * ay, bx * bx + by * by, cx * cx + cy * cy
        ux = F(a2 * (by - cy) + b2 * (cy - ay) + c2 * (ay - by), d)
        uy = F(a2 * (cx - bx) + b2 * (ax - cx) + c2 * (bx - ax), d)
        pts.add((ux, uy))
    return [p for p in pts if _region.contains(sides, p[0], p[1])]


def _hull(points):
    """Convex hull, counter-clockwise, collinear points dropped (monotone chain)."""
    pts = sorted(set(points))
    if len(pts) <= 2:
        return pts

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return lower[:-1] + upper[:-1]


def diagram(x, y, box, region=None):
    """List of CCW label lists (not rotated) per site, plus the hull vertices per site.  X is the
    box, or the convex polygon region = (vx, vy) when given."""
    x = [int(v) for v in x]
    y = [int(v) for v in y]
    sides = _region.side_lines(box, region)
    n = len(x)
    cand = _candidates(x, y, sides, _region.vertices(box, region))
    near = []
    for p in cand:
        d = [(p[0] - x[i]) ** 2 + (p[1] - y[i]) ** 2 for i in range(n)]
        m = min(d)
        near.append({i for i in range(n) if d[i] == m})
    cells, verts = [], []
    for k in range(n):
        pts = [p for p, s in zip(cand, near) if k in s]
        h = _hull(pts)
        labels = []
        for a, b in zip(h, h[1:] + h[:1]):
            lab = []
            for e, (nx, ny, c) in enumerate(sides):
                if nx * a[0] + ny * a[1] == c and nx * b[0] + ny * b[1] == c:
                    lab.append(-(e + 1))
            for j in range(n):
                if j == k:
                    continue
                ea = (a[0] - x[k]) ** 2 + (a[1] - y[k]) ** 2 == (a[0] - x[j]) ** 2 + (a[1] - y[j]) ** 2
                eb = (b[0] - x[k]) ** 2 + (b[1] - y[k]) ** 2 == (b[0] - x[j]) ** 2 + (b[1] - y[j]) ** 2
                if ea and eb:
                    lab.append(j)
            if len(lab) != 1:
                raise AssertionError(f"edge of cell {k} carries {lab}")
            labels.append(lab[0])
        cells.append(labels)
        verts.append(h)
    return cells, verts
