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


def _candidates(x, y, box):
    x0, y0, x1, y1 = box
    pts = {(F(x0), F(y0)), (F(x1), F(y0)), (F(x1), F(y1)), (F(x0), F(y1))}
    n = len(x)
    # bisector of (i, j) meets the four side lines
    for i, j in combinations(range(n), 2):
        nx, ny = 2 * (x[j] - x[i]), 2 * (y[j] - y[i])
        c = (x[j] ** 2 + y[j] ** 2) - (x[i] ** 2 + y[i] ** 2)
        for yy in (y0, y1):
            if nx != 0:
                pts.add((F(c - ny * yy, nx), F(yy)))
        for xx in (x0, x1):
            if ny != 0:
                pts.add((F(xx), F(c - nx * xx, ny)))
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
    return [p for p in pts if x0 <= p[0] <= x1 and y0 <= p[1] <= y1]


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


def diagram(x, y, box):
    """List of CCW label lists (not rotated) per site, plus the hull vertices per site."""
    x = [int(v) for v in x]
    y = [int(v) for v in y]
    x0, y0, x1, y1 = box
    n = len(x)
    cand = _candidates(x, y, box)
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
            if a[1] == y0 and b[1] == y0:
                lab.append(-1)
            if a[0] == x1 and b[0] == x1:
                lab.append(-2)
            if a[1] == y1 and b[1] == y1:
                lab.append(-3)
            if a[0] == x0 and b[0] == x0:
                lab.append(-4)
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
