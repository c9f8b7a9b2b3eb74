"""The region X of the diagram: an axis-aligned box or a convex polygon -- TEST INFRASTRUCTURE
ONLY.

Remark 11.1 allows any convex polygon X.  Side e of a polygon with vertices v_0..v_{K-1}
(counter-clockwise) runs from v_e to v_{e+1}, is named -(e+1), and lies on N.x <= N.v_e with
N = (dy, -dx) / gcd(|dx|, |dy|) for (dx, dy) = v_{e+1} - v_e: the primitive outward normal.  A
box is the polygon (x0,y0), (x1,y0), (x1,y1), (x0,y1), which gives the box codes -1 (y = y0),
-2 (x = x1), -3 (y = y1), -4 (x = x0) with unit normals.
"""
from __future__ import annotations

from fractions import Fraction as F
from math import gcd


def vertices(box, region=None):
    """Integer vertices (x, y), counter-clockwise, side e from vertex e to vertex e + 1."""
    if region is None:
        x0, y0, x1, y1 = (int(v) for v in box)
        return [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    vx, vy = region
    return [(int(a), int(b)) for a, b in zip(vx, vy)]


def side_lines(box, region=None):
    """[(Nx, Ny, c)] of the sides, code -(e+1) at index e."""
    v = vertices(box, region)
    K = len(v)
    out = []
    for e in range(K):
        (ax, ay), (bx, by) = v[e], v[(e + 1) % K]
        dx, dy = bx - ax, by - ay
        g = gcd(abs(dx), abs(dy))
        nx, ny = dy // g, -dx // g
        out.append((nx, ny, nx * ax + ny * ay))
    return out


def area(box, region=None):
    """Exact area of X (shoelace)."""
    v = vertices(box, region)
    s = 0
    for (ax, ay), (bx, by) in zip(v, v[1:] + v[:1]):
        s += ax * by - ay * bx
    return F(s, 2)


def contains(lines, px, py):
    """p in the closed region (exact; coordinates may be Fractions)."""
    return all(nx * px + ny * py <= c for nx, ny, c in lines)
