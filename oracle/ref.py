"""Independent exact-rational reference for small inputs -- TEST INFRASTRUCTURE ONLY.

Same definition as the C oracle (Section 2, Definition of the Voronoi diagram: the cell is X
intersected with the bisector half-planes), computed differently: the polygon is a list of
rational vertices (Python ``Fraction``) with the label of the edge that leaves each vertex, and
each half-plane is applied by clipping the vertex cycle against it.  Pure Python loops, so
only for a few hundred sites.
"""
from __future__ import annotations

from fractions import Fraction as F

from . import region as _region


def _line(x, y, k, j):
    """(Nx, Ny, c) of the closed bisector half-plane N.v <= c bounding the cell of site k."""
    return (2 * (x[j] - x[k]), 2 * (y[j] - y[k]),
            (x[j] ** 2 + y[j] ** 2) - (x[k] ** 2 + y[k] ** 2))


def cell(x, y, box, k, region=None):
    """Counter-clockwise list of line labels of the cell of site k (not rotated).  X is the box,
    or the convex polygon region = (vx, vy) when given."""
    x = [int(v) for v in x]
    y = [int(v) for v in y]
    # vertices of X counter-clockwise; label = line of the edge leaving the vertex
    poly = [((F(a), F(b)), -(e + 1)) for e, (a, b) in enumerate(_region.vertices(box, region))]
    for j in range(len(x)):
        if j == k:
            continue
        nx, ny, c = _line(x, y, k, j)
        f = [c - (nx * v[0] + ny * v[1]) for v, _ in poly]
        if all(fv >= 0 for fv in f):
            continue
        m = len(poly)
        out = []
        for i in range(m):
            (a, lab) = poly[i]
            (b, _) = poly[(i + 1) % m]
            fa, fb = f[i], f[(i + 1) % m]
            if fa >= 0:
                out.append((a, j if (fa == 0 and fb < 0) else lab))
            if (fa > 0 and fb < 0) or (fa < 0 and fb > 0):
                t = fa / (fa - fb)
                xpt = (a[0] + (b[0] - a[0]) * t, a[1] + (b[1] - a[1]) * t)
                out.append((xpt, j if fa > 0 else lab))
        poly = out
    return [lab for _, lab in poly], [v for v, _ in poly]


def rotate_canonical(ids):
    if not ids:
        return ids
    i = min(range(len(ids)), key=lambda t: ids[t] & 0xFFFFFFFF)
    return ids[i:] + ids[:i]


def diagram(x, y, box, region=None):
    """All cells, canonically rotated: list of label lists."""
    return [rotate_canonical(cell(x, y, box, k, region)[0]) for k in range(len(x))]
