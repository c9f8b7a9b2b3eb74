"""Invariant checkers for a Voronoi diagram restricted to a box or a convex polygon X -- TEST
INFRASTRUCTURE ONLY.

Every output of the oracle and of the GPU path can be run through these.  They check what the
mathematics fixes, independent of how the diagram was computed:

* symmetry     : j is a neighbour of k via an edge iff k is a neighbour of j (Section 7);
* convexity    : consecutive lines of a cell turn counter-clockwise (D > 0 in pair form);
* vertices     : every vertex is equidistant from k and the sites of its two lines, it lies in
                 X, and no site is strictly closer (Section 2, definition of the cell);
* area         : the cells tile X: the exact areas sum to the area of X;
* euler        : V - E + F = 1 for the planar subdivision of the disk X (F = n cells);
* delaunay     : the Delaunay edge count equals the number of interior Voronoi edges.
"""
from __future__ import annotations

from fractions import Fraction as F
from math import gcd

from . import region as _region


def line(x, y, box, k, j, region=None):
    """(Nx, Ny, c) of the line with label j in the cell of k, absolute coordinates."""
    if j >= 0:
        return (2 * (int(x[j]) - int(x[k])), 2 * (int(y[j]) - int(y[k])),
                (int(x[j]) ** 2 + int(y[j]) ** 2) - (int(x[k]) ** 2 + int(y[k]) ** 2))
    return _region.side_lines(box, region)[-int(j) - 1]


def pair_form(x, y, box, k, a, b, region=None):
    """Intersection of lines a and b of cell k by Cramer's rule: (X, Y, D), point = (X/D, Y/D)."""
    n1x, n1y, c1 = line(x, y, box, k, a, region)
    n2x, n2y, c2 = line(x, y, box, k, b, region)
    D = n1x * n2y - n1y * n2x
    X = c1 * n2y - c2 * n1y
    Y = n1x * c2 - n2x * c1
    return X, Y, D


def reduced(X, Y, D):
    g = gcd(gcd(abs(X), abs(Y)), abs(D))
    return (X // g, Y // g, D // g)


def check_symmetry(cells):
    n = len(cells)
    s = set()
    for k, ids in enumerate(cells):
        for j in ids:
            if j >= 0:
                assert 0 <= j < n and j != k, (k, j)
                s.add((k, int(j)))
    for (k, j) in s:
        assert (j, k) in s, f"asymmetric neighbours {k} -> {j}"
    return True


def check_cell_vertices(x, y, box, cells, every_site=True, region=None):
    """Convexity, equidistance and emptiness of every vertex; returns the reduced vertices."""
    n = len(x)
    sides = _region.side_lines(box, region)
    out = []
    for k, ids in enumerate(cells):
        m = len(ids)
        assert m >= 3, (k, ids)
        assert len(set(ids)) == m, f"repeated line in cell {k}: {ids}"
        vs = []
        for t in range(m):
            a, b = ids[t], ids[(t + 1) % m]
            X, Y, D = pair_form(x, y, box, k, a, b, region)
            assert D > 0, f"cell {k}: lines {a},{b} do not turn CCW"
            vx, vy = F(X, D), F(Y, D)
            assert _region.contains(sides, vx, vy)
            dk = (vx - int(x[k])) ** 2 + (vy - int(y[k])) ** 2
            for j in (a, b):
                if j >= 0:
                    assert (vx - int(x[j])) ** 2 + (vy - int(y[j])) ** 2 == dk
            if every_site:
                for j in range(n):
                    assert (vx - int(x[j])) ** 2 + (vy - int(y[j])) ** 2 >= dk, \
                        f"site {j} strictly closer to vertex of cell {k}"
            vs.append(reduced(X, Y, D))
        out.append(vs)
    return out


def check_area(x, y, box, cells, region=None):
    total = F(0)
    for k, ids in enumerate(cells):
        m = len(ids)
        pts = []
        for t in range(m):
            X, Y, D = pair_form(x, y, box, k, ids[t], ids[(t + 1) % m], region)
            pts.append((F(X, D), F(Y, D)))
        a = F(0)
        for t in range(m):
            (ax, ay), (bx, by) = pts[t], pts[(t + 1) % m]
            a += ax * by - ay * bx
        assert a > 0, f"cell {k} has non-positive area"
        total += a / 2
    assert total == _region.area(box, region), f"areas sum to {total}"
    return True


def check_euler(cells, reduced_vertices):
    V = set()
    E = set()
    for k, vs in enumerate(reduced_vertices):
        m = len(vs)
        for t in range(m):
            V.add(vs[t])
            a, b = vs[t - 1], vs[t]       # edge t runs from vertex t-1 to vertex t
            assert a != b, f"zero-length edge in cell {k}"
            E.add((a, b) if a < b else (b, a))
    n = len(cells)
    assert len(V) - len(E) + n == 1, f"V={len(V)} E={len(E)} F={n}"
    return True


def delaunay_pairs(cells):
    return sorted((k, int(j)) for k, ids in enumerate(cells) for j in ids if j > k)


def check_delaunay_count(cells, reduced_vertices):
    interior = set()
    for k, (ids, vs) in enumerate(zip(cells, reduced_vertices)):
        m = len(ids)
        for t in range(m):
            if ids[t] >= 0:
                a, b = vs[t - 1], vs[t]
                interior.add((a, b) if a < b else (b, a))
    assert len(interior) == len(delaunay_pairs(cells))
    return True


def check_all(x, y, box, cells, every_site=True, region=None):
    check_symmetry(cells)
    rv = check_cell_vertices(x, y, box, cells, every_site, region)
    check_area(x, y, box, cells, region)
    check_euler(cells, rv)
    check_delaunay_count(cells, rv)
    return True
