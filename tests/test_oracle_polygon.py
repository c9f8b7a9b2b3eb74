"""Pins of the oracle for a convex polygon X (Remark 11.1 on a general convex region), CPU only.

Side e of X runs from vertex e to vertex e + 1 (counter-clockwise) and is named -(e+1); its line
uses the primitive outward normal.  The pins: brute force (every corner of X, bisector / side
point and circumcentre, exact) == C oracle == Fraction reference on tiny sets in random convex
polygons; closed forms (one site: the cell is X; a box given as a polygon gives the box's
diagram); invariants (tiling of X by exact areas, Euler, symmetry, empty circles); the bound on
the total number of edges for a polygon with |X_e| sides; input validation.
"""
import numpy as np
import pytest

import sitegen
from oracle import brute, cdiagram, checks, ref
from oracle import region as oregion


def c_cells(ps, which=None):
    c = cdiagram.cells(ps.x, ps.y, ps.box, which=which, threads=4, region=ps.region)
    return [c.lines(i) for i in range(c.cells.shape[0])], c


def tiny_polygon_set(seed):
    """2..8 sites in a polygon with 3..12 sides and small integer coordinates (a thin polygon
    with too few interior points is replaced by the next seed's)."""
    K = 3 + seed % 10
    n = 2 + seed % 7
    for t in range(10):
        reg = sitegen.convex_polygon(K, 40 + 8 * (seed % 4), seed=300 + seed + 1000 * t)
        try:
            return sitegen.in_polygon(n, reg, seed=400 + seed)
        except ValueError:
            continue
    raise AssertionError("no polygon")


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_matches_oracle_in_polygons(seed):
    """Small integer coordinates (many ties), polygons with 3 to 12 sides."""
    ps = tiny_polygon_set(seed)
    cl, _ = c_cells(ps)
    b, _ = brute.diagram(ps.x, ps.y, ps.box, region=ps.region)
    assert cl == [ref.rotate_canonical(v) for v in b]
    assert cl == ref.diagram(ps.x, ps.y, ps.box, region=ps.region)
    checks.check_all(ps.x, ps.y, ps.box, cl, region=ps.region)


@pytest.mark.parametrize("K", [3, 5, 16, 64])
def test_single_site_is_the_polygon(K):
    reg = sitegen.convex_polygon(K, 1 << 16, seed=K)
    Kr = len(reg[0])
    ps = sitegen.in_polygon(1, reg, seed=1)
    cl, c = c_cells(ps)
    # the sides in order, rotated to start at the smallest uint32 label (-K)
    want = [-(e + 1) for e in range(Kr)]
    i = want.index(-Kr)
    assert cl[0] == want[i:] + want[:i]
    # vertex t of the cell is the polygon's vertex where its two sides meet
    V = oregion.vertices(ps.box, ps.region)
    for t in range(Kr):
        a = cl[0][t]
        X, Y, D = int(c.vx[t]), int(c.vy[t]), int(c.vd[t])
        assert (X, Y) == (V[(-a) % Kr][0] * D, V[(-a) % Kr][1] * D)


def test_box_as_polygon_gives_the_box_diagram():
    ps = sitegen.uniform(3000, 1 << 16, seed=9)
    x0, y0, x1, y1 = ps.box
    reg = (np.array([x0, x1, x1, x0], np.int32), np.array([y0, y0, y1, y1], np.int32))
    a = cdiagram.cells(ps.x, ps.y, ps.box)
    b = cdiagram.cells(ps.x, ps.y, ps.box, region=reg)
    assert np.array_equal(a.nbr, b.nbr) and np.array_equal(a.off, b.off)
    assert list(a.vx) == list(b.vx) and list(a.vy) == list(b.vy) and list(a.vd) == list(b.vd)


@pytest.mark.parametrize("kind,K", [("uniform", 6), ("uniform", 40), ("clustered", 16)])
def test_invariants_in_polygons(kind, K):
    reg = sitegen.convex_polygon(K, 1 << 20, seed=K + 17)
    ps = sitegen.in_polygon(400, reg, seed=K, kind=kind)
    cl, _ = c_cells(ps)
    checks.check_all(ps.x, ps.y, ps.box, cl, region=ps.region)
    # Remark 11.1 / the bound on edges: sum e_k <= (|X_e| + 6) n for a convex polygon X
    Kr = len(ps.region[0])
    assert sum(len(c) for c in cl) <= (Kr + 6) * ps.n


def test_two_sites_split_a_triangle():
    vx = np.array([0, 100, 0], np.int32)
    vy = np.array([0, 0, 100], np.int32)
    x = np.array([20, 21], np.int32)
    y = np.array([20, 60], np.int32)
    c = cdiagram.cells(x, y, (0, 0, 100, 100), region=(vx, vy))
    cl = [c.lines(0), c.lines(1)]
    checks.check_all(x, y, (0, 0, 100, 100), cl, region=(vx, vy))
    assert 1 in cl[0] and 0 in cl[1]
    assert oregion.area((0, 0, 100, 100), (vx, vy)) == 5000


@pytest.mark.parametrize("name,vx,vy,code", [
    ("clockwise", [0, 0, 100], [0, 100, 0], -1),
    ("collinear", [0, 50, 100, 0], [0, 0, 0, 100], -1),
    ("not convex", [0, 100, 30, 0], [0, 0, 30, 100], -1),
    ("pentagram", [0, 60, -40, 40, -60], [100, -80, 30, 30, -80], -1),
    ("two vertices", [0, 100], [0, 0], -1),
    ("too wide", [0, (1 << 24) + 1, 0], [0, 0, 100], -2),
])
def test_polygon_validation(name, vx, vy, code):
    x = np.array([10], np.int32)
    y = np.array([10], np.int32)
    r = cdiagram.validate(x, y, (0, 0, 1, 1), region=(np.array(vx, np.int32),
                                                       np.array(vy, np.int32)))
    assert r == code, name


def test_sites_outside_the_polygon_are_rejected():
    vx = np.array([0, 100, 0], np.int32)
    vy = np.array([0, 0, 100], np.int32)
    for px, py in [(60, 60), (-1, 5), (51, 50)]:   # outside
        r = cdiagram.validate(np.array([px], np.int32), np.array([py], np.int32),
                              (0, 0, 100, 100), region=(vx, vy))
        assert r == -2, (px, py)
    for px, py in [(50, 50), (0, 10), (0, 0)]:     # on the hypotenuse, a side, a vertex
        r = cdiagram.validate(np.array([px], np.int32), np.array([py], np.int32),
                              (0, 0, 100, 100), region=(vx, vy))
        assert r == 0, (px, py)
    r = cdiagram.validate(np.array([10, 10], np.int32), np.array([10, 10], np.int32),
                          (0, 0, 100, 100), region=(vx, vy))
    assert r == -3
