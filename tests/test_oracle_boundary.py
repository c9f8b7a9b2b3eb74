"""Pins of the oracle for sites on the boundary of X (CPU only).

The problem statement of Section 2 places the sites in the interior of X and notes that the
definition extends to sites on its boundary; the cell is still X intersected with the closed
half-planes of the other sites.  Closed forms (a site at a corner, sites on opposite sides, the
four corners, a lattice that fills the closed box), brute force == C oracle == Fraction
reference on tiny tie-heavy sets with boundary sites in boxes and polygons, and the invariants
on moderate sets."""
from fractions import Fraction as F

import numpy as np
import pytest

import sitegen
from oracle import brute, cdiagram, checks, ref


def lines_and_points(x, y, box, region=None):
    c = cdiagram.cells(np.array(x, np.int32), np.array(y, np.int32), box, region=region)
    pts = [[(F(int(a), int(d)), F(int(b), int(d))) for a, b, d in
            zip(c.vx[c.off[i]:c.off[i + 1]], c.vy[c.off[i]:c.off[i + 1]],
                c.vd[c.off[i]:c.off[i + 1]])] for i in range(len(x))]
    return [c.lines(i) for i in range(len(x))], pts


def test_site_at_a_corner_owns_the_box():
    cl, pts = lines_and_points([0], [0], (0, 0, 10, 10))
    assert cl[0] == [-4, -1, -2, -3]
    assert pts[0] == [(0, 0), (10, 0), (10, 10), (0, 10)]


def test_sites_on_opposite_sides_split_in_the_middle():
    cl, pts = lines_and_points([0, 10], [5, 5], (0, 0, 10, 10))
    assert cl[0] == [1, -3, -4, -1]          # x <= 5: bisector, top, left, bottom
    assert cl[1] == [0, -1, -2, -3]
    assert sorted(pts[0]) == [(0, 0), (0, 10), (5, 0), (5, 10)]


def test_four_corners_give_four_squares():
    x, y = [0, 10, 10, 0], [0, 0, 10, 10]
    cl, pts = lines_and_points(x, y, (0, 0, 10, 10))
    for k in range(4):
        assert len(cl[k]) == 4
        xs = sorted({p[0] for p in pts[k]})
        ys = sorted({p[1] for p in pts[k]})
        assert xs in ([0, 5], [5, 10]) and ys in ([0, 5], [5, 10])
    # the two diagonal pairs meet only at the centre: not neighbours (Section 7, via an edge)
    assert 2 not in cl[0] and 3 not in cl[1]


@pytest.mark.parametrize("k", [2, 3, 6])
def test_lattice_filling_the_closed_box(k):
    """Sites (i h, j h), i, j = 0 .. k-1, in X = [0, (k-1) h]^2: corner cells are h/2 squares,
    side cells h/2 x h rectangles, inner cells h squares; the Delaunay graph is the grid graph."""
    h = 8
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    x, y = (h * ii.ravel()).tolist(), (h * jj.ravel()).tolist()
    box = (0, 0, (k - 1) * h, (k - 1) * h)
    cl, pts = lines_and_points(x, y, box)
    for t in range(k * k):
        xs = [p[0] for p in pts[t]]
        ys = [p[1] for p in pts[t]]
        w = (max(xs) - min(xs), max(ys) - min(ys))
        i, j = ii.ravel()[t], jj.ravel()[t]
        ex = (F(h, 2) if i in (0, k - 1) else h, F(h, 2) if j in (0, k - 1) else h)
        assert w == ex, (t, w, ex)
    c = cdiagram.cells(np.array(x, np.int32), np.array(y, np.int32), box)
    assert cdiagram.delaunay(c).shape[0] == 2 * k * (k - 1)


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_matches_oracle_with_boundary_sites(seed):
    n = 2 + seed % 7
    coord = 4 + seed % 5
    ps = sitegen.small_integer_set(n, coord, seed=3000 + seed)
    ps = sitegen.with_boundary_sites(ps, 1 + seed % 4, seed=seed)
    assert cdiagram.validate(ps.x, ps.y, ps.box) == 0
    c = cdiagram.cells(ps.x, ps.y, ps.box, threads=2)
    cl = [c.lines(i) for i in range(ps.n)]
    b, _ = brute.diagram(ps.x, ps.y, ps.box)
    assert cl == [ref.rotate_canonical(v) for v in b]
    assert cl == ref.diagram(ps.x, ps.y, ps.box)
    checks.check_all(ps.x, ps.y, ps.box, cl)


@pytest.mark.parametrize("seed", range(20))
def test_brute_force_matches_oracle_with_sites_on_polygon_sides(seed):
    for t in range(20):
        try:
            reg = sitegen.convex_polygon(3 + seed % 6, 24 + 4 * (seed % 3),
                                         seed=5000 + seed + 97 * t)
            ps = sitegen.in_polygon(1 + seed % 4, reg, seed=6000 + seed)
            break
        except ValueError:
            continue
    ps = sitegen.with_boundary_sites(ps, 2 + seed % 3, seed=seed)
    assert cdiagram.validate(ps.x, ps.y, ps.box, region=ps.region) == 0
    c = cdiagram.cells(ps.x, ps.y, ps.box, threads=2, region=ps.region)
    cl = [c.lines(i) for i in range(ps.n)]
    b, _ = brute.diagram(ps.x, ps.y, ps.box, region=ps.region)
    assert cl == [ref.rotate_canonical(v) for v in b]
    assert cl == ref.diagram(ps.x, ps.y, ps.box, region=ps.region)
    checks.check_all(ps.x, ps.y, ps.box, cl, region=ps.region)


@pytest.mark.parametrize("kind", ["uniform", "lattice"])
def test_invariants_with_many_boundary_sites(kind):
    if kind == "uniform":
        ps = sitegen.uniform(600, 1 << 12, seed=8)
    else:
        ps = sitegen.lattice(400, 1 << 16, seed=9)
    ps = sitegen.with_boundary_sites(ps, 120, seed=10)
    c = cdiagram.cells(ps.x, ps.y, ps.box, threads=4)
    cl = [c.lines(i) for i in range(ps.n)]
    checks.check_all(ps.x, ps.y, ps.box, cl)


def test_outside_is_still_an_error():
    box = (0, 0, 16, 16)
    for x, y in [([-1, 3], [4, 4]), ([17, 3], [4, 4]), ([3, 3], [4, 17])]:
        assert cdiagram.validate(np.array(x, np.int32), np.array(y, np.int32), box) == -2
    assert cdiagram.validate(np.array([0, 16], np.int32), np.array([16, 0], np.int32), box) == 0
