"""Pins of the Lloyd step of the oracle (CPU only): the double-precision centroid against the
exact rational centroid of the cell, closed forms (one site moves to the rounded centroid of X;
a square lattice at bucket centres is a fixed point), the collision rule, and the invariants
(sites stay distinct and strictly inside X)."""
from fractions import Fraction as F

import numpy as np
import pytest

import sitegen
from oracle import cdiagram, lloyd
from oracle import region as oregion


def exact_centroid(X, Y, D):
    pts = [(F(int(a), int(d)), F(int(b), int(d))) for a, b, d in zip(X, Y, D)]
    a2 = F(0)
    sx = F(0)
    sy = F(0)
    m = len(pts)
    for t in range(m):
        (x0, y0), (x1, y1) = pts[t], pts[(t + 1) % m]
        c = x0 * y1 - x1 * y0
        a2 += c
        sx += (x0 + x1) * c
        sy += (y0 + y1) * c
    return sx / (3 * a2), sy / (3 * a2)


@pytest.mark.parametrize("kind", ["uniform", "clustered", "polygon"])
def test_double_centroid_matches_the_exact_centroid(kind):
    if kind == "polygon":
        reg = sitegen.convex_polygon(9, 1 << 20, seed=4)
        ps = sitegen.in_polygon(800, reg, seed=5)
    else:
        ps = getattr(sitegen, kind)(800, 1 << 20, seed=6)
    oc = cdiagram.cells(ps.x, ps.y, ps.box, region=ps.region)
    worst = 0.0
    for k in range(ps.n):
        o0, o1 = int(oc.off[k]), int(oc.off[k + 1])
        px, py = int(ps.x[k]), int(ps.y[k])
        cx, cy = lloyd._centroid_offset(oc.vx[o0:o1], oc.vy[o0:o1], oc.vd[o0:o1], px, py)
        ex, ey = exact_centroid(oc.vx[o0:o1], oc.vy[o0:o1], oc.vd[o0:o1])
        worst = max(worst, abs(float(ex - px) - cx), abs(float(ey - py) - cy))
        # the rounding agrees with the exact centroid's unless it sits at a half-integer
        for e, c in ((ex - px, cx), (ey - py, cy)):
            frac = e - (e.numerator // e.denominator)
            if abs(frac - F(1, 2)) > F(1, 10 ** 6):
                assert int(np.rint(c)) == round(e), (k, e, c)
    assert worst < 1e-6


def test_one_site_moves_to_the_centroid_of_x():
    x, y, m, _ = lloyd.step(np.array([10], np.int32), np.array([20], np.int32), (0, 0, 100, 60))
    assert (int(x[0]), int(y[0]), m) == (50, 30, 1)
    vx = np.array([0, 90, 0], np.int32)
    vy = np.array([0, 0, 90], np.int32)
    x, y, m, _ = lloyd.step(np.array([5], np.int32), np.array([5], np.int32), (0, 0, 90, 90),
                            region=(vx, vy))
    assert (int(x[0]), int(y[0])) == (30, 30)   # centroid of the triangle


def test_square_lattice_at_cell_centres_is_a_fixed_point():
    k, h = 12, 10
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    x = (h // 2 + h * ii.ravel()).astype(np.int32)
    y = (h // 2 + h * jj.ravel()).astype(np.int32)
    nx, ny, moved = lloyd.iterate(x, y, (0, 0, k * h, k * h), 3)
    assert moved == [0, 0, 0]
    assert np.array_equal(nx, x) and np.array_equal(ny, y)


def test_collision_rule():
    x = np.array([0, 10, 20, 30], np.int64)
    y = np.zeros(4, np.int64)
    # sites 0 and 1 propose the same point; site 2 proposes site 3's current position while
    # site 3 stays: 0 and 1 go back, then 2 goes back
    qx = np.array([5, 5, 30, 30])
    qy = np.zeros(4, np.int64)
    nx, ny, rounds = lloyd.resolve(x, y, qx, qy)
    assert nx.tolist() == [0, 10, 20, 30] and rounds >= 1
    qx = np.array([5, 5, 25, 30])
    nx, ny, rounds = lloyd.resolve(x, y, qx, qy)
    assert nx.tolist() == [0, 10, 25, 30]


@pytest.mark.parametrize("kind", ["dense", "uniform", "polygon"])
def test_iterations_keep_sites_distinct_and_inside(kind):
    if kind == "dense":
        ps = sitegen.uniform(300, 40, seed=3)        # crowded: rounding makes collisions
    elif kind == "uniform":
        ps = sitegen.uniform(1000, 1 << 16, seed=4)
    else:
        reg = sitegen.convex_polygon(7, 1 << 12, seed=5)
        ps = sitegen.in_polygon(400, reg, seed=6)
    x, y, moved = lloyd.iterate(ps.x, ps.y, ps.box, 4, region=ps.region)
    assert cdiagram.validate(x, y, ps.box, region=ps.region) == 0
    assert moved[0] > 0


def test_collision_set_exercises_the_rule():
    """The dense 18-site set has two cells whose centroids round to one point."""
    ps = sitegen.small_integer_set(18, 11, seed=30)
    qx, qy = lloyd.proposals(ps.x, ps.y, ps.box)
    _, _, rounds = lloyd.resolve(ps.x, ps.y, qx, qy)
    assert rounds > 0
