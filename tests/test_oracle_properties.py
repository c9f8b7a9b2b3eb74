"""Property tier for the oracle (CPU only): hypothesis draws small integer point sets, many of
them full of ties (points on a small grid: collinear and cocircular quadruples everywhere,
sites on the boundary of the box), and checks what the mathematics fixes:

* the C oracle equals the brute-force diagram (empty circles over every bisector / side
  intersection point, exact) and the Fraction reference, for up to seven sites;
* the invariants of a Voronoi diagram restricted to X (symmetry, vertices equidistant with no
  site closer and inside X, areas tiling X, Euler's formula, the Delaunay edge count);
* the combinatorics do not change under translation, integer scaling, relabelling of the sites,
  or the reflection that swaps the axes (which reverses each cycle and swaps the box's sides).

The draws are derandomised, so a run is reproducible.
"""
import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

from oracle import brute, cdiagram, checks, ref

SETTINGS = dict(deadline=None, derandomize=True, database=None,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


@st.composite
def point_sets(draw, max_n=10, max_grid=24):
    """(x, y, box): distinct sites on a small grid, in the closed box (which may be larger)."""
    g = draw(st.integers(2, max_grid))
    pts = draw(st.sets(st.tuples(st.integers(0, g), st.integers(0, g)), min_size=1,
                       max_size=max_n))
    pts = sorted(pts)
    x = np.array([p[0] for p in pts], np.int32)
    y = np.array([p[1] for p in pts], np.int32)
    pad = draw(st.tuples(*[st.integers(0, 3)] * 4))
    box = (-pad[0], -pad[1], g + pad[2], g + pad[3])
    return x, y, box


def lines(x, y, box):
    c = cdiagram.cells(x, y, box, threads=1, vertices=False)
    return [c.lines(i) for i in range(c.cells.shape[0])]


def cyclic_equal(a, b):
    """a and b are the same cyclic sequence."""
    if len(a) != len(b):
        return False
    if not a:
        return True
    s = a + a
    return any(s[i:i + len(b)] == b for i in range(len(a)))


@settings(max_examples=300, **SETTINGS)
@given(point_sets(max_n=7, max_grid=8))
def test_oracle_equals_brute_force_and_reference(ps):
    x, y, box = ps
    cl = lines(x, y, box)
    b, _ = brute.diagram(x, y, box)
    assert cl == [ref.rotate_canonical(v) for v in b]
    assert cl == ref.diagram(x, y, box)


@settings(max_examples=300, **SETTINGS)
@given(point_sets(max_n=40, max_grid=24))
def test_invariants_of_the_diagram(ps):
    x, y, box = ps
    checks.check_all(x, y, box, lines(x, y, box))


@settings(max_examples=100, **SETTINGS)
@given(point_sets(max_n=20), st.integers(-1000, 1000), st.integers(-1000, 1000),
       st.integers(2, 7))
def test_translation_and_scaling_change_nothing(ps, dx, dy, s):
    x, y, box = ps
    base = lines(x, y, box)
    moved = lines(x + dx, y + dy, (box[0] + dx, box[1] + dy, box[2] + dx, box[3] + dy))
    assert moved == base
    scaled = lines(x * s, y * s, tuple(v * s for v in box))
    assert scaled == base


@settings(max_examples=100, **SETTINGS)
@given(point_sets(max_n=20), st.randoms(use_true_random=False))
def test_relabelling_the_sites(ps, rnd):
    x, y, box = ps
    n = x.shape[0]
    perm = list(range(n))
    rnd.shuffle(perm)          # site k of the new order is site perm[k] of the old one
    inv = [0] * n
    for k, p in enumerate(perm):
        inv[p] = k
    base = lines(x, y, box)
    new = lines(x[perm], y[perm], box)
    for k in range(n):
        mapped = [inv[j] if j >= 0 else j for j in base[perm[k]]]
        assert cyclic_equal(new[k], mapped)


# the reflection (x, y) -> (y, x) maps the bottom side (y = y0, code -1) to the left one (x = x0,
# code -4) and the right side (-2) to the top one (-3), and back
SWAP = {-1: -4, -4: -1, -2: -3, -3: -2}


@settings(max_examples=100, **SETTINGS)
@given(point_sets(max_n=20))
def test_reflection_swapping_the_axes(ps):
    x, y, box = ps
    base = lines(x, y, box)
    refl = lines(y, x, (box[1], box[0], box[3], box[2]))
    for k in range(x.shape[0]):
        mapped = [SWAP.get(j, j) for j in reversed(base[k])]   # a reflection reverses the cycle
        assert cyclic_equal(refl[k], mapped)
