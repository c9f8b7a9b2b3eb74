"""Pins of the oracle against what the paper and the mathematics fix (CPU only)."""
import json
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest

import sitegen
from oracle import brute, cdiagram, checks, paper_forms, ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def c_cells(ps, which=None):
    c = cdiagram.cells(ps.x, ps.y, ps.box, which=which, threads=4)
    return [c.lines(i) for i in range(c.cells.shape[0])], c


# ---------------------------------------------------------------- brute force, n <= 8
@pytest.mark.parametrize("seed", range(60))
def test_brute_force_matches_oracle_tiny_ties(seed):
    """Brute force (empty circles + bisector/side points + corners, exact) == C oracle ==
    Fraction reference, on tiny integer sets with many cocircular and collinear ties."""
    n = 2 + seed % 7
    coord = 4 + seed % 5
    ps = sitegen.small_integer_set(n, coord, seed=1000 + seed)
    cl, _ = c_cells(ps)
    b, _ = brute.diagram(ps.x, ps.y, ps.box)
    b = [ref.rotate_canonical(v) for v in b]
    r = ref.diagram(ps.x, ps.y, ps.box)
    assert cl == b
    assert cl == r
    checks.check_all(ps.x, ps.y, ps.box, cl)


@pytest.mark.parametrize("seed", range(10))
def test_brute_force_matches_oracle_general(seed):
    ps = sitegen.small_integer_set(8, 1 << 12, seed=2000 + seed)
    cl, _ = c_cells(ps)
    b, _ = brute.diagram(ps.x, ps.y, ps.box)
    assert cl == [ref.rotate_canonical(v) for v in b]


# ---------------------------------------------------------------- closed forms
def test_single_site_is_the_box():
    x = np.array([3], np.int32); y = np.array([5], np.int32)
    c = cdiagram.cells(x, y, (0, 0, 10, 10))
    # the box, CCW from the bottom side, rotated to start at the smallest uint32 label (-4)
    assert c.lines(0) == [-4, -1, -2, -3]
    X, Y, D = [int(v) for v in c.vx], [int(v) for v in c.vy], [int(v) for v in c.vd]
    pts = [(F(a, d), F(b, d)) for a, b, d in zip(X, Y, D)]
    assert pts == [(0, 0), (10, 0), (10, 10), (0, 10)]


def test_two_sites_split_by_bisector():
    x = np.array([2, 8], np.int32); y = np.array([5, 5], np.int32)
    cl, c = c_cells(sitegen.PointSet(x, y, (0, 0, 10, 10)))
    assert cl[0] == [1, -3, -4, -1]
    assert cl[1] == [0, -1, -2, -3]
    # the shared edge is x = 5
    v = [(F(int(a), int(d)), F(int(b), int(d))) for a, b, d in zip(c.vx, c.vy, c.vd)]
    assert v[0] == (5, 10) and v[3] == (5, 0)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_lattice_cells_are_squares(k):
    """k x k lattice in [0, k h]^2 at (h/2 + i h, h/2 + j h): every cell is an h x h square;
    the Delaunay graph is the 4-neighbour grid (diagonal cells meet at a point only)."""
    h = 10
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    x = (h // 2 + h * ii.ravel()).astype(np.int32)
    y = (h // 2 + h * jj.ravel()).astype(np.int32)
    box = (0, 0, k * h, k * h)
    cl, c = c_cells(sitegen.PointSet(x, y, box))
    for idx in range(k * k):
        i, j = idx % k, idx // k
        expect = {(i, j - 1): -1, (i + 1, j): -2, (i, j + 1): -3, (i - 1, j): -4}
        labels = set()
        for (a, b), side in expect.items():
            labels.add(b * k + a if (0 <= a < k and 0 <= b < k) else side)
        assert set(cl[idx]) == labels
        assert len(cl[idx]) == 4
    dl = cdiagram.delaunay(c)
    assert dl.shape[0] == 2 * k * (k - 1)
    checks.check_all(x, y, box, cl)


def test_collinear_row_gives_vertical_strips():
    """Sites on one horizontal line: the cells are vertical strips between midpoints."""
    xs = [3, 7, 15, 16, 30]
    x = np.array(xs, np.int32); y = np.full(5, 20, np.int32)
    box = (0, 0, 40, 40)
    cl, c = c_cells(sitegen.PointSet(x, y, box))
    assert cl[0] == [1, -3, -4, -1]
    for i in range(1, 4):
        assert sorted(cl[i]) == sorted([i - 1, i + 1, -1, -3])
    assert cl[4] == [3, -1, -2, -3]
    checks.check_all(x, y, box, cl)


def test_twelve_cocircular_points_meet_at_centre():
    """The 12 integer points at distance 5 from a centre: all cells share the centre vertex and
    the Delaunay graph is the 12-cycle."""
    offs = [(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3), (-5, 0),
            (-4, 3), (-3, 4), (0, 5)]
    cx = cy = 50
    x = np.array([cx + a for a, _ in offs], np.int32)
    y = np.array([cy + b for _, b in offs], np.int32)
    box = (0, 0, 100, 100)
    cl, c = c_cells(sitegen.PointSet(x, y, box))
    for k in range(12):
        sites = sorted(j for j in cl[k] if j >= 0)
        assert sites == sorted([(k - 1) % 12, (k + 1) % 12])
    for k in range(12):
        o = c.off[k]
        pts = {(F(int(c.vx[t]), int(c.vd[t])), F(int(c.vy[t]), int(c.vd[t])))
               for t in range(o, o + c.counts[k])}
        assert (cx, cy) in pts
    assert cdiagram.delaunay(c).shape[0] == 12
    checks.check_all(x, y, box, cl)


# ---------------------------------------------------------------- invariants at moderate n
@pytest.mark.parametrize("gen", ["uniform", "clustered", "lattice"])
def test_invariants_moderate(gen):
    if gen == "uniform":
        ps = sitegen.uniform(400, 1 << 16, seed=7)
    elif gen == "clustered":
        ps = sitegen.clustered(400, 1 << 16, seed=8)
    else:
        ps = sitegen.lattice(400, 1 << 24, seed=9)
    cl, c = c_cells(ps)
    checks.check_all(ps.x, ps.y, ps.box, cl, every_site=(gen != "lattice"))
    # pair-form vertices written by the C oracle equal Cramer's rule on the cell's lines
    for k in range(0, ps.n, 37):
        o = c.off[k]
        m = c.counts[k]
        for t in range(m):
            X, Y, D = checks.pair_form(ps.x, ps.y, ps.box, k, cl[k][t], cl[k][(t + 1) % m])
            assert (int(c.vx[o + t]), int(c.vy[o + t]), int(c.vd[o + t])) == (X, Y, D)


def test_reference_matches_oracle_random_150():
    ps = sitegen.uniform(150, 1 << 16, seed=11)
    cl, _ = c_cells(ps)
    assert cl == ref.diagram(ps.x, ps.y, ps.box)


def test_reference_matches_oracle_jittered_lattice():
    ps = sitegen.lattice(100, 1 << 24, seed=12)
    cl, _ = c_cells(ps)
    assert cl == ref.diagram(ps.x, ps.y, ps.box)


def test_subset_cells_equal_full_diagram():
    ps = sitegen.uniform(3000, 1 << 20, seed=13)
    full, _ = c_cells(ps)
    which = np.array([0, 5, 77, 2999, 1500], np.int32)
    sub, _ = c_cells(ps, which)
    assert sub == [full[i] for i in which]


def test_edge_totals_within_paper_bound():
    """Lemma on the node count: sum of e_k <= (|X_e| + 6) n = 10 n for a rectangle."""
    for ps in (sitegen.uniform(2000, 1 << 16, 21), sitegen.clustered(2000, 1 << 20, 22),
               sitegen.lattice(2000, 1 << 24, 23)):
        _, c = c_cells(ps)
        assert int(c.counts.sum()) <= 10 * ps.n


# ---------------------------------------------------------------- checkers catch mistakes
def test_checkers_reject_planted_mistakes():
    ps = sitegen.uniform(60, 1 << 12, seed=31)
    cl, _ = c_cells(ps)
    checks.check_all(ps.x, ps.y, ps.box, cl)
    k = next(i for i, v in enumerate(cl) if len(v) >= 4)
    dropped = [list(v) for v in cl]
    dropped[k] = dropped[k][:-1]                 # a dropped edge
    reversed_ = [list(v) for v in cl]
    reversed_[k] = reversed_[k][::-1]            # wrong orientation
    swapped = [list(v) for v in cl]
    swapped[k][0], swapped[k][1] = swapped[k][1], swapped[k][0]
    for bad in (dropped, reversed_, swapped):
        with pytest.raises(AssertionError):
            checks.check_all(ps.x, ps.y, ps.box, bad)


# ---------------------------------------------------------------- input validation
def test_validate_codes():
    box = (0, 0, 16, 16)
    ok = (np.array([1, 2], np.int32), np.array([1, 2], np.int32))
    assert cdiagram.validate(*ok, box) == 0
    assert cdiagram.validate(np.array([-1, 2], np.int32), np.array([1, 2], np.int32), box) == -2
    assert cdiagram.validate(np.array([17, 2], np.int32), np.array([1, 2], np.int32), box) == -2
    assert cdiagram.validate(np.array([0, 16], np.int32), np.array([1, 2], np.int32), box) == 0
    assert cdiagram.validate(np.array([3, 3], np.int32), np.array([4, 4], np.int32), box) == -3
    assert cdiagram.validate(*ok, (5, 0, 5, 16)) == -1
    assert cdiagram.validate(*ok, (0, 0, (1 << 24) + 1, 16)) == -2


# ---------------------------------------------------------------- paper closed forms
def test_integer_rectangle_worked_example():
    g = json.load(open(os.path.join(GOLD, "integer_rectangle_example.json")))
    r = paper_forms.eta(g["beta"], g["s"])
    assert abs(r - g["eta_approx"]) < 0.01
    si = paper_forms.integer_rectangle(tuple(g["y"]), r, g["s"])
    assert [list(a) for a in si] == g["expected_S_I"]
    X = g["X"]
    cut = [[max(si[0][0], X[0]), min(si[0][1], X[2])], [max(si[1][0], X[1]), min(si[1][1], X[3])]]
    assert cut == g["expected_S_I_cut_to_X"]
    assert 1 + math.floor(8 * math.sqrt(2) * (g["beta"] + 1.01)) == g["expected_buckets_per_side_alpha2_root"]


def test_integer_rectangle_contains_square_and_is_minimal():
    rng = np.random.default_rng(5)
    for _ in range(500):
        s = int(rng.integers(1, 9))
        y = (F(int(rng.integers(-500, 500)), int(rng.integers(1, 7))),
             F(int(rng.integers(-500, 500)), int(rng.integers(1, 7))))
        r = F(int(rng.integers(1, 300)), int(rng.integers(1, 5)))
        (a, b), (c, d) = paper_forms.integer_rectangle(y, r, s)
        assert a <= y[0] - r and y[0] + r < b and c <= y[1] - r and y[1] + r < d
        assert a % s == 0 and b % s == 0 and a + s > y[0] - r and b - s <= y[0] + r


def test_theorem_constants():
    g = json.load(open(os.path.join(GOLD, "theorem_constants.json")))
    for case in g["cases"]:
        n = 10 ** 100 if case["n"] == "1e100" else int(case["n"])
        tc = paper_forms.theorem_constants(n, case["eps"])
        for key in ("alpha1", "beta", "alpha2", "per_site_bound"):
            assert tc[key] == case[key], key
        assert tc["cond1"] and tc["cond2"]
        if "printed_bound" in case:
            assert tc["per_site_bound"] <= case["printed_bound"] == 3 * tc["alpha2"] * 22


def test_sites_closer_to_y_lie_in_the_integer_rectangle():
    """Lemma on sites in the large square (Appendix 1) with eq. (S_I): for a point y on a ray
    from p, every site not farther from y than p lies in the buckets of S_I[y, |y - p|]; and the
    disks of the points y' of [p, y] nest (B[y', |y' - p|] inside B[y, |y - p|], the lemma on
    B(y, y')).  Brute force over every lattice site of a window, in exact integers scaled by the
    common denominator: rays along Pythagorean directions, so that |y - p| is rational."""
    rng = np.random.default_rng(11)
    triples = [(3, 4, 5), (5, 12, 13), (8, 15, 17), (7, 24, 25), (20, 21, 29), (1, 0, 1)]
    checked = 0
    for _ in range(400):
        a, b, c = triples[int(rng.integers(0, len(triples)))]
        if rng.random() < 0.5:
            a, b = b, a
        a, b = a * int(rng.choice([-1, 1])), b * int(rng.choice([-1, 1]))
        p = (int(rng.integers(0, 60)), int(rng.integers(0, 60)))
        s = int(rng.integers(1, 9))
        tn, td = int(rng.integers(1, 400)), int(rng.integers(1, 12))
        t = F(tn, td)
        y = (p[0] + t * F(a, c), p[1] + t * F(b, c))
        (A0, B0), (A1, B1) = paper_forms.integer_rectangle(y, t, s)
        un = int(rng.integers(0, 1000))                 # y' = p + (un / 1000) t theta on [p, y]
        # every lattice point of a window around y, coordinates scaled by L = c td 1000
        L = c * td * 1000
        qx, qy = np.meshgrid(np.arange(math.floor(y[0] - t) - 2, math.ceil(y[0] + t) + 3),
                             np.arange(math.floor(y[1] - t) - 2, math.ceil(y[1] + t) + 3))
        qx, qy = qx.ravel().astype(np.int64), qy.ravel().astype(np.int64)
        Yx, Yy = p[0] * L + tn * a * 1000, p[1] * L + tn * b * 1000       # y * L
        R = tn * c * 1000                                                # |y - p| * L
        Y2x, Y2y = p[0] * L + tn * a * un, p[1] * L + tn * b * un        # y' * L
        R2 = tn * c * un
        near = (qx * L - Yx) ** 2 + (qy * L - Yy) ** 2 <= R * R
        near2 = (qx * L - Y2x) ** 2 + (qy * L - Y2y) ** 2 <= R2 * R2
        assert not np.any(near2 & ~near), "disk of y' not inside the disk of y"
        inr = (qx >= A0) & (qx < B0) & (qy >= A1) & (qy < B1)
        assert np.all(inr[near]), (p, y, t, s)
        checked += int(near.sum())
    assert checked > 100000
