"""Parity of the adaptive bucketing (refined crowded buckets, coordinate-rectangle scans) with
the oracle, through the C ABI.

Configurations: the default grid-first path on clustered data (cells that meet a crowded
bucket move to the adaptive pass); every cell through the coordinate-rectangle pass; a coarse
grid (64 sites per bucket) so that even small sets are refined; the one-wave-per-cell pass over
refined buckets (small sets); exact-only precision over refined buckets.
"""
import os

import numpy as np
import pytest

import sitegen
from tests.gpu_util import assert_matches_oracle, say, symmetric

pytestmark = pytest.mark.gpu

# name -> (precision, sites_per_bucket, scan_path, leaf_halfwidth, coop_below)
CONFIGS = {
    "tree_all": ("filtered", 1.0, 1, 0, 0),
    "tree_all_h1": ("filtered", 1.0, 1, 1, 0),
    "coarse_grid_first": ("filtered", 64.0, 0, 0, 0),
    "coarse_coop": ("filtered", 64.0, 0, 0, 1 << 30),
    "coarse_exact": ("exact", 64.0, 0, 0, 0),
    "coarse_exact_h2": ("exact", 64.0, 0, 2, 0),
}


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


@pytest.fixture(scope="module", params=list(CONFIGS))
def actx(request, vor):
    prec, rho, path, ht, coop = CONFIGS[request.param]
    old = os.environ.get("VOR_COOP_BELOW")
    os.environ["VOR_COOP_BELOW"] = str(coop)
    try:
        c = vor.Context(device=0, precision=vor.VOR_FP32_FILTERED if prec == "filtered"
                        else vor.VOR_EXACT_ONLY)
    finally:
        if old is None:
            del os.environ["VOR_COOP_BELOW"]
        else:
            os.environ["VOR_COOP_BELOW"] = old
    c.tune(rho, 256, 0, ht, path)
    c.name = request.param
    yield c
    c.close()


def run(ctx, ps, name):
    say(f"[{ctx.name}] {name}: n={ps.n} box={ps.box}")
    return ctx.compute(ps.x, ps.y, ps.box)


@pytest.mark.parametrize("seed", range(24))
def test_small_tie_heavy(actx, seed):
    n = 1 + (seed * 7) % 60
    ps = sitegen.small_integer_set(n, 9 + seed % 5, seed=7000 + seed)
    assert_matches_oracle(run(actx, ps, f"small seed={seed}"), ps)


def test_twelve_cocircular_and_row(actx):
    offs = [(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3), (-5, 0),
            (-4, 3), (-3, 4), (0, 5)]
    x = np.array([50 + a for a, _ in offs] + [10 + 3 * i for i in range(20)], np.int32)
    y = np.array([50 + b for _, b in offs] + [90] * 20, np.int32)
    ps = sitegen.PointSet(x, y, (0, 0, 100, 100))
    assert_matches_oracle(run(actx, ps, "cocircular + row"), ps)


@pytest.mark.parametrize("dist,n", [("clustered", 20000), ("lattice", 4000),
                                    ("uniform", 6000)])
def test_moderate(actx, dist, n):
    ps = getattr(sitegen, dist)(n, 1 << 24, seed=3)
    r = run(actx, ps, f"{dist} n={n}")
    assert_matches_oracle(r, ps)
    assert symmetric(r)


def test_dense_cluster_small_box(actx):
    # a few thousand sites within a few hundred units: many buckets refined to unit sides
    rng = np.random.default_rng(11)
    pts = set()
    while len(pts) < 3000:
        v = np.rint(rng.normal(400, 60, size=2)).astype(int)
        if 0 < v[0] < 1 << 20 and 0 < v[1] < 1 << 20:
            pts.add((int(v[0]), int(v[1])))
    pts = sorted(pts)
    ps = sitegen.PointSet(np.array([p[0] for p in pts], np.int32),
                          np.array([p[1] for p in pts], np.int32), (0, 0, 1 << 20, 1 << 20))
    assert_matches_oracle(run(actx, ps, "dense cluster"), ps)


def test_duplicates_inside_refined_bucket(actx, vor):
    ps = sitegen.clustered(5000, 1 << 24, seed=9)
    x = np.concatenate([ps.x, ps.x[1234:1235]])
    y = np.concatenate([ps.y, ps.y[1234:1235]])
    say(f"[{actx.name}] duplicate in a cluster")
    with pytest.raises(vor.VorError) as e:
        actx.compute(x, y, ps.box)
    assert e.value.status == vor.VOR_E_DUPLICATE


def test_repeat_identical(actx):
    ps = sitegen.clustered(8000, 1 << 24, seed=21)
    a = run(actx, ps, "repeat 1")
    b = run(actx, ps, "repeat 2")
    assert np.array_equal(a.nbr, b.nbr) and np.array_equal(a.dele, b.dele)
    assert_matches_oracle(b, ps)


def test_grid_first_hands_clustered_cells_on(vor):
    """With the default path, clustered cells reach the adaptive pass (stats), results exact."""
    with vor.Context(device=0) as c:
        ps = sitegen.clustered(30000, 1 << 24, seed=3)
        say(f"[default] clustered n={ps.n}: adaptive pass")
        r = c.compute(ps.x, ps.y, ps.box)
        assert r.stats.adaptive_cells > 0
        assert_matches_oracle(r, ps)
        ps = sitegen.uniform(30000, 1 << 24, seed=2)
        say(f"[default] uniform n={ps.n}: no adaptive pass")
        r = c.compute(ps.x, ps.y, ps.box)
        assert r.stats.adaptive_cells < ps.n // 100
        assert_matches_oracle(r, ps, vertices=False)


@pytest.mark.parametrize("dist", ["clustered", "uniform"])
def test_two_run_adaptive_pass_full_parity(vor, dist):
    """More than 65536 cells through the adaptive pass (every cell, 2 sites per bucket): the
    list-only run and the full run both take part; every cell equals the oracle's."""
    n = 90000
    ps = (sitegen.clustered(n, 1 << 24, seed=13) if dist == "clustered"
          else sitegen.uniform(n, 1 << 22, seed=14))
    with vor.Context(device=0) as c:
        c.tune(2.0, 256, 0, 0, vor.VOR_PATH_TREE)
        say(f"[tree, two runs] {dist} n={n}")
        r = c.compute(ps.x, ps.y, ps.box)
        assert r.stats.adaptive_cells == n
        assert_matches_oracle(r, ps)
        assert symmetric(r)
