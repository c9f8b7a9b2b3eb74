"""Sites on the boundary of X, through the C ABI, against the oracle (both precisions).

Such a cell is computed in the box grown by one unit and intersected with X side by side (the
embedding of the paper's remark on a non-polygonal X, Section 10); every other cell is computed
as usual.  Tiny tie-heavy sets with boundary sites, a site at a corner, the four corners, a
lattice that fills the closed box, moderate uniform / clustered / lattice sets with many
boundary sites, polygons with sites on their sides, a batch and a request stream mixing them."""
import time

import numpy as np
import pytest

import sitegen
from tests.gpu_util import assert_matches_oracle, say, symmetric

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


@pytest.fixture(scope="module", params=["filtered", "exact"])
def ctx(request, vor):
    prec = vor.VOR_FP32_FILTERED if request.param == "filtered" else vor.VOR_EXACT_ONLY
    c = vor.Context(device=0, precision=prec)
    c.mode = request.param
    yield c
    c.close()


def run(ctx, ps, name):
    say(f"[{ctx.mode}] {name}: n={ps.n}")
    return ctx.compute(ps.x, ps.y, ps.box, region=ps.region)


@pytest.mark.parametrize("seed", range(30))
def test_tiny_sets_with_boundary_sites(ctx, seed):
    n = 2 + seed % 7
    ps = sitegen.small_integer_set(n, 4 + seed % 5, seed=3000 + seed)
    ps = sitegen.with_boundary_sites(ps, 1 + seed % 4, seed=seed)
    assert_matches_oracle(run(ctx, ps, f"tiny seed={seed}"), ps)


def test_corners(ctx):
    for x, y in [([0], [0]), ([0, 10, 10, 0], [0, 0, 10, 10]), ([0, 10], [5, 5]),
                 ([5, 0, 10, 5], [0, 5, 5, 10])]:
        ps = sitegen.PointSet(np.array(x, np.int32), np.array(y, np.int32), (0, 0, 10, 10))
        assert_matches_oracle(run(ctx, ps, f"corners {x} {y}"), ps)


@pytest.mark.parametrize("k", [2, 7, 40])
def test_lattice_filling_the_closed_box(ctx, k):
    h = 16
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    ps = sitegen.PointSet((h * ii.ravel()).astype(np.int32), (h * jj.ravel()).astype(np.int32),
                          (0, 0, (k - 1) * h, (k - 1) * h))
    r = run(ctx, ps, f"closed lattice {k}x{k}")
    assert_matches_oracle(r, ps)
    assert r.dele.shape[0] == 2 * k * (k - 1)


@pytest.mark.parametrize("kind", ["uniform", "clustered", "lattice"])
def test_moderate_sets_with_many_boundary_sites(ctx, kind):
    if kind == "uniform":
        ps = sitegen.uniform(20000, 1 << 20, seed=31)
    elif kind == "clustered":
        ps = sitegen.clustered(20000, 1 << 20, seed=32)
    else:
        ps = sitegen.lattice(20000, 1 << 24, seed=33)
    ps = sitegen.with_boundary_sites(ps, 600, seed=34)
    r = run(ctx, ps, f"{kind} + boundary")
    assert_matches_oracle(r, ps)
    assert symmetric(r)


def test_sites_on_polygon_sides(ctx):
    for K, n, B, seed in [(16, 5000, 1 << 20, 41), (5, 40, 200, 42), (3, 300, 1 << 16, 43)]:
        reg = sitegen.convex_polygon(K, B, seed=seed)
        ps = sitegen.with_boundary_sites(sitegen.in_polygon(n, reg, seed=seed), 60, seed=seed)
        assert_matches_oracle(run(ctx, ps, f"{len(reg[0])}-gon + boundary"), ps)


def test_batch_and_requests_mixing_boundary_sites(vor):
    reg = sitegen.convex_polygon(9, 1 << 18, seed=51)
    mix = [sitegen.with_boundary_sites(sitegen.uniform(3000, 1 << 20, seed=52), 80, seed=52),
           sitegen.uniform(2000, 1 << 20, seed=53),
           sitegen.with_boundary_sites(sitegen.in_polygon(1500, reg, seed=54), 40, seed=54),
           sitegen.with_boundary_sites(sitegen.small_integer_set(6, 6, seed=55), 3, seed=55)]
    with vor.Context() as c:
        rc, res = c.compute_batch([(p.x, p.y, p.box, p.region) if p.region is not None
                                   else (p.x, p.y, p.box) for p in mix])
        assert rc == vor.VOR_OK
        for r, p in zip(res, mix):
            assert_matches_oracle(r, p)
        tickets = [c.submit(p.x, p.y, p.box, region=p.region) for p in mix]
        out = {}
        t0 = time.time()
        while len(out) < len(tickets):
            for t in tickets:
                if t not in out:
                    st, r = c.poll(t)
                    if st != vor.VOR_PENDING:
                        assert st == vor.VOR_OK, st
                        out[t] = r
            assert time.time() - t0 < 60
            time.sleep(0.002)
        for t, p in zip(tickets, mix):
            assert_matches_oracle(out[t], p)


def test_outside_sites_are_still_errors(vor):
    with vor.Context() as c:
        for x, y in [([-1, 5], [6, 7]), ([101, 5], [6, 7]), ([5, 50], [6, 101])]:
            with pytest.raises(vor.VorError) as e:
                c.compute(np.array(x, np.int32), np.array(y, np.int32), (0, 0, 100, 100))
            assert e.value.status == vor.VOR_E_DOMAIN
