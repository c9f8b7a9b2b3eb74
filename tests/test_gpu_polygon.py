"""Parity with the oracle when X is a convex polygon (Remark 11.1: any convex polygon X; side e
named -(e+1), primitive outward normals), through the C ABI.

Small sets (the one-wave-per-cell path) in polygons with 3 to 12 sides and many ties; moderate
uniform and clustered sets (the filtered and adaptive passes) in polygons with up to 200 sides;
a box given as a polygon (identical output to the box); one site (its cell is X); batches and
requests mixing boxes and polygons; the edge bound (|X_e| + 6) n; input errors.
"""
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
    say(f"[{ctx.mode}] {name}: n={ps.n} sides={len(ps.region[0])}")
    return ctx.compute(ps.x, ps.y, ps.box, region=ps.region)


def tiny_polygon_set(seed):
    K = 3 + seed % 10
    n = 2 + seed % 7
    for t in range(10):
        reg = sitegen.convex_polygon(K, 40 + 8 * (seed % 4), seed=300 + seed + 1000 * t)
        try:
            return sitegen.in_polygon(n, reg, seed=400 + seed)
        except ValueError:
            continue
    raise AssertionError("no polygon")


@pytest.mark.parametrize("seed", range(24))
def test_tiny_sets_in_polygons(ctx, seed):
    ps = tiny_polygon_set(seed)
    assert_matches_oracle(run(ctx, ps, f"tiny seed={seed}"), ps)


@pytest.mark.parametrize("kind,K,n,B", [("uniform", 16, 20000, 1 << 20),
                                        ("clustered", 6, 20000, 1 << 24),
                                        ("uniform", 3, 6000, 1 << 16),
                                        ("uniform", 200, 8000, 1 << 22)])
def test_moderate_sets_in_polygons(ctx, kind, K, n, B):
    reg = sitegen.convex_polygon(K, B, seed=K + 5)
    ps = sitegen.in_polygon(n, reg, seed=n + K, kind=kind)
    r = run(ctx, ps, f"{kind} K={K}")
    assert_matches_oracle(r, ps)
    assert symmetric(r)
    Kr = len(ps.region[0])
    assert int(r.cell_off[-1]) <= (Kr + 6) * ps.n


def test_single_site_is_the_polygon(ctx):
    reg = sitegen.convex_polygon(12, 1 << 18, seed=12)
    ps = sitegen.in_polygon(1, reg, seed=3)
    r = run(ctx, ps, "single site")
    K = len(ps.region[0])
    want = [-(e + 1) for e in range(K)]
    i = want.index(-K)
    assert r.lines(0) == want[i:] + want[:i]
    assert_matches_oracle(r, ps)


def test_box_as_polygon_is_the_box(ctx):
    ps = sitegen.uniform(20000, 1 << 20, seed=13)
    x0, y0, x1, y1 = ps.box
    reg = (np.array([x0, x1, x1, x0], np.int32), np.array([y0, y0, y1, y1], np.int32))
    say(f"[{ctx.mode}] box as a polygon: n={ps.n}")
    a = ctx.compute(ps.x, ps.y, ps.box)
    b = ctx.compute(ps.x, ps.y, ps.box, region=reg)
    assert np.array_equal(a.cell_off, b.cell_off) and np.array_equal(a.nbr, b.nbr)
    assert a.vertices_int() == b.vertices_int()
    assert np.array_equal(a.dele, b.dele)
    assert_matches_oracle(b, ps)


def test_batch_and_requests_mixing_boxes_and_polygons(vor):
    sets = []
    for i in range(12):
        if i % 3 == 0:
            ps = sitegen.uniform(500 + 700 * i, 1 << 20, seed=40 + i)
        else:
            reg = sitegen.convex_polygon(3 + 5 * i, 1 << 20, seed=60 + i)
            ps = sitegen.in_polygon(500 + 700 * i, reg, seed=80 + i,
                                    kind="clustered" if i % 2 else "uniform")
        sets.append(ps)
    with vor.Context(device=0) as c:
        say(f"batch of {len(sets)} sets, boxes and polygons")
        rc, res = c.compute_batch([(p.x, p.y, p.box) if p.region is None else
                                   (p.x, p.y, p.box, p.region) for p in sets])
        assert rc == vor.VOR_OK
        for ps, r in zip(sets, res):
            assert_matches_oracle(r, ps)
        say("requests, boxes and polygons")
        tickets = [c.submit(p.x, p.y, p.box, p.region) for p in sets]
        import time
        for ps, t in zip(sets, tickets):
            deadline = time.time() + 60
            while True:
                st, r = c.poll(t)
                if st != vor.VOR_PENDING:
                    break
                assert time.time() < deadline
                time.sleep(0.001)
            assert st == vor.VOR_OK
            assert_matches_oracle(r, ps)


def test_polygon_errors(vor):
    x = np.array([10, 20], np.int32)
    y = np.array([10, 20], np.int32)
    with vor.Context(device=0) as c:
        say("polygon errors")
        for vx, vy, code in [([0, 0, 100], [0, 100, 0], vor.VOR_E_INVAL),          # clockwise
                             ([0, 50, 100, 0], [0, 0, 0, 100], vor.VOR_E_INVAL),   # collinear
                             ([0, 100, 30, 0], [0, 0, 30, 100], vor.VOR_E_INVAL),  # not convex
                             ([0, 60, -40, 40, -60], [100, -80, 30, 30, -80],
                              vor.VOR_E_INVAL),                                     # pentagram
                             ([0, 100, 0], [0, 0, 20], vor.VOR_E_DOMAIN)]:          # site outside
            with pytest.raises(vor.VorError) as e:
                c.compute(x, y, (0, 0, 100, 100),
                          region=(np.array(vx, np.int32), np.array(vy, np.int32)))
            assert e.value.status == code, (vx, vy)
        ang = np.linspace(0, 2 * np.pi, 300, endpoint=False)
        big = (np.rint(1e6 + 9e5 * np.cos(ang)).astype(np.int32),
               np.rint(1e6 + 9e5 * np.sin(ang)).astype(np.int32))
        with pytest.raises(vor.VorError) as e:   # more than VOR_MAX_SIDES vertices
            c.compute(np.array([1000000], np.int32), np.array([1000000], np.int32),
                      (0, 0, 1, 1), region=big)
        assert e.value.status == vor.VOR_E_INVAL


def round_polygon(K, R=1 << 22, c=1 << 23):
    """A strictly convex K-gon with integer vertices on (about) a circle, counter-clockwise."""
    import math
    vx = np.array([c + round(R * math.cos(2 * math.pi * k / K)) for k in range(K)], np.int32)
    vy = np.array([c + round(R * math.sin(2 * math.pi * k / K)) for k in range(K)], np.int32)
    return vx, vy


def sites_in_round_polygon(n, K, seed):
    from oracle import cdiagram
    reg = round_polygon(K)
    ps = sitegen.in_polygon(n, reg, seed=seed)
    assert cdiagram.validate(ps.x, ps.y, ps.box, region=ps.region) == 0
    return ps


def test_many_sides_few_sites(ctx):
    """Entry capacity with many sides: one site in a 256-gon (its cell is X, 256 entries), five
    sites in a 200-gon; more entries than 10 per site (sized by 6n + K)."""
    for n, K in ((1, 256), (5, 200), (2, 256)):
        ps = sites_in_round_polygon(n, K, seed=70 + n)
        r = run(ctx, ps, f"{n} sites, {K} sides")
        assert int(r.cell_off[-1]) > 10 * n
        assert_matches_oracle(r, ps)


def test_many_sides_in_a_mixed_batch_and_stream(vor):
    import time
    polys = [sites_in_round_polygon(5, 200, seed=81), sites_in_round_polygon(1, 256, seed=82)]
    boxes = [sitegen.uniform(3000, 1 << 20, seed=83), sitegen.uniform(40, 1 << 16, seed=84)]
    mix = [boxes[0], polys[0], boxes[1], polys[1]]
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
