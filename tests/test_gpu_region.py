"""The certified candidate regions of the scans, checked in exact rational arithmetic.

A ray's scan stops growing once its region holds every site that is not farther from
y = p + (T/2) d_s than p (Method 11.6; by the lemma on sites in the large square all such sites
lie in the square S[y, |y - p|], and by the nesting lemma the squares of the points of [p, y]
lie inside it).  T is an upper bound of the endpoint parameter that the FP32 filter certifies
only up to a factor 1 + 7.01u (u = 2^-24), so the exact point tested here is taken with
T (1 + 2^-21).  The diagnostic entry vor_region_diag runs the device functions of the scans
(bucket rectangle, coordinate rectangle, pruning disk) on given instances; for every instance
this test enumerates the integer points on the boundary of the exact closed disk B(y, |y - p|)
inside X (the extreme points of every row and column it tests) and requires each of them to be
inside the bucket rectangle, inside the coordinate rectangle, and admitted by the disk test.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

SLACK = 1 + F(1, 1 << 21)


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


def le_q_plus_sqrt(a, q, R):
    """a <= q + sqrt(R), exactly (R >= 0)."""
    t = a - q
    return t <= 0 or t * t <= R


def floor_q_plus_sqrt(q, R):
    approx = q + F(math.isqrt(int(R * (1 << 96))), 1 << 48)
    k = math.floor(approx)
    while not le_q_plus_sqrt(k, q, R):
        k -= 1
    while le_q_plus_sqrt(k + 1, q, R):
        k += 1
    return k


def ceil_q_minus_sqrt(q, R):
    return -floor_q_plus_sqrt(-q, R)


def boundary_points(y, R, W, H, rng, extra=6):
    """Integer points of the closed disk B(y, sqrt(R)) inside [0, W] x [0, H] at the ends of
    selected columns and rows (the extreme columns and rows among them)."""
    pts = set()
    xlo, xhi = max(0, ceil_q_minus_sqrt(y[0], R)), min(W, floor_q_plus_sqrt(y[0], R))
    ylo, yhi = max(0, ceil_q_minus_sqrt(y[1], R)), min(H, floor_q_plus_sqrt(y[1], R))
    for axis, lo, hi in ((0, xlo, xhi), (1, ylo, yhi)):
        if lo > hi:
            continue
        c = y[axis]
        cols = {lo, hi, min(hi, lo + 1), max(lo, hi - 1)}
        for v in (math.floor(c), math.ceil(c)):
            if lo <= v <= hi:
                cols.add(v)
        for _ in range(extra):
            cols.add(int(rng.integers(lo, hi + 1)))
        o = y[1 - axis]
        ext = H if axis == 0 else W
        for v in cols:
            h2 = R - (v - c) ** 2
            if h2 < 0:
                continue
            a, b = max(0, ceil_q_minus_sqrt(o, h2)), min(ext, floor_q_plus_sqrt(o, h2))
            for w in {a, b}:
                if a <= w <= b:
                    pts.add((v, w) if axis == 0 else (w, v))
    return sorted(pts)


def make_instances(rng, count):
    geom, dxs, dys, Ts = [], [], [], []
    for i in range(count):
        W = int(rng.choice([1 << 16, 1 << 20, 1 << 24, int(rng.integers(1000, 1 << 24))]))
        H = W if rng.random() < 0.6 else int(rng.integers(1000, 1 << 24))
        n = int(np.exp(rng.uniform(np.log(32), np.log(1 << 22))))
        s = max(1, math.ceil(math.sqrt(W * H * float(rng.uniform(0.5, 4.0)) / n)))
        gx, gy = -(-W // s), -(-H // s)
        px, py = int(rng.integers(1, W)), int(rng.integers(1, H))
        if rng.random() < 0.25:   # on or next to a bucket edge
            px = min(W - 1, max(1, s * int(rng.integers(0, gx)) + int(rng.integers(-1, 2))))
            py = min(H - 1, max(1, s * int(rng.integers(0, gy)) + int(rng.integers(-1, 2))))
        kind = i % 3
        while True:
            if kind == 0:
                dx, dy = [(7, -4), (0, 1), (-7, -4), (1, 0), (-1, 1)][int(rng.integers(0, 5))]
                if rng.random() < 0.5:
                    dx, dy = int(rng.integers(-9, 10)), int(rng.integers(-9, 10))
            elif kind == 1:
                dx, dy = int(rng.integers(-(1 << 24), 1 << 24)), int(rng.integers(-(1 << 24), 1 << 24))
            else:   # vertex directions of the walk reach 2^77
                b = int(rng.integers(30, 78))
                dx = int(rng.integers(-(1 << 62), 1 << 62)) << max(0, b - 62)
                dy = int(rng.integers(-(1 << 62), 1 << 62)) << max(0, b - 62)
            if dx or dy:
                break
        sig = max(abs(dx), abs(dy)).bit_length() - 1
        norm = math.hypot(dx / 2.0 ** sig, dy / 2.0 ** sig)
        rho = math.exp(rng.uniform(math.log(0.5), math.log(float(1 << 25))))
        T = np.float32(2.0 * rho / norm)
        if i % 50 == 7:
            T = np.float32(np.inf)
        geom.append((px, py, W, H, s, gx, gy))
        dxs.append(dx)
        dys.append(dy)
        Ts.append(T)
    return np.array(geom, np.int32), dxs, dys, np.array(Ts, np.float32)


def test_regions_cover_the_exact_disk(vor):
    rng = np.random.default_rng(2026)
    count = 2400
    geom, dxs, dys, Ts = make_instances(rng, count)
    first = vor.vor_region_diag(geom, dxs, dys, Ts, np.zeros((count, 2), np.int32))
    pts_inst, pts = [], []
    exact = []
    for i in range(count):
        px, py, W, H, s, gx, gy = (int(v) for v in geom[i])
        T = float(Ts[i])
        br, cr = first["bucket_rect"][i], first["coord_rect"][i]
        if math.isinf(T):
            assert list(br) == [0, gx - 1, 0, gy - 1] and list(cr) == [0, W, 0, H], i
            exact.append(None)
            continue
        sig = int(first["sigma"][i])
        e = (F(dxs[i], 1) / F(2) ** sig, F(dys[i], 1) / F(2) ** sig)
        h = F(T) * SLACK / 2
        y = (px + h * e[0], py + h * e[1])
        R = h * h * (e[0] ** 2 + e[1] ** 2)
        P = boundary_points(y, R, W, H, rng)
        exact.append(len(P))
        for (zx, zy) in P:
            assert (zx - y[0]) ** 2 + (zy - y[1]) ** 2 <= R
            bx, by = min(zx // s, gx - 1), min(zy // s, gy - 1)
            assert br[0] <= bx <= br[1] and br[2] <= by <= br[3], \
                f"instance {i}: bucket ({bx},{by}) of {(zx, zy)} outside {list(br)}"
            assert cr[0] <= zx <= cr[1] and cr[2] <= zy <= cr[3], \
                f"instance {i}: {(zx, zy)} outside {list(cr)}"
            pts_inst.append(i)
            pts.append((zx, zy))
    say(f"{count} instances, {len(pts)} boundary points of the exact disks")
    assert len(pts) > 5 * count
    idx = np.array(pts_inst)
    second = vor.vor_region_diag(geom[idx], [dxs[i] for i in idx], [dys[i] for i in idx],
                                 Ts[idx], np.array(pts, np.int32))
    bad = np.nonzero(second["inside"] == 0)[0]
    assert bad.size == 0, f"disk test rejects {bad.size} points, first instance {idx[bad[0]]}"


def test_regions_are_not_the_whole_grid(vor):
    """Soundness alone would hold for the whole grid: a near bound gives a small region."""
    geom = np.array([[5000, 5000, 1 << 16, 1 << 16, 64, 1024, 1024]] * 3, np.int32)
    T = np.array([np.float32(200.0)] * 3, np.float32)
    out = vor.vor_region_diag(geom, [7, 0, -7], [-4, 1, -4], T, np.zeros((3, 2), np.int32))
    for i, (dx, dy) in enumerate([(7, -4), (0, 1), (-7, -4)]):
        br, cr = out["bucket_rect"][i], out["coord_rect"][i]
        r = 100.0 * math.hypot(dx, dy) / 2.0 ** int(out["sigma"][i])
        wide = 2 * (r * 1.001 + 3)        # the square S[y, r] plus the margin, in coordinates
        assert cr[1] - cr[0] <= wide and cr[3] - cr[2] <= wide
        assert br[1] - br[0] <= wide / 64 + 1 and br[3] - br[2] <= wide / 64 + 1


def test_region_diag_rejects_bad_arguments(vor):
    g = np.array([[10, 10, 100, 100, 10, 10, 10]], np.int32)
    z = np.zeros((1, 2), np.int32)
    with pytest.raises(vor.VorError):
        vor.vor_region_diag(g, [0], [0], np.array([1.0], np.float32), z)      # d = 0
    g2 = g.copy()
    g2[0, 5] = 5                                                               # grid too small
    with pytest.raises(vor.VorError):
        vor.vor_region_diag(g2, [1], [0], np.array([1.0], np.float32), z)
    with pytest.raises(vor.VorError):
        vor.vor_region_diag(g, [1], [0], np.array([np.nan], np.float32), z)
