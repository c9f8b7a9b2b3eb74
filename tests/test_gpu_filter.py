"""Soundness of the FP32 filter, checked in exact rational arithmetic.

The cell passes decide the endpoint of a ray (eq. Tdef, Theorem 2.2: T = min c / (N.d) over
the lines with N.d > 0) with FP32 keys and take the exact 128/192-bit comparison only when the
keys cannot separate the candidates.  That is correct only if every certified key brackets the
exact value: key_lo (1 - 2^-19) <= c 2^sigma / (N.d) <= key_hi (1 + 2^-19), key_hi finite only
when N.d > 0, and key_lo finite whenever N.d > 0 and the exact key is inside FP32's range (a
box side ahead of the ray always has a key of at most 2^25, so no larger key decides anything).  The keys come from the device functions the
passes use (diagnostic entry vor_filter_keys); the exact values are Python integers/fractions.

Instances: random sites and lines, huge ray directions (up to 2^99, beyond the 2^77 that
vertex directions reach), rays nearly perpendicular to the line normal (N.d tiny against |N||d|), sites at the
2^24 extent, and cocircular lattice configurations whose rays pass exactly through a Voronoi
vertex (exact ties, which must never be certified either way) or one unit away from it.
"""
from fractions import Fraction

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

U = Fraction(1, 1 << 24)
SLACK = 1 - Fraction(701, 100) * U     # the analytic bound of the filter's key error
E24 = 1 << 24
HUGE = Fraction(1 << 127)


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


def F(x):
    return Fraction(float(x))


def run(vor, inst):
    kind = [k for k, _, _, _, _, _ in inst]
    nx = [a for _, a, _, _, _, _ in inst]
    ny = [b for _, _, b, _, _, _ in inst]
    c = [cc for _, _, _, cc, _, _ in inst]
    dx = [x for _, _, _, _, x, _ in inst]
    dy = [y for _, _, _, _, _, y in inst]
    return vor.vor_filter_keys(kind, nx, ny, c, dx, dy)


def exact_key(inst, sigma):
    """(N.d, c 2^sigma / (N.d) or None)."""
    k, a, b, c, dx, dy = inst
    cc = a * a + b * b if k == 0 else c
    den = a * dx + b * dy
    return den, (Fraction(cc << sigma, den) if den > 0 else None)


def check_sound(inst, out, sigma, tight=None):
    """Every bracket property the passes rely on, for every instance."""
    inf = float("inf")
    for i, t in enumerate(inst):
        klo, khi, klo_c, khi_c, xup, fx, fy, _ = (float(v) for v in out[i])
        s = int(sigma[i])
        dx, dy = t[4], t[5]
        # d_s = d 2^-sigma rounded componentwise, max component in [1, 2)
        assert s >= 0 and 1 <= max(abs(fx), abs(fy)) <= 2, (i, t)
        for f, e in ((fx, dx), (fy, dy)):   # via double: one extra rounding of 2^-53
            ex = Fraction(e, 1 << s)
            assert abs(Fraction(f) - ex) <= (U + Fraction(1, 1 << 52)) * abs(ex), (i, t)
        den, key = exact_key(t, s)
        if key is None:
            assert khi == inf and khi_c == inf, ("key_hi finite with N.d <= 0", i, t)
            assert xup == inf, (i, t)
            continue
        if klo == inf:
            # only an FP32 overflow may give +inf: the exact key is then beyond 2^127, far
            # above the key of the box side ahead of the ray (at most 2^25), so it never wins
            assert key > HUGE, ("key_lo infinite for a finite key", i, t)
        else:
            assert F(klo_c) <= key, ("certified lower key above the exact key", i, t)
            assert F(klo) * SLACK <= key, ("lower key outside its analytic bound", i, t)
        if khi < inf:
            assert F(khi_c) >= key, ("certified upper key below the exact key", i, t)
            assert F(khi) >= key * SLACK, ("upper key outside its analytic bound", i, t)
        if xup < inf:
            assert F(xup) >= key, ("exact-winner bound below the exact key", i, t)
        else:
            assert key > HUGE, ("exact-winner bound infinite for a moderate key", i, t)
        if tight is not None and tight[i]:
            # a well-conditioned instance (|N.d| >= S / 2): the keys are within 32u of the
            # exact value, so a filter that is sound only by being vacuous fails here
            assert abs(F(klo) - key) <= 32 * U * key and khi < inf, (i, t)
            assert abs(F(khi) - key) <= 32 * U * key, (i, t)


def rand_dir(rng, bits):
    while True:
        x = int(rng.integers(-(1 << 62), 1 << 62)) >> (62 - min(bits, 62))
        y = int(rng.integers(-(1 << 62), 1 << 62)) >> (62 - min(bits, 62))
        if bits > 62:
            x = (x << (bits - 62)) + int(rng.integers(0, 1 << 40))
            y = (y << (bits - 62)) - int(rng.integers(0, 1 << 40))
        if x or y:
            return x, y


def test_random_sites_and_lines(vor):
    rng = np.random.default_rng(1212)
    inst, tight = [], []
    for i in range(6000):
        bits = int(rng.choice([3, 12, 25, 40, 60, 77, 90, 99]))
        dx, dy = rand_dir(rng, bits)
        if i % 3 == 2:   # general line (box sides are such lines)
            a, b = (int(v) for v in rng.integers(-E24, E24, 2))
            if i % 9 == 2:
                a, b = [(0, 1), (1, 0), (0, -1), (-1, 0)][i % 4]
            c = int(rng.integers(1, 1 << 50))
            inst.append((1, a, b, c, dx, dy))
        else:
            sc = int(rng.choice([4, 8, 16, 24]))
            a, b = (int(v) for v in rng.integers(-(1 << sc) + 1, 1 << sc, 2))
            if a == 0 and b == 0:
                a = 1
            inst.append((0, a, b, 0, dx, dy))
        den = a * dx + b * dy
        tight.append(den > 0 and 2 * den >= abs(a * dx) + abs(b * dy))
    say(f"filter keys: {len(inst)} random instances")
    out, sigma = run(vor, inst)
    check_sound(inst, out, sigma, tight)
    assert sum(tight) > 1000


def test_near_perpendicular_rays(vor):
    """d = M N_perp + j N + r: N.d = j |N|^2 + N.r is tiny against |N| |d|, of either sign."""
    rng = np.random.default_rng(77)
    inst = []
    for i in range(4000):
        sc = int(rng.choice([2, 10, 20, 24]))
        a, b = (int(v) for v in rng.integers(-(1 << sc) + 1, 1 << sc, 2))
        if a == 0 and b == 0:
            b = 1
        M = int(rng.integers(1, 1 << 40)) << int(rng.integers(0, 99 - 40 - sc))
        j = int(rng.integers(-1, 2))
        r = [int(v) for v in rng.integers(-3, 4, 2)]
        dx, dy = -b * M + j * a + r[0], a * M + j * b + r[1]
        if abs(dx) >= 1 << 100 or abs(dy) >= 1 << 100 or (dx == 0 and dy == 0):
            continue
        if i % 2:
            inst.append((0, a, b, 0, dx, dy))
        else:
            inst.append((1, a, b, int(rng.integers(1, 1 << 50)), dx, dy))
    say(f"filter keys: {len(inst)} near-perpendicular instances")
    out, sigma = run(vor, inst)
    check_sound(inst, out, sigma)


def circle_points(R):
    """Integer points on the circle x^2 + y^2 = R^2."""
    pts = []
    for x in range(-R, R + 1):
        y2 = R * R - x * x
        y = int(round(y2 ** 0.5))
        for yy in (y - 1, y, y + 1):
            if yy >= 0 and yy * yy == y2:
                pts.append((x, yy))
                if yy:
                    pts.append((x, -yy))
    return sorted(set(pts))


def certified_less(out, i, j):
    """The filter's certification: the upper key of i below the lower key of j."""
    return float(out[i, 3]) < float(out[j, 2])


@pytest.mark.parametrize("R,scale", [(5, 1), (25, 1), (65, 3), (325, 1), (65, 60000),
                                     (25, 300000)])
def test_cocircular_exact_ties_never_certified(vor, R, scale):
    """Sites on one circle through p: the ray from p towards the centre meets every bisector at
    the same point (a Voronoi vertex of all of them), so no candidate may be certified nearer
    than another; a site moved one unit breaks the tie, and a certification must then agree
    with the exact order."""
    pts = [(x * scale, y * scale) for x, y in circle_points(R)]
    assert len(pts) >= 12
    rng = np.random.default_rng(R * 1000 + scale)
    inst, groups = [], []
    for pi in range(min(len(pts), 24)):
        p = pts[int(rng.integers(0, len(pts)))]
        d = (-p[0], -p[1])   # towards the centre; the doubled frame scales t, not the order
        g0 = len(inst)
        for a in pts:
            if a == p:
                continue
            inst.append((0, a[0] - p[0], a[1] - p[1], 0, d[0], d[1]))
        # near-ties: each site one unit off the circle, in turn
        for a in pts[:8]:
            if a == p:
                continue
            for e in ((1, 0), (0, 1), (-1, 0), (0, -1)):
                inst.append((0, a[0] + e[0] - p[0], a[1] + e[1] - p[1], 0, d[0], d[1]))
        groups.append((g0, len(inst)))
    say(f"filter keys: R={R} scale={scale}, {len(inst)} cocircular instances")
    out, sigma = run(vor, inst)
    check_sound(inst, out, sigma)
    ties = certs = 0
    for g0, g1 in groups:
        keys = [exact_key(inst[i], int(sigma[i]))[1] for i in range(g0, g1)]
        for i in range(g0, g1):
            for j in range(g0, g1):
                ki, kj = keys[i - g0], keys[j - g0]
                if i == j or ki is None or kj is None:
                    continue
                if certified_less(out, i, j):
                    certs += 1
                    assert ki < kj, ("certified a wrong order", inst[i], inst[j])
                if ki == kj:
                    ties += 1
                    assert not certified_less(out, i, j), ("certified a tie", inst[i], inst[j])
    assert ties > 0


def test_vertex_directions_of_line_pairs(vor):
    """Rays through the intersection of two lines (the Z directions of the subedge walk): the
    direction is the exact integer vertex numerator, both lines are hit at the same t."""
    rng = np.random.default_rng(5)
    inst, pairs = [], []
    while len(pairs) < 2000:
        sc = int(rng.choice([3, 12, 24]))
        a1, b1, a2, b2 = (int(v) for v in rng.integers(-(1 << sc) + 1, 1 << sc, 4))
        cr = a1 * b2 - b1 * a2
        if cr == 0:
            continue
        c1, c2 = a1 * a1 + b1 * b1, a2 * a2 + b2 * b2
        if c1 == 0 or c2 == 0:
            continue
        dx, dy = c1 * b2 - c2 * b1, a1 * c2 - a2 * c1
        if cr < 0:
            dx, dy = -dx, -dy
        if dx == 0 and dy == 0:
            continue
        i = len(inst)
        inst.append((0, a1, b1, 0, dx, dy))
        inst.append((0, a2, b2, 0, dx, dy))
        pairs.append(i)
    say(f"filter keys: {len(inst)} vertex-direction instances")
    out, sigma = run(vor, inst)
    check_sound(inst, out, sigma)
    for i in pairs:
        k1 = exact_key(inst[i], int(sigma[i]))[1]
        k2 = exact_key(inst[i + 1], int(sigma[i + 1]))[1]
        assert k1 == k2
        assert not certified_less(out, i, i + 1) and not certified_less(out, i + 1, i)


def test_argument_errors(vor):
    with pytest.raises(vor.VorError) as e:
        vor.vor_filter_keys([2], [1], [1], [1], [1], [1])
    assert e.value.status == vor.VOR_E_INVAL
    with pytest.raises(vor.VorError):
        vor.vor_filter_keys([1], [1], [1], [0], [1], [1])      # c must be positive
    with pytest.raises(vor.VorError):
        vor.vor_filter_keys([0], [1], [1], [0], [0], [0])      # zero direction
    with pytest.raises(vor.VorError):
        vor.vor_filter_keys([0], [1], [1], [0], [1 << 100], [1])
    out, sigma = vor.vor_filter_keys([], [], [], [], [], [])
    assert out.shape == (0, 8)


@pytest.mark.parametrize("family", range(5))
def test_bulk_exact_check(vor, family):
    """2*10^7 seeded instances per family (10^8 in all): random sites, random lines and box
    sides, near-perpendicular rays, vertex directions of two bisectors against either line or a
    site one unit away, cocircular lattice sites against the ray towards the centre.  The keys
    come from the device; oracle/filter_exact.c decides every bracket in exact integers."""
    from oracle import filter_exact as fe
    chunk, chunks = 5_000_000, 4
    counts = np.zeros(len(fe.COUNTS), np.int64)
    counts[-1] = -1
    for k in range(chunks):
        say(f"bulk filter check: family {fe.FAMILIES[family]}, chunk {k + 1}/{chunks}")
        kind, nx, ny, c, d = fe.generate(family, 1212, k * chunk, chunk)
        out, sigma = vor.vor_filter_keys_words(kind, nx, ny, c, d)
        first = int(counts[-1])
        bad, counts = fe.check(kind, nx, ny, c, d, out, sigma, counts)
        if bad:
            i = int(counts[-1]) if first < 0 else 0
            raise AssertionError(f"{bad} unsound instances, first: kind={kind[i]} N=({nx[i]}, "
                                 f"{ny[i]}) c={c[i]} dir={d[i].tolist()} keys={out[i].tolist()} "
                                 f"sigma={sigma[i]}; counts {dict(zip(fe.COUNTS, counts))}")
    say(f"  {dict(zip(fe.COUNTS, counts.tolist()))}")
    assert counts[0] == chunk * chunks
    assert counts[1] > chunk * chunks // 3           # a third at least hit the line
    assert counts[4] > chunk * chunks // 50          # and some are well conditioned
