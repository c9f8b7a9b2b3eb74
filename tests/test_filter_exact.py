"""Pins of the exact key checker (oracle/filter_exact.c) that the FP32-filter soundness test
relies on (CPU only).

Keys built here from Python fractions, rounded outward to FP32 exactly, must pass; the same
keys moved by one FP32 step across the exact value must fail, each under its own counter.  The
instance generator is pinned to its stated domain and to the exact ties of its cocircular and
vertex-direction families.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import filter_exact as fe

INF = np.float32(np.inf)


def words_to_int(w):
    hi, lo = int(w[0]), int(w[1]) & ((1 << 64) - 1)
    return (hi << 64) + lo


def instances(family, n=1500, seed=5):
    kind, nx, ny, c, d = fe.generate(family, seed, 0, n)
    rows = []
    for i in range(n):
        dx, dy = words_to_int(d[i, :2]), words_to_int(d[i, 2:])
        a, b = int(nx[i]), int(ny[i])
        cc = a * a + b * b if kind[i] == 0 else int(c[i])
        rows.append((a, b, cc, dx, dy))
    return (kind, nx, ny, c, d), rows


def sigma_of(dx, dy):
    return max(abs(dx), abs(dy)).bit_length() - 1


def down(K):
    f = np.float32(float(K))
    while Fraction(float(f)) > K:
        f = np.nextafter(f, np.float32(-np.inf))
    return f


def up(K):
    if K > Fraction(float(np.finfo(np.float32).max)):
        return INF
    f = np.float32(float(K))
    while Fraction(float(f)) < K:
        f = np.nextafter(f, INF)
    return f


def exact_keys(rows):
    """Outward-rounded keys in the checker's layout, plus sigma and the exact keys."""
    n = len(rows)
    out = np.zeros((n, 8), np.float32)
    sig = np.zeros(n, np.int32)
    keys = []
    for i, (a, b, cc, dx, dy) in enumerate(rows):
        s = sigma_of(dx, dy)
        sig[i] = s
        den = a * dx + b * dy
        if den <= 0:
            out[i, :5] = [1.0, INF, 1.0, INF, INF]
            keys.append(None)
            continue
        K = Fraction(cc << s, den)
        lo, hi = down(K), up(K)
        out[i, :5] = [lo, hi, lo, hi, hi]
        keys.append(K)
    return out, sig, keys


def run(arrs, out, sig):
    counts = np.zeros(len(fe.COUNTS), np.int64)
    counts[-1] = -1
    bad, counts = fe.check(*arrs, out, sig, counts)
    return bad, dict(zip(fe.COUNTS, counts.tolist()))


@pytest.mark.parametrize("family", range(5))
def test_exact_outward_keys_pass(family):
    arrs, rows = instances(family)
    out, sig, keys = exact_keys(rows)
    bad, cnt = run(arrs, out, sig)
    assert bad == 0, cnt
    assert cnt["total"] == len(rows)
    assert cnt["positive"] == sum(k is not None for k in keys)


@pytest.mark.parametrize("family", range(5))
def test_keys_one_step_past_the_exact_value_fail(family):
    arrs, rows = instances(family)
    out, sig, keys = exact_keys(rows)
    pos = [i for i, k in enumerate(keys) if k is not None]
    fmax = np.float32(np.finfo(np.float32).max)
    # certified lower key one step up: above the exact key
    o = out.copy()
    for i in pos:
        o[i, 2] = np.nextafter(o[i, 2], INF)
    bad, cnt = run(arrs, o, sig)
    assert cnt["bad_lo"] == sum(out[i, 2] < fmax for i in pos) and bad == cnt["bad_lo"], cnt
    # certified upper key one step down
    o = out.copy()
    fin = [i for i in pos if np.isfinite(out[i, 3])]
    for i in fin:
        o[i, 3] = np.nextafter(o[i, 3], np.float32(0))
    bad, cnt = run(arrs, o, sig)
    assert cnt["bad_hi"] == len(fin) and bad == len(fin), cnt
    # the exact-winner bound one step down
    o = out.copy()
    for i in fin:
        o[i, 4] = np.nextafter(o[i, 4], np.float32(0))
    bad, cnt = run(arrs, o, sig)
    assert cnt["bad_xup"] == len(fin), cnt
    # a lower key of +inf for a key inside FP32's range
    o = out.copy()
    moderate = [i for i in pos if keys[i] <= 2 ** 127]
    for i in moderate:
        o[i, 0] = INF
    bad, cnt = run(arrs, o, sig)
    assert cnt["bad_lo_inf"] == len(moderate), cnt


def test_finite_upper_key_without_a_hit_fails():
    arrs, rows = instances(2)
    out, sig, keys = exact_keys(rows)
    neg = [i for i, k in enumerate(keys) if k is None]
    assert len(neg) > 100
    o = out.copy()
    for i in neg:
        o[i, 1] = o[i, 3] = np.float32(1e30)
    bad, cnt = run(arrs, o, sig)
    assert cnt["bad_sign"] == len(neg) and bad == len(neg), cnt


def test_loose_keys_of_well_conditioned_instances_fail():
    arrs, rows = instances(0)
    out, sig, keys = exact_keys(rows)
    o = out.copy()
    tight = []
    for i, (a, b, cc, dx, dy) in enumerate(rows):
        den = a * dx + b * dy
        if keys[i] is not None and 2 * den >= abs(a * dx) + abs(b * dy):
            tight.append(i)
            o[i, 0] = down(keys[i] * (1 - Fraction(40, 1 << 24)))
            o[i, 2] = o[i, 0]
    bad, cnt = run(arrs, o, sig)
    assert len(tight) > 300
    assert cnt["tight"] == len(tight) and cnt["bad_tight"] == len(tight), cnt


@pytest.mark.parametrize("family", range(5))
def test_generator_domain(family):
    (kind, nx, ny, c, d), rows = instances(family, n=4000, seed=9)
    for k, (a, b, cc, dx, dy) in zip(kind, rows):
        assert (a, b) != (0, 0) and abs(a) <= 1 << 24 and abs(b) <= 1 << 24
        assert 0 < cc <= 1 << 50
        assert (dx, dy) != (0, 0) and abs(dx) < 1 << 78 and abs(dy) < 1 << 78
        assert k == (1 if family == 1 else k)


def test_generator_families_hold_exact_ties():
    """Cocircular family: p = 0 and a site delta on the circle about o through p satisfy
    |delta|^2 = 2 delta.o, so with d = f o the key is the same 2/f for every site of the circle:
    the instances not moved a unit (about half) have 2 delta.d = f |delta|^2 with f a positive
    integer.  Vertex-direction family: a line through the vertex Z/cross of two bisectors has
    N.Z = c |cross|, so N.d is a multiple of c for the instances not moved (about a third)."""
    _, rows = instances(4, n=4000, seed=3)
    on = sum(1 for a, b, cc, dx, dy in rows if (2 * (a * dx + b * dy)) % cc == 0 and
             a * dx + b * dy > 0)
    assert 0.4 * len(rows) < on < 0.6 * len(rows)
    _, rows = instances(3, n=6000, seed=3)
    on = sum(1 for a, b, cc, dx, dy in rows if (a * dx + b * dy) % cc == 0 and
             a * dx + b * dy > 0)
    assert 0.25 * len(rows) < on < 0.45 * len(rows)
