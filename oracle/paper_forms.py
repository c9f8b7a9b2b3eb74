"""Closed forms printed in the paper -- TEST INFRASTRUCTURE ONLY.

* ``integer_rectangle`` -- eq. (S_I) of Appendix 1: the smallest bucket-aligned rectangle that
  contains the square S[y, r] (one more column/row when S[y, r] is itself bucket-aligned).
* ``theorem_constants`` -- the parameters of Theorem 9.1(e) (eqs. alpha1, OneTwo, beta,
  alpha2, m) and the resulting bound on the distance comparisons, (3 alpha2 - 1) 22 n.
* ``eta`` -- the probe distance of the improved endpoint method (Method 11.6, step 1).
"""
from __future__ import annotations

import math


def integer_rectangle(y, r, s):
    """eq. (S_I): [s floor((y1-r)/s), s (floor((y1+r)/s)+1)] x [same for y2]."""
    y1, y2 = y
    return ((s * math.floor((y1 - r) / s), s * (math.floor((y1 + r) / s) + 1)),
            (s * math.floor((y2 - r) / s), s * (math.floor((y2 + r) / s) + 1)))


def eta(beta, s):
    return 4.0 * math.sqrt(2.0) * (beta + 1.01) * s


def theorem_constants(n, eps):
    """Theorem 9.1(e): returns dict with m, alpha1, beta, alpha2, the two side conditions and
    the comparison bound per site (3 alpha2 - 1) * 22."""
    m = math.isqrt(n) ** 2 if isinstance(n, int) else int(math.floor(math.sqrt(n))) ** 2
    lnv = math.log(n) + math.log1p(2.0 * math.exp(-400.0)) - math.log(eps)
    fl = int(math.floor(math.sqrt(lnv)))
    one_two = 1 if fl % 2 == 0 else 2
    alpha1 = (fl + one_two) ** 2
    beta = (math.isqrt(alpha1) - 1) // 2
    alpha2 = (1 + int(math.floor(8.0 * math.sqrt(2.0) * (beta + 1.01)))) ** 2
    cond1 = alpha1 < ((m // 5) + 2) / 3.0          # floor(0.2 m) = m // 5 for integer m
    cond2 = alpha2 < math.exp(-2.0) * ((m // 5) + 1)
    return {"m": m, "alpha1": alpha1, "beta": beta, "alpha2": alpha2, "cond1": cond1,
            "cond2": cond2, "per_site_bound": (3 * alpha2 - 1) * 22,
            "r_k_bound": 3 * alpha2}
