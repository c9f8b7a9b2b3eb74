"""ctypes wrapper of ``libfilterexact.so``: seeded endpoint-key instances and the exact check of
FP32 keys against them (eq. Tdef of Theorem 2.2).  Test infrastructure only."""
import ctypes as C
import os

import numpy as np

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfilterexact.so")
_lib = None
FAMILIES = ("site", "line", "near_perpendicular", "vertex_direction", "cocircular")
COUNTS = ("total", "positive", "lo_finite", "hi_finite", "tight", "bad_sign", "bad_lo_inf",
          "bad_lo", "bad_hi", "bad_xup", "bad_tight", "first_bad")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is not built: run oracle.build.build()")
        L = C.CDLL(_LIB)
        P = C.POINTER
        L.fx_generate.argtypes = [C.c_int, C.c_uint64, C.c_int64, C.c_int64, P(C.c_int32),
                                  P(C.c_int32), P(C.c_int32), P(C.c_int64), P(C.c_int64)]
        L.fx_generate.restype = C.c_int
        L.fx_check.argtypes = [C.c_int64, P(C.c_int32), P(C.c_int32), P(C.c_int32),
                               P(C.c_int64), P(C.c_int64), P(C.c_float), P(C.c_int32),
                               P(C.c_int64)]
        L.fx_check.restype = C.c_int64
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def generate(family: int, seed: int, first: int, n: int):
    """(kind, nx, ny, c, dir[n, 4]) of instances first .. first + n - 1 of a family."""
    kind = np.empty(n, np.int32)
    nx = np.empty(n, np.int32)
    ny = np.empty(n, np.int32)
    c = np.empty(n, np.int64)
    d = np.empty((n, 4), np.int64)
    rc = lib().fx_generate(family, seed, first, n, _p(kind, C.c_int32), _p(nx, C.c_int32),
                           _p(ny, C.c_int32), _p(c, C.c_int64), _p(d, C.c_int64))
    if rc != 0:
        raise ValueError(f"unknown family {family}")
    return kind, nx, ny, c, d


def check(kind, nx, ny, c, d, out, sigma, counts=None):
    """Adds to ``counts`` (int64[12], see COUNTS); returns the number of failing instances."""
    if counts is None:
        counts = np.zeros(len(COUNTS), np.int64)
        counts[-1] = -1
    out = np.ascontiguousarray(out, np.float32)
    sigma = np.ascontiguousarray(sigma, np.int32)
    bad = lib().fx_check(kind.shape[0], _p(kind, C.c_int32), _p(nx, C.c_int32),
                         _p(ny, C.c_int32), _p(c, C.c_int64), _p(d, C.c_int64),
                         _p(out, C.c_float), _p(sigma, C.c_int32), _p(counts, C.c_int64))
    return int(bad), counts
