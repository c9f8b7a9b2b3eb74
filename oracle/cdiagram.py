"""ctypes wrapper of the C oracle (exact half-plane clipping).  Test infrastructure only.

Implements the plain definition (Section 2, Definition of the Voronoi diagram): each cell is
X intersected with the n-1 bisector half-planes.  Output conventions follow Section 6 (lines
named by neighbour index, box sides -1..-4, sides of a convex polygon X -1..-K) and Section 7 (Delaunay edges = neighbours via an
edge, restricted to X).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -2: "site outside X / box too large",
          -3: "duplicate sites", -4: "capacity", -5: "out of memory"}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        i32p = C.POINTER(C.c_int32)
        L.vor_oracle_validate.restype = C.c_int
        L.vor_oracle_validate.argtypes = [C.c_int32, i32p, i32p] + [C.c_int32] * 4
        L.vor_oracle_cells.restype = C.c_int64
        L.vor_oracle_cells.argtypes = ([C.c_int32, i32p, i32p] + [C.c_int32] * 4 +
                                       [C.c_int32, i32p, C.c_int32, i32p, C.c_int64, i32p,
                                        C.POINTER(C.c_int64)])
        L.vor_oracle_vertices.restype = C.c_int
        L.vor_oracle_vertices.argtypes = ([C.c_int32, i32p, i32p] + [C.c_int32] * 4 +
                                          [C.c_int32, i32p, i32p, i32p,
                                           C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                           C.POINTER(C.c_int64)])
        L.vor_oracle_validate_poly.restype = C.c_int
        L.vor_oracle_validate_poly.argtypes = [C.c_int32, i32p, i32p, C.c_int32, i32p, i32p]
        L.vor_oracle_cells_poly.restype = C.c_int64
        L.vor_oracle_cells_poly.argtypes = ([C.c_int32, i32p, i32p, C.c_int32, i32p, i32p] +
                                            [C.c_int32, i32p, C.c_int32, i32p, C.c_int64, i32p,
                                             C.POINTER(C.c_int64)])
        L.vor_oracle_vertices_poly.restype = C.c_int
        L.vor_oracle_vertices_poly.argtypes = ([C.c_int32, i32p, i32p, C.c_int32, i32p, i32p] +
                                               [C.c_int32, i32p, i32p, i32p,
                                                C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                                C.POINTER(C.c_int64)])
        L.vor_oracle_default_threads.restype = C.c_int32
        L.vor_oracle_default_threads.argtypes = []
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def default_threads() -> int:
    return int(lib().vor_oracle_default_threads())


def _region_args(region):
    vx = np.ascontiguousarray(region[0], dtype=np.int32)
    vy = np.ascontiguousarray(region[1], dtype=np.int32)
    return vx, vy, (vx.shape[0], _p(vx, C.c_int32), _p(vy, C.c_int32))


def validate(x, y, box, region=None) -> int:
    """0, or the oracle's error code; X is the box, or the convex polygon region = (vx, vy)."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    if region is not None:
        vx, vy, ra = _region_args(region)
        return int(lib().vor_oracle_validate_poly(x.shape[0], _p(x, C.c_int32),
                                                  _p(y, C.c_int32), *ra))
    return int(lib().vor_oracle_validate(x.shape[0], _p(x, C.c_int32), _p(y, C.c_int32), *box))


@dataclass
class Cells:
    cells: np.ndarray    # int32 [m]  site index of each computed cell
    counts: np.ndarray   # int32 [m]
    off: np.ndarray      # int64 [m+1]
    nbr: np.ndarray      # int32 [sum counts]
    vx: np.ndarray | None = None   # object array of Python ints (X numerators)
    vy: np.ndarray | None = None
    vd: np.ndarray | None = None   # int64
    vwords: np.ndarray | None = None   # uint64 [E, 5] with raw=True

    def lines(self, i: int) -> list:
        return self.nbr[self.off[i]:self.off[i + 1]].tolist()


def cells(x, y, box, which=None, threads: int | None = None, vertices: bool = True,
          region=None, raw: bool = False) -> Cells:
    """Cells of the listed sites (all by default).  X is the box, or, when region = (vx, vy) is
    given, that convex polygon (counter-clockwise; sides named -1, -2, ...).  raw: keep the
    vertices as 64-bit words only (``vwords`` [E, 5]: X low, X high, Y low, Y high, D, the
    little-endian layout of a pair-form vertex) instead of Python integers."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    n = x.shape[0]
    if which is None:
        which = np.arange(n, dtype=np.int32)
    which = np.ascontiguousarray(which, dtype=np.int32)
    m = which.shape[0]
    counts = np.zeros(max(m, 1), dtype=np.int32)
    if threads is None:
        threads = default_threads()
    cap = max(16, 12 * m)
    needed = C.c_int64(0)
    for attempt in range(3):
        buf = np.zeros(cap, dtype=np.int32)
        if region is not None:
            vx, vy, ra = _region_args(region)
            r = lib().vor_oracle_cells_poly(n, _p(x, C.c_int32), _p(y, C.c_int32), *ra, m,
                                            _p(which, C.c_int32), int(threads),
                                            _p(counts, C.c_int32), cap, _p(buf, C.c_int32),
                                            C.byref(needed))
        else:
            r = lib().vor_oracle_cells(n, _p(x, C.c_int32), _p(y, C.c_int32), *box, m,
                                       _p(which, C.c_int32), int(threads),
                                       _p(counts, C.c_int32), cap, _p(buf, C.c_int32),
                                       C.byref(needed))
        if r == -4 and attempt < 2 and int(needed.value) + 16 > cap:
            cap = int(needed.value) + 16
            continue
        if r < 0:
            raise ValueError(f"oracle error {r}: {ERRORS.get(int(r), '?')}")
        break
    counts = counts[:m]
    off = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    nbr = buf[:off[-1]].copy()
    out = Cells(which, counts, off, nbr)
    if vertices:
        tot = int(off[-1])
        X2 = np.zeros(2 * max(tot, 1), dtype=np.uint64)
        Y2 = np.zeros(2 * max(tot, 1), dtype=np.uint64)
        D = np.zeros(max(tot, 1), dtype=np.int64)
        tail = (m, _p(which, C.c_int32), _p(counts, C.c_int32), _p(nbr, C.c_int32),
                _p(X2, C.c_uint64), _p(Y2, C.c_uint64), _p(D, C.c_int64))
        if region is not None:
            vx, vy, ra = _region_args(region)
            r = lib().vor_oracle_vertices_poly(n, _p(x, C.c_int32), _p(y, C.c_int32), *ra,
                                               *tail)
        else:
            r = lib().vor_oracle_vertices(n, _p(x, C.c_int32), _p(y, C.c_int32), *box, *tail)
        if r != 0:
            raise ValueError("oracle vertex error")
        if raw:
            w = np.empty((tot, 5), dtype=np.uint64)
            w[:, 0] = X2[0:2 * tot:2]
            w[:, 1] = X2[1:2 * tot:2]
            w[:, 2] = Y2[0:2 * tot:2]
            w[:, 3] = Y2[1:2 * tot:2]
            w[:, 4] = D[:tot].view(np.uint64)
            out.vwords = w
            return out
        out.vx = limbs_to_int(X2[:2 * tot])
        out.vy = limbs_to_int(Y2[:2 * tot])
        out.vd = D[:tot].copy()
    return out


def limbs_to_int(a: np.ndarray) -> np.ndarray:
    """(lo, hi) uint64 pairs of a two's-complement int128 -> object array of Python ints."""
    lo = a[0::2].astype(object)
    hi = a[1::2].astype(np.int64).astype(object)
    return np.array([int(h) * (1 << 64) + int(l) for l, h in zip(lo, hi)], dtype=object)


def delaunay(c: Cells) -> np.ndarray:
    """Delaunay graph restricted to X (Section 7): pairs (i, j), i < j, j a neighbour of i via
    an edge; sorted lexicographically.  Needs every cell (which == arange(n))."""
    k = np.repeat(c.cells.astype(np.int64), c.counts)
    j = c.nbr.astype(np.int64)
    sel = (j >= 0) & (j > k)
    pairs = np.stack([k[sel], j[sel]], axis=1)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return pairs[order].astype(np.uint32)
