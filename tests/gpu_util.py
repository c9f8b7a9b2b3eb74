"""Helpers shared by the GPU tests: run the HIP path and compare with the oracle."""
import sys

import numpy as np

from oracle import cdiagram


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_matches_oracle(r, ps, which=None, vertices=True):
    """Element-by-element equality of neighbour lists (and pair-form vertices) with the oracle,
    for all cells or for the listed cells."""
    oc = cdiagram.cells(ps.x, ps.y, ps.box, which=which, region=getattr(ps, "region", None))
    if which is None:
        assert r.cell_off.shape[0] == ps.n + 1
        assert np.array_equal(r.cell_off.astype(np.int64), oc.off), "cell offsets"
        if not np.array_equal(r.nbr, oc.nbr):
            bad = [k for k in range(ps.n) if r.lines(k) != oc.lines(k)]
            raise AssertionError(f"{len(bad)} cells differ, first {bad[:5]}: "
                                 f"gpu {r.lines(bad[0])} oracle {oc.lines(bad[0])}")
        if vertices:
            X, Y, D = r.vertices_int()
            assert X == list(oc.vx), "vertex X"
            assert Y == list(oc.vy), "vertex Y"
            assert D == [int(v) for v in oc.vd], "vertex D"
        assert np.array_equal(r.dele, cdiagram.delaunay(oc)), "delaunay edges"
        return oc
    for i, k in enumerate(which):
        got = r.lines(int(k))
        exp = oc.lines(i)
        assert got == exp, f"cell {k}: gpu {got} oracle {exp}"
        if vertices and r.vtx is not None:
            lo, hi = int(r.cell_off[k]), int(r.cell_off[k + 1])
            v = r.vtx[lo:hi]
            X = [int(h) * (1 << 64) + int(l) for l, h in zip(v["x_lo"], v["x_hi"])]
            Y = [int(h) * (1 << 64) + int(l) for l, h in zip(v["y_lo"], v["y_hi"])]
            o0, o1 = int(oc.off[i]), int(oc.off[i + 1])
            assert X == list(oc.vx[o0:o1]) and Y == list(oc.vy[o0:o1])
            assert [int(d) for d in v["d"]] == [int(d) for d in oc.vd[o0:o1]]
    return oc


def symmetric(r):
    n = r.n
    k = np.repeat(np.arange(n, dtype=np.int64), np.diff(r.cell_off.astype(np.int64)))
    j = r.nbr.astype(np.int64)
    s = j >= 0
    a = set(zip(k[s].tolist(), j[s].tolist()))
    return all((b, a_) in a for (a_, b) in a)
