"""Lloyd iterations on the integer grid -- TEST INFRASTRUCTURE ONLY.

The paper motivates fast diagram computation by algorithms that recompute the diagram many
times, centroidal Voronoi relaxation among them.  One step, as this library defines it (the paper
fixes no rounding), with the cell computed by the C oracle (the plain definition):

1. for each cell k with site p and vertices (X_t/D_t, Y_t/D_t) in the stored order, the vertex
   relative to p is u_t = (fl(X_t - p_x D_t) / fl(D_t), fl(Y_t - p_y D_t) / fl(D_t)) in IEEE
   double (fl: correctly rounded conversion of the exact integer);
2. c_t = u_t.x u_{t+1}.y - u_{t+1}.x u_t.y (two products, then the difference), A2 = sum c_t,
   S = sum (u_t + u_{t+1}) c_t (sums from t = 0 upwards), centroid offset = S / (3 A2);
3. the proposal is p + rint(offset) (round half to even); a proposal not strictly inside X is
   replaced by p;
4. collisions: while some position is proposed by more than one site, every such site whose
   proposal differs from its own current position goes back to it (sites at their current
   positions never collide with each other, so this ends).
"""
from __future__ import annotations

import numpy as np

from . import cdiagram
from . import region as _region


def _centroid_offset(X, Y, D, px, py):
    m = len(D)
    ux = [float(int(X[t]) - px * int(D[t])) / float(int(D[t])) for t in range(m)]
    uy = [float(int(Y[t]) - py * int(D[t])) / float(int(D[t])) for t in range(m)]
    a2 = 0.0
    sx = 0.0
    sy = 0.0
    for t in range(m):
        s = (t + 1) % m
        c = ux[t] * uy[s] - ux[s] * uy[t]
        a2 += c
        sx += (ux[t] + ux[s]) * c
        sy += (uy[t] + uy[s]) * c
    return sx / (3.0 * a2), sy / (3.0 * a2)


def proposals(x, y, box, region=None):
    """Step 1-3: the rounded centroid of every cell (or the site where that leaves X)."""
    n = len(x)
    oc = cdiagram.cells(x, y, box, region=region)
    lines = _region.side_lines(box, region)
    px_new = np.array(x, dtype=np.int64)
    py_new = np.array(y, dtype=np.int64)
    for k in range(n):
        o0, o1 = int(oc.off[k]), int(oc.off[k + 1])
        px, py = int(x[k]), int(y[k])
        cx, cy = _centroid_offset(oc.vx[o0:o1], oc.vy[o0:o1], oc.vd[o0:o1], px, py)
        qx, qy = px + int(np.rint(cx)), py + int(np.rint(cy))
        if all(nx * qx + ny * qy < c for nx, ny, c in lines):
            px_new[k], py_new[k] = qx, qy
    return px_new, py_new


def resolve(x, y, qx, qy):
    """Step 4 on proposals (qx, qy) from current sites (x, y); returns the new sites and the
    number of rounds that reverted something."""
    qx = np.array(qx, dtype=np.int64)
    qy = np.array(qy, dtype=np.int64)
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    rounds = 0
    while True:
        key = (qx << 32) ^ (qy & 0xFFFFFFFF)
        _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
        clash = (cnt[inv] > 1) & ((qx != x) | (qy != y))
        if not clash.any():
            return qx, qy, rounds
        qx[clash] = x[clash]
        qy[clash] = y[clash]
        rounds += 1


def step(x, y, box, region=None):
    """One Lloyd step: (new x, new y, number of sites moved, reverting rounds)."""
    qx, qy = proposals(x, y, box, region)
    nx, ny, rounds = resolve(x, y, qx, qy)
    moved = int(np.count_nonzero((nx != np.asarray(x)) | (ny != np.asarray(y))))
    return nx.astype(np.int32), ny.astype(np.int32), moved, rounds


def iterate(x, y, box, iters, region=None):
    """`iters` steps: (final x, final y, [sites moved per step])."""
    moved = []
    for _ in range(iters):
        x, y, m, _ = step(x, y, box, region)
        moved.append(m)
    return np.asarray(x, np.int32), np.asarray(y, np.int32), moved
