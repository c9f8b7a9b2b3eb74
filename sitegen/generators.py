"""Input recipes (shapes, sizes and value distributions of the five workloads).

* uniform    : integers uniform in [1, B-1]^2, X = [0, B]^2.
* clustered  : 90% from 64 isotropic Gaussians (centres uniform in [0, B)^2, sigma = 2^(8 + 8U)),
               rounded half-to-even and clipped to [1, B-1]; 10% uniform background.
* lattice    : a contiguous ceil(sqrt(n)) x ceil(sqrt(n)) block of the lattice 2^9 + 2^10 (i, j),
               truncated to n points, each coordinate jittered by an independent draw from {-1, 0, 1}.
* batch      : set sizes floor(32 * 2048^U) clamped to [32, 65536], uniform sites in [1, 2^20 - 1]^2.
* requests   : Poisson arrivals, sizes log-uniform in [100, 2^20], class mix 45/45/10
               (uniform / clustered / lattice) in [1, 2^24 - 1]^2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class PointSet:
    x: np.ndarray            # int32 [n]
    y: np.ndarray            # int32 [n]
    box: tuple               # (x0, y0, x1, y1), X = [x0, x1] x [y0, y1]
    kind: str = "uniform"
    seed: int = 0
    meta: dict = field(default_factory=dict)
    region: tuple | None = None   # (vx, vy) int32: X is this convex polygon (box = its bbox)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _first_occurrence_mask(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """True for every point that does not repeat an earlier point (draw order)."""
    key = (x.astype(np.int64) << 32) | (y.astype(np.int64) & 0xFFFFFFFF)
    _, first = np.unique(key, return_index=True)
    keep = np.zeros(x.shape[0], dtype=bool)
    keep[first] = True
    return keep


def _redraw_until_distinct(x, y, draw_one_batch, lo, hi, max_rounds=1000):
    """Redraw (in the same stream) every point that is a repeat or lies outside [lo, hi]."""
    for _ in range(max_rounds):
        bad = ~_first_occurrence_mask(x, y)
        bad |= (x < lo) | (x > hi) | (y < lo) | (y > hi)
        idx = np.nonzero(bad)[0]
        if idx.size == 0:
            return x, y
        nx, ny = draw_one_batch(idx)
        x[idx] = nx
        y[idx] = ny
    raise RuntimeError("could not draw distinct interior sites")


def uniform(n: int, B: int = 1 << 16, seed: int = 1) -> PointSet:
    rng = _rng(seed)
    pts = rng.integers(1, B, size=(n, 2), dtype=np.int64)
    x = pts[:, 0].copy()
    y = pts[:, 1].copy()

    def draw(idx):
        p = rng.integers(1, B, size=(idx.size, 2), dtype=np.int64)
        return p[:, 0], p[:, 1]

    x, y = _redraw_until_distinct(x, y, draw, 1, B - 1)
    return PointSet(x.astype(np.int32), y.astype(np.int32), (0, 0, B, B), "uniform", seed)


def clustered(n: int, B: int = 1 << 24, seed: int = 3, n_clusters: int = 64,
              frac: float = 0.9) -> PointSet:
    rng = _rng(seed)
    centres = rng.uniform(0, B, size=(n_clusters, 2))
    sigma = 2.0 ** (8.0 + 8.0 * rng.uniform(0, 1, size=n_clusters))
    n_c = int(round(frac * n))
    cls = np.full(n, -1, dtype=np.int64)
    cls[:n_c] = rng.integers(0, n_clusters, size=n_c)

    def draw_for(idx):
        out = np.empty((idx.size, 2), dtype=np.int64)
        c = cls[idx]
        g = c >= 0
        if g.any():
            k = c[g]
            v = centres[k] + sigma[k][:, None] * rng.standard_normal(size=(int(g.sum()), 2))
            out[g] = np.clip(np.rint(v), 1, B - 1).astype(np.int64)
        if (~g).any():
            out[~g] = rng.integers(1, B, size=(int((~g).sum()), 2), dtype=np.int64)
        return out[:, 0], out[:, 1]

    x, y = draw_for(np.arange(n))
    x, y = _redraw_until_distinct(x.copy(), y.copy(), draw_for, 1, B - 1)
    return PointSet(x.astype(np.int32), y.astype(np.int32), (0, 0, B, B), "clustered", seed,
                    {"sigma": sigma.tolist()})


def lattice(n: int, B: int = 1 << 24, seed: int = 5, spacing: int = 1 << 10,
            offset: int = 1 << 9) -> PointSet:
    rng = _rng(seed)
    side = int(math.ceil(math.sqrt(n)))
    per_axis = (B - offset) // spacing          # lattice points 2^9 + 2^10 i <= B - 1 - 1
    if side > per_axis:
        raise ValueError("lattice block does not fit the box")
    ox, oy = rng.integers(0, per_axis - side + 1, size=2)
    k = np.arange(n)
    i = ox + (k % side)
    j = oy + (k // side)
    jit = rng.integers(-1, 2, size=(n, 2))
    x = offset + spacing * i + jit[:, 0]
    y = offset + spacing * j + jit[:, 1]
    return PointSet(x.astype(np.int32), y.astype(np.int32), (0, 0, B, B), "lattice", seed)


def batch_sizes(k: int = 4096, seed: int = 4, lo: int = 32, hi: int = 65536) -> np.ndarray:
    rng = _rng(seed)
    u = rng.uniform(0, 1, size=k)
    n = np.floor(lo * (hi / lo) ** u).astype(np.int64)
    return np.clip(n, lo, hi)


def batch_sets(k: int = 4096, seed: int = 4, B: int = 1 << 20, lo: int = 32,
               hi: int = 65536, sizes=None) -> list:
    """Independent uniform sets of uneven size; set s uses sub-seed (seed, s)."""
    if sizes is None:
        sizes = batch_sizes(k, seed, lo, hi)
    out = []
    for s, n in enumerate(sizes):
        ps = uniform(int(n), B, seed=int(seed) * 1_000_003 + s)
        ps.kind = "batch"
        out.append(ps)
    return out


def request_stream(count: int, qps: float, seed: int = 5, lo: int = 100, hi: int = 1 << 20,
                   B: int = 1 << 24, mix=(0.45, 0.45, 0.10)):
    """Poisson request stream: returns a list of (arrival_time_s, PointSet)."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps)
    u = rng.uniform(0, 1, size=count)
    sizes = np.floor(lo * (hi / lo) ** u).astype(np.int64)
    cls = rng.choice(3, size=count, p=list(mix))
    reqs = []
    for r in range(count):
        sub = int(seed) * 1_000_003 + r
        n = int(sizes[r])
        if cls[r] == 0:
            ps = uniform(n, B, seed=sub)
        elif cls[r] == 1:
            ps = clustered(n, B, seed=sub)
        else:
            ps = lattice(n, B, seed=sub)
        reqs.append((float(t[r]), ps))
    return reqs


def small_integer_set(n: int, coord_max: int, seed: int, box_pad: int = 1) -> PointSet:
    """Tiny sets with many ties (small coordinates): sites in [box_pad, coord_max]^2,
    box [0, coord_max + box_pad]^2."""
    rng = _rng(seed)
    B = coord_max + box_pad
    lo = box_pad
    pts = rng.integers(lo, coord_max + 1, size=(n, 2), dtype=np.int64)
    x = pts[:, 0].copy()
    y = pts[:, 1].copy()

    def draw(idx):
        p = rng.integers(lo, coord_max + 1, size=(idx.size, 2), dtype=np.int64)
        return p[:, 0], p[:, 1]

    x, y = _redraw_until_distinct(x, y, draw, lo, coord_max)
    return PointSet(x.astype(np.int32), y.astype(np.int32), (0, 0, B, B), "small", seed)


def convex_polygon(K: int, B: int = 1 << 20, seed: int = 7, origin: int = 0) -> tuple:
    """A strictly convex polygon with at most K integer vertices, counter-clockwise, inside
    [origin, origin + B]^2: K sorted random angles on an ellipse of random axes, rounded, then
    the convex hull with collinear points dropped.  Returns (vx, vy) int32 arrays."""
    rng = _rng(seed)
    ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=K))
    ax, ay = rng.uniform(0.3, 0.5, size=2) * B
    cx, cy = origin + B / 2, origin + B / 2
    px = np.rint(cx + ax * np.cos(ang)).astype(np.int64)
    py = np.rint(cy + ay * np.sin(ang)).astype(np.int64)
    pts = sorted(set(zip(px.tolist(), py.tolist())))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    hull = lower[:-1] + upper[:-1]
    if len(hull) < 3:
        raise ValueError("degenerate polygon")
    return (np.array([p[0] for p in hull], np.int32), np.array([p[1] for p in hull], np.int32))


def inside_polygon(region, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Strictly inside the counter-clockwise convex polygon: strictly left of every edge."""
    vx = np.asarray(region[0], np.int64)
    vy = np.asarray(region[1], np.int64)
    ok = np.ones(px.shape[0], dtype=bool)
    for e in range(vx.shape[0]):
        f = (e + 1) % vx.shape[0]
        ok &= (vx[f] - vx[e]) * (py - vy[e]) - (vy[f] - vy[e]) * (px - vx[e]) > 0
    return ok


def in_polygon(n: int, region, seed: int = 1, kind: str = "uniform") -> PointSet:
    """n distinct sites strictly inside the convex polygon region = (vx, vy): uniform over the
    polygon, or clustered (90% from 8 Gaussians with centres inside, sigma 1/64 of the extent,
    10% uniform).  The box is the polygon's bounding box."""
    rng = _rng(seed)
    vx = np.asarray(region[0], np.int64)
    vy = np.asarray(region[1], np.int64)
    x0, x1, y0, y1 = int(vx.min()), int(vx.max()), int(vy.min()), int(vy.max())
    ext = max(x1 - x0, y1 - y0)
    centres = []
    while kind == "clustered" and len(centres) < 8:
        c = rng.integers([x0, y0], [x1 + 1, y1 + 1], size=(1, 2))
        if inside_polygon(region, c[:, 0], c[:, 1])[0]:
            centres.append(c[0])

    def draw(m):
        if kind == "clustered":
            u = rng.random(m) < 0.1
            k = rng.integers(0, len(centres), size=m)
            g = np.array(centres)[k] + rng.normal(0.0, ext / 64.0, size=(m, 2))
            b = rng.integers([x0, y0], [x1 + 1, y1 + 1], size=(m, 2))
            p = np.where(u[:, None], b, np.rint(g)).astype(np.int64)
        else:
            p = rng.integers([x0, y0], [x1 + 1, y1 + 1], size=(m, 2))
        return p[:, 0], p[:, 1]

    xs = np.zeros(0, np.int64)
    ys = np.zeros(0, np.int64)
    for _ in range(1000):
        if xs.shape[0] >= n:
            break
        px, py = draw(2 * (n - xs.shape[0]) + 16)
        keep = inside_polygon(region, px, py)
        xs = np.concatenate([xs, px[keep]])
        ys = np.concatenate([ys, py[keep]])
        first = _first_occurrence_mask(xs, ys)
        xs, ys = xs[first], ys[first]
    if xs.shape[0] < n:
        raise ValueError("the polygon holds fewer distinct interior points than requested")
    xs, ys = xs[:n], ys[:n]
    return PointSet(xs.astype(np.int32), ys.astype(np.int32), (x0, y0, x1, y1), kind, seed,
                    region=(vx.astype(np.int32), vy.astype(np.int32)))


def boundary_points(box, region=None, count: int = 8, seed: int = 1):
    """`count` distinct integer points on the boundary of X (sides and corners): X is the box
    (x0, y0, x1, y1), or the convex polygon region = (vx, vy), whose side from v_e to v_{e+1}
    holds the points v_e + t (dx, dy) / gcd(|dx|, |dy|), t = 0 .. gcd."""
    rng = _rng(seed)
    if region is None:
        x0, y0, x1, y1 = box
        region = (np.array([x0, x1, x1, x0], np.int64), np.array([y0, y0, y1, y1], np.int64))
    vx = np.asarray(region[0], np.int64)
    vy = np.asarray(region[1], np.int64)
    K = vx.shape[0]
    pts = {(int(vx[e]), int(vy[e])) for e in rng.permutation(K)[:max(1, count // 4)]}
    for _ in range(50 * count):
        if len(pts) >= count:
            break
        e = int(rng.integers(0, K))
        f = (e + 1) % K
        dx, dy = int(vx[f] - vx[e]), int(vy[f] - vy[e])
        g = math.gcd(abs(dx), abs(dy))
        t = int(rng.integers(0, g + 1))
        pts.add((int(vx[e]) + t * (dx // g), int(vy[e]) + t * (dy // g)))
    pts = sorted(pts)[:count]
    order = rng.permutation(len(pts))
    return (np.array([pts[i][0] for i in order], np.int32),
            np.array([pts[i][1] for i in order], np.int32))


def with_boundary_sites(ps: PointSet, count: int, seed: int = 1) -> PointSet:
    """ps with up to `count` more sites on the boundary of its X (distinct from its sites),
    inserted at random positions of the id order."""
    rng = _rng(seed)
    bx, by = boundary_points(ps.box, ps.region, count, seed)
    have = set(zip(ps.x.tolist(), ps.y.tolist()))
    keep = [i for i in range(bx.shape[0]) if (int(bx[i]), int(by[i])) not in have]
    x = np.concatenate([ps.x, bx[keep]])
    y = np.concatenate([ps.y, by[keep]])
    perm = rng.permutation(x.shape[0])
    return PointSet(x[perm].astype(np.int32), y[perm].astype(np.int32), ps.box,
                    ps.kind + "+boundary", ps.seed, dict(ps.meta), ps.region)
