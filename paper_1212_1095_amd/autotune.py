"""Autotuner: picks the grid density, block half-width, workgroup size, leaf half-width and
scan path for a workload shape by timing the C-ABI pipeline on the device (results are exact
whatever the parameters; only the speed changes).

    python -m paper_1212_1095_amd.autotune --n 1048576 --box 16777216 [--out tuning.json]
    python -m paper_1212_1095_amd.autotune --batch --box 1048576 [--out tuning.json]

The table maps a distribution tag and "log2(n)" (rounded) to the best (sites_per_bucket, block,
block_halfwidth, leaf_halfwidth, scan_path).  ``best_params`` looks a shape up (nearest
log2 n) and returns the arguments of ``Context.tune``.  With --batch the sweep times batches of
equal-sized sets (about 2^20 sites per batch) for every size class 2^5 .. 2^16 and stores the
per-set parameters (sites_per_bucket, block_halfwidth, leaf_halfwidth) under "<dist>_batch";
``size_table`` turns that into the argument of ``Context.size_tuning``, which the library
applies set by set inside a batch or an admitted group of requests.  Every entry of the shipped
table is written by this script from its sweep grid (the "grid" field says which points).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")

# (sites_per_bucket, block_halfwidth, leaf_halfwidth, scan_path)
DEFAULT_GRID = [(0.5, 1, 0, 0), (0.7, 1, 0, 0), (1.0, 1, 0, 0), (1.5, 1, 0, 0), (2.0, 1, 0, 0),
                (0.35, 2, 0, 0), (0.5, 2, 0, 0), (0.7, 2, 0, 0), (1.0, 2, 0, 0),
                (1.25, 2, 0, 0), (1.5, 2, 0, 0), (2.0, 2, 0, 0), (1.5, 3, 0, 0),
                (1.0, 0, 1, 0), (1.0, 0, 0, 1), (2.0, 0, 0, 1), (3.0, 0, 0, 1)]
# per-set parameters of a batch (block and scan path are launch-wide and stay the context's)
BATCH_GRID = [(0.7, 1, 0), (1.0, 1, 0), (1.5, 1, 0), (2.0, 1, 0), (0.7, 2, 0), (1.0, 2, 0),
              (1.5, 2, 0), (2.0, 2, 0), (1.5, 3, 0)]
BATCH_SIZES = list(range(5, 17))
DEFAULT_BLOCKS = (256,)
KEYS = ("sites_per_bucket", "block", "block_halfwidth", "leaf_halfwidth", "scan_path")


def time_config(ctx, xd, yd, n, box, rho, h, block, ht=0, path=0, reps=5, warmup=2):
    import torch
    ctx.tune(rho, block, h, ht, path)
    for _ in range(warmup):
        ctx.compute((xd.data_ptr(), n), (yd.data_ptr(), n), box, device_ptrs=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = ctx.compute((xd.data_ptr(), n), (yd.data_ptr(), n), box, device_ptrs=True)
    torch.cuda.synchronize()
    return 1000.0 * (time.perf_counter() - t0) / reps, r


def sweep(x, y, box, grid=DEFAULT_GRID, blocks=DEFAULT_BLOCKS, reps=5, log=print):
    import numpy as np
    import torch
    from ._binding import Context, VOR_RESULT_DEVICE, VOR_TIME_KERNELS
    n = int(np.asarray(x).shape[0])
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.int32)).cuda()
    rows = []
    with Context(flags=VOR_RESULT_DEVICE | VOR_TIME_KERNELS) as ctx:
        for rho, h, ht, path in grid:
            for block in blocks:
                ms, r = time_config(ctx, xd, yd, n, box, rho, h, block, ht, path, reps)
                row = {"sites_per_bucket": rho, "block_halfwidth": h, "block": block,
                       "leaf_halfwidth": ht, "scan_path": path, "ms": ms,
                       "cells_ms": r.cells_ms, "adaptive_ms": r.adaptive_ms,
                       "exact_ms": r.exact_ms,
                       "evals_per_cell": r.stats.evals / n, "shells_per_cell": r.stats.shells / n}
                rows.append(row)
                log(json.dumps(row))
    rows.sort(key=lambda r: r["ms"])
    return rows


def sweep_batch(sizes_log2, box, dist="uniform", grid=BATCH_GRID, reps=3, seed=4, log=print,
                target_sites=1 << 20):
    """For each size class 2^k: a batch of equal-sized sets (about target_sites in all), every
    grid point applied to all sets; returns {k: [rows sorted by device ms]}."""
    import numpy as np
    import sitegen
    from ._binding import Context, VOR_NO_VERTICES
    gen = {"uniform": sitegen.uniform, "clustered": sitegen.clustered}[dist]
    out = {}
    for k in sizes_log2:
        n = 1 << k
        count = max(1, target_sites // n)
        sets = [gen(n, box, seed=seed * 1_000_003 + k * 4096 + i) for i in range(count)]
        args = [(s.x, s.y, s.box) for s in sets]
        rows = []
        with Context(flags=VOR_NO_VERTICES) as ctx:
            for rho, h, ht in grid:
                ctx.size_tuning([(k, rho, h, ht)])
                ctx.compute_batch(args)   # warm-up, graph capture
                ms = []
                for _ in range(reps):
                    rc, res = ctx.compute_batch(args)
                    ms.append(res[0].device_ms)
                row = {"sites_per_bucket": rho, "block_halfwidth": h, "leaf_halfwidth": ht,
                       "ms": float(np.min(ms)), "sets": count, "n": n}
                rows.append(row)
                log(json.dumps(row))
        rows.sort(key=lambda r: r["ms"])
        out[k] = rows
    return out


def size_table(dist="uniform", path=TABLE):
    """The per-set entries [(log2 n, sites_per_bucket, block_halfwidth, leaf_halfwidth)] of the
    table's "<dist>_batch" section, for Context.size_tuning (empty when there are none)."""
    t = load_table(path).get(dist + "_batch", {})
    return [(int(k), float(e["sites_per_bucket"]), int(e["block_halfwidth"]),
             int(e.get("leaf_halfwidth", 0))) for k, e in sorted(t.items(), key=lambda x: int(x[0]))]


def load_table(path=TABLE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def best_params(n: int, dist: str = "uniform", path=TABLE):
    """(sites_per_bucket, block, block_halfwidth, leaf_halfwidth, scan_path) for the nearest
    tuned log2(n), or None."""
    t = load_table(path).get(dist, {})
    if not t:
        return None
    key = min(t.keys(), key=lambda k: abs(int(k) - round(math.log2(max(n, 1)))))
    e = t[key]
    return tuple(e.get(k, d) for k, d in zip(KEYS, (1.0, 256, 0, 0, 0)))


def main():
    sys.path.insert(0, os.path.dirname(HERE))
    import sitegen
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--box", type=int, default=1 << 24)
    ap.add_argument("--dist", default="uniform", choices=["uniform", "clustered", "lattice"])
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=None, help="merge the best entry into this table")
    ap.add_argument("--batch", action="store_true",
                    help="per-set parameters of batches, size classes 2^5..2^16")
    a = ap.parse_args()
    if a.batch:
        res = sweep_batch(BATCH_SIZES, a.box, a.dist, reps=a.reps,
                          log=lambda s: print(s, flush=True))
        if a.out:
            t = load_table(a.out)
            sec = t.setdefault(a.dist + "_batch", {})
            for k, rows in res.items():
                best = rows[0]
                sec[str(k)] = {kk: best[kk] for kk in ("sites_per_bucket", "block_halfwidth",
                                                       "leaf_halfwidth", "ms", "sets")}
                sec[str(k)]["grid"] = "BATCH_GRID"
                sec[str(k)]["box"] = a.box
            with open(a.out, "w") as f:
                json.dump(t, f, indent=1, sort_keys=True)
        return
    gen = {"uniform": sitegen.uniform, "clustered": sitegen.clustered,
           "lattice": sitegen.lattice}[a.dist]
    ps = gen(a.n, a.box, seed=a.seed)
    rows = sweep(ps.x, ps.y, ps.box, reps=a.reps, log=lambda s: print(s, flush=True))
    best = rows[0]
    print(json.dumps({"best": best}), flush=True)
    if a.out:
        t = load_table(a.out)
        e = {k: best[k] for k in KEYS + ("ms",)}
        e["grid"] = "DEFAULT_GRID"
        e["n"], e["box"], e["seed"] = a.n, a.box, a.seed
        t.setdefault(a.dist, {})[str(round(math.log2(a.n)))] = e
        with open(a.out, "w") as f:
            json.dump(t, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
