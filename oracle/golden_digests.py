"""Digests of the oracle's full diagrams for the five workloads -- TEST INFRASTRUCTURE ONLY.

Writes ``tests/golden/fullsize_digests.json``: SHA-256 digests of the canonical output arrays
that the oracle (exact half-plane clipping, ``cdiagram``) gives for every cell of

* config1  n = 1,000 uniform sites in [1, 2^16)^2, X = [0, 2^16]^2, seed 1;
* config2  n = 2^20 uniform sites in [1, 2^24)^2, X = [0, 2^24]^2, seed 2;
* config3  n = 2^20 clustered sites (64 Gaussians + 10% uniform), X = [0, 2^24]^2, seed 3;
* config1_batch  4,096 sets of the config-1 shape (n = 1,000 uniform in [1, 2^16)^2, X =
           [0, 2^16]^2), seeds 1001..5096 (the batched small-set shape);
* config4  4,096 sets, sizes log-uniform in [32, 65536], uniform in [1, 2^20)^2, seed 4;
* config5  every request with n <= 2^16 of the 200-request stream (seed 5, sizes log-uniform in
           [100, 2^20], 45/45/10 uniform / clustered / lattice in [1, 2^24)^2).

Inputs come from ``sitegen`` and results from ``oracle`` only.  The canonical form of one
diagram (Section 6 representation, Section 7 Delaunay graph) is four little-endian arrays:
``cell_off`` uint32 [n+1], ``nbr`` int32 [E], ``vtx`` 40-byte pair-form vertices [E] (X low,
X high, Y low, Y high as 64-bit words of the two 128-bit numerators, then the 64-bit D), and
``del`` uint32 [2m] (pairs i < j in lexicographic order).  A set of several diagrams (config 4,
config 5) hashes the concatenation of its diagrams' arrays per kind, and also keeps one short
digest per diagram so that a mismatch names its set.

Run: ``python -m oracle.golden_digests [config1 config2 ...]`` (default: all); entries of
configs not named are kept from the existing file.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import sitegen  # noqa: E402
from oracle import cdiagram  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "fullsize_digests.json")
KINDS = ("cell_off", "nbr", "vtx", "del")
CONFIG5_COUNT = 200
CONFIG5_MAX_N = 1 << 16


def canonical_bytes(off, nbr, vwords, dele):
    """The four canonical byte strings of one diagram (vwords may be None: no vertices)."""
    return {
        "cell_off": np.ascontiguousarray(np.asarray(off).astype(np.int64).astype("<u4")).tobytes(),
        "nbr": np.ascontiguousarray(np.asarray(nbr), dtype="<i4").tobytes(),
        "vtx": (None if vwords is None else
                np.ascontiguousarray(np.asarray(vwords).reshape(-1, 5), dtype="<u8").tobytes()),
        "del": np.ascontiguousarray(np.asarray(dele).reshape(-1), dtype="<u4").tobytes(),
    }


class Digest:
    """Running SHA-256 per array kind over one or more diagrams, plus a short digest of each."""

    def __init__(self):
        self.h = {k: hashlib.sha256() for k in KINDS}
        self.per = []

    def add(self, off, nbr, vwords, dele):
        b = canonical_bytes(off, nbr, vwords, dele)
        one = hashlib.sha256()
        for k in KINDS:
            if b[k] is None:
                continue
            self.h[k].update(b[k])
            one.update(b[k])
        self.per.append(one.hexdigest()[:16])

    def result(self, per_set=False):
        out = {"sha256": {k: v.hexdigest() for k, v in self.h.items()}}
        if per_set:
            out["per_set"] = self.per
        return out


def oracle_diagram(ps, threads=None):
    """(off, nbr, vwords, del) of every cell of ps by the oracle."""
    oc = cdiagram.cells(ps.x, ps.y, ps.box, threads=threads, vertices=True, raw=True,
                        region=getattr(ps, "region", None))
    return oc.off, oc.nbr, oc.vwords, cdiagram.delaunay(oc)


def config_sets(name):
    """(description, [PointSet]) of a named workload."""
    if name == "config1":
        return ("n=1000 uniform in [1,2^16)^2, X=[0,2^16]^2, seed 1",
                [sitegen.uniform(1000, 1 << 16, seed=1)])
    if name == "config2":
        return ("n=2^20 uniform in [1,2^24)^2, X=[0,2^24]^2, seed 2",
                [sitegen.uniform(1 << 20, 1 << 24, seed=2)])
    if name == "config3":
        return ("n=2^20 clustered (64 Gaussians, sigma 2^(8+8U), 10% uniform), X=[0,2^24]^2, "
                "seed 3", [sitegen.clustered(1 << 20, 1 << 24, seed=3)])
    if name == "config1_batch":
        return ("4096 sets of n=1000 uniform in [1,2^16)^2, X=[0,2^16]^2, seeds 1001..5096",
                config1_batch_sets())
    if name == "config4":
        return ("4096 sets, sizes floor(32*2048^U) in [32,65536], uniform in [1,2^20)^2, "
                "X=[0,2^20]^2, seed 4 (set s: sub-seed 4*1000003+s)",
                sitegen.batch_sets(4096, 4, B=1 << 20, lo=32, hi=65536))
    if name == "config5":
        reqs = config5_requests()
        return (f"requests with n <= {CONFIG5_MAX_N} of the {CONFIG5_COUNT}-request stream "
                f"(seed 5, sizes log-uniform in [100,2^20], 45/45/10 uniform/clustered/lattice), "
                f"in stream order", [ps for _, ps in reqs])
    raise KeyError(name)


def config1_batch_sets(k=4096):
    return [sitegen.uniform(1000, 1 << 16, seed=1001 + i) for i in range(k)]


def config5_requests():
    """(index in the stream, PointSet) of the config-5 requests the digests cover."""
    reqs = sitegen.request_stream(CONFIG5_COUNT, 1.0, seed=5, lo=100, hi=1 << 20)
    return [(i, ps) for i, (_, ps) in enumerate(reqs) if ps.n <= CONFIG5_MAX_N]


def compute(name, threads=None):
    desc, sets = config_sets(name)
    t0 = time.perf_counter()
    dg = Digest()
    for i, ps in enumerate(sets):
        dg.add(*oracle_diagram(ps, threads))
        if len(sets) > 1 and (i + 1) % 256 == 0:
            print(f"  {name}: {i + 1}/{len(sets)} sets, {time.perf_counter() - t0:.0f} s",
                  flush=True)
    rec = {"workload": desc, "sets": len(sets), "sites": int(sum(s.n for s in sets))}
    rec.update(dg.result(per_set=len(sets) > 1))
    if name == "config5":
        rec["stream_index"] = [i for i, _ in config5_requests()]
    rec["oracle_seconds"] = round(time.perf_counter() - t0, 1)
    return rec


def main(argv):
    names = argv or ["config1", "config2", "config3", "config4", "config5", "config1_batch"]
    for name in names:
        print(f"{name} ...", flush=True)
        rec = compute(name)
        print(f"{name}: {rec['sha256']} ({rec['oracle_seconds']} s)", flush=True)
        store(name, rec)


def store(name, rec):
    """Merge one workload's record into the file (re-read first: runs may overlap)."""
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["note"] = ("SHA-256 of the canonical arrays (cell_off uint32, nbr int32, vtx 40-byte "
                    "pair-form vertices, del uint32 pairs; little-endian) of every cell, written "
                    "by oracle/golden_digests.py from the oracle's exact half-plane clipping "
                    "(definition of the Voronoi diagram, Section 2; representation of Section 6; "
                    "Delaunay graph of Section 7)")
    data.setdefault("configs", {})[name] = rec
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=1)
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
