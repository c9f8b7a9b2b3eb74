"""The stored full-size digests (tests/golden/fullsize_digests.json) and the canonical byte form
they hash (CPU only)."""
import json
import os

import numpy as np

import sitegen
from oracle import cdiagram, golden_digests

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_digests.json")


def test_every_config_is_stored():
    g = json.load(open(GOLD))["configs"]
    for name in ("config1", "config2", "config3", "config4", "config5", "config1_batch"):
        assert set(g[name]["sha256"]) == {"cell_off", "nbr", "vtx", "del"}, name
    assert g["config2"]["sites"] == g["config3"]["sites"] == 1 << 20
    assert g["config4"]["sets"] == 4096 and len(g["config4"]["per_set"]) == 4096
    assert g["config1_batch"]["sets"] == 4096 and g["config1_batch"]["sites"] == 4096000
    reqs = golden_digests.config5_requests()
    assert g["config5"]["sets"] == len(reqs) == len(g["config5"]["stream_index"])
    assert all(ps.n <= golden_digests.CONFIG5_MAX_N for _, ps in reqs)


def test_config1_digest_recomputed_from_the_oracle():
    rec = golden_digests.compute("config1")
    assert rec["sha256"] == json.load(open(GOLD))["configs"]["config1"]["sha256"]


def test_raw_vertex_words_equal_the_pair_form_integers():
    """The 40-byte canonical vertex (X low, X high, Y low, Y high, D) is the two's-complement
    split of the oracle's Python-integer vertices."""
    ps = sitegen.uniform(300, 1 << 24, seed=9)
    a = cdiagram.cells(ps.x, ps.y, ps.box, raw=True)
    b = cdiagram.cells(ps.x, ps.y, ps.box)
    w = a.vwords
    X = [int(np.int64(h)) * (1 << 64) + int(lo) for lo, h in zip(w[:, 0], w[:, 1].view(np.int64))]
    Y = [int(h) * (1 << 64) + int(lo) for lo, h in zip(w[:, 2], w[:, 3].view(np.int64))]
    assert X == list(b.vx) and Y == list(b.vy)
    assert np.array_equal(w[:, 4].view(np.int64), b.vd)


def test_digest_sees_a_single_changed_entry():
    ps = sitegen.uniform(200, 1 << 16, seed=3)
    off, nbr, vw, dele = golden_digests.oracle_diagram(ps)
    d0 = golden_digests.Digest()
    d0.add(off, nbr, vw, dele)
    nbr2 = nbr.copy()
    nbr2[17] ^= 1
    d1 = golden_digests.Digest()
    d1.add(off, nbr2, vw, dele)
    a, b = d0.result()["sha256"], d1.result()["sha256"]
    assert a["nbr"] != b["nbr"] and a["vtx"] == b["vtx"] and a["del"] == b["del"]
