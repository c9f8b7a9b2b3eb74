"""Parity at the full workload sizes, in the launch configuration the benchmark times:
sampled cells against the oracle (one by one) plus properties that hold at any size."""
import numpy as np
import pytest

import sitegen
from oracle import cdiagram
from tests.gpu_util import assert_matches_oracle, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


def check_symmetric(r):
    n = r.n
    k = np.repeat(np.arange(n, dtype=np.int64), np.diff(r.cell_off.astype(np.int64)))
    j = r.nbr.astype(np.int64)
    s = j >= 0
    a = np.unique(k[s] * n + j[s])
    b = np.unique(j[s] * n + k[s])
    assert a.shape == b.shape and np.array_equal(a, b), "neighbour lists not symmetric"
    # the Delaunay list is exactly the neighbour pairs with i < j, sorted
    kk, jj = k[s], j[s]
    m = jj > kk
    pairs = np.stack([kk[m], jj[m]], 1)
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
    assert np.array_equal(r.dele.astype(np.int64), pairs)


def sample_check(r, ps, m=1500, seed=0):
    rng = np.random.default_rng(seed)
    which = np.sort(rng.choice(ps.n, size=min(m, ps.n), replace=False)).astype(np.int32)
    assert_matches_oracle(r, ps, which=which)


@pytest.mark.parametrize("name", ["config2_uniform", "config3_clustered"])
def test_large_single_set(vor, name):
    n = 1 << 20
    if name == "config2_uniform":
        ps = sitegen.uniform(n, 1 << 24, seed=2)
    else:
        ps = sitegen.clustered(n, 1 << 24, seed=3)
    say(f"{name}: n={ps.n}")
    with vor.Context(flags=vor.VOR_CHECK_SYMMETRY) as ctx:
        r = ctx.compute(ps.x, ps.y, ps.box)
    say(f"  device {r.device_ms:.2f} ms, deferred {r.stats.deferred_cells}, "
        f"exact {r.stats.exact_decisions}, asym {r.stats.asym_pairs}")
    assert r.stats.asym_pairs == 0
    E = int(r.cell_off[-1])
    assert E <= 10 * ps.n and r.stats.edges == E
    assert r.stats.rays <= 11 * ps.n + 64 * r.stats.deferred_cells
    check_symmetric(r)
    sample_check(r, ps)


def test_config4_batch_full(vor):
    """4096 sets, sizes log-uniform in [32, 65536], uniform in [1, 2^20)^2."""
    sets = sitegen.batch_sets(4096, 4, B=1 << 20, lo=32, hi=65536)
    say(f"config4: {len(sets)} sets, {sum(s.n for s in sets)} sites")
    with vor.Context(flags=vor.VOR_NO_VERTICES) as ctx:
        rc, res = ctx.compute_batch([(s.x, s.y, s.box) for s in sets])
    assert rc == vor.VOR_OK
    rng = np.random.default_rng(4)
    for i in rng.choice(len(sets), size=24, replace=False):
        s, r = sets[int(i)], res[int(i)]
        if s.n <= 4000:
            assert_matches_oracle(r, s, vertices=False)
        else:
            sample_check(r, s, m=300, seed=int(i))
    for r in res[::64]:
        check_symmetric(r)


def test_config5_request_sample(vor):
    """A served stream of the config-5 mix (uniform / clustered / lattice, up to 2^20 sites);
    every request is compared on sampled cells, and small ones in full."""
    reqs = sitegen.request_stream(12, 100.0, seed=5)
    with vor.Context(flags=vor.VOR_NO_VERTICES) as ctx:
        tickets = [ctx.submit(r.x, r.y, r.box) for _, r in reqs]
        out = {}
        import time
        t0 = time.time()
        while len(out) < len(tickets):
            for t in tickets:
                if t not in out:
                    st, res = ctx.poll(t)
                    if st != vor.VOR_PENDING:
                        out[t] = (st, res)
            assert time.time() - t0 < 240
            time.sleep(0.002)
    for (t, (_, ps)) in zip(tickets, reqs):
        st, r = out[t]
        say(f"  request n={ps.n} kind={ps.kind} status={st}")
        assert st == vor.VOR_OK
        check_symmetric(r)
        if ps.n <= 3000:
            assert_matches_oracle(r, ps, vertices=False)
        else:
            sample_check(r, ps, m=200, seed=ps.n)


# ------------------------------------------------------------------ every cell, by digest
# tests/golden/fullsize_digests.json holds SHA-256 digests of the oracle's canonical arrays for
# every cell of each workload (written by oracle/golden_digests.py from the oracle alone).  The
# GPU's arrays are hashed the same way; a mismatch is then localised with the oracle itself.
import json  # noqa: E402
import os  # noqa: E402

from oracle import golden_digests  # noqa: E402

_GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "fullsize_digests.json")
PRECISIONS = ["filtered", "exact"]


def golden(name):
    with open(_GOLD_PATH) as f:
        return json.load(f)["configs"][name]


def vwords(r):
    return np.frombuffer(r.vtx.tobytes(), dtype="<u8").reshape(-1, 5)


def gpu_digest(results):
    dg = golden_digests.Digest()
    for r in results:
        dg.add(r.cell_off, r.nbr, vwords(r), r.dele)
    return dg


def bench_tuning(n, dist):
    """The tuning bench.py applies to this workload (the autotuner's table), or None."""
    from paper_1212_1095_amd import autotune
    return autotune.best_params(n, dist)


def precision_of(vor, name):
    return vor.VOR_FP32_FILTERED if name == "filtered" else vor.VOR_EXACT_ONLY


def explain_mismatch(results, sets, gold, got):
    """First differing set (by the per-set digests), checked against the oracle for a message."""
    per = gold.get("per_set")
    idx = 0
    if per is not None:
        diff = [i for i, (a, b) in enumerate(zip(per, got.per)) if a != b]
        idx = diff[0] if diff else 0
        say(f"  {len(diff)} of {len(per)} sets differ, first {diff[:8]}")
    r, ps = results[idx], sets[idx]
    if ps.n <= 5000:
        assert_matches_oracle(r, ps)
    else:
        sample_check(r, ps, m=3000, seed=7)
    raise AssertionError(f"digests differ (set {idx}) but the sampled cells match the oracle")


def check_digests(results, sets, name):
    gold = golden(name)
    assert gold["sets"] == len(sets) and gold["sites"] == sum(s.n for s in sets)
    got = gpu_digest(results)
    res = got.result()["sha256"]
    if res != gold["sha256"]:
        say(f"  {name}: digests {res} != {gold['sha256']}")
        explain_mismatch(results, sets, gold, got)


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("name", ["config1", "config2", "config3"])
def test_every_cell_single_set(vor, name, prec):
    """Configs 1-3, every cell: neighbour lists, vertices and Delaunay edges byte for byte."""
    _, sets = golden_digests.config_sets(name)
    ps = sets[0]
    dist = "clustered" if name == "config3" else "uniform"
    say(f"{name} {prec}: n={ps.n}")
    with vor.Context(precision=precision_of(vor, prec)) as ctx:
        t = bench_tuning(ps.n, dist) if prec == "filtered" else None
        if t is not None:
            ctx.tune(*t)
        r = ctx.compute(ps.x, ps.y, ps.box)
    say(f"  device {r.device_ms:.2f} ms, exact decisions {r.stats.exact_decisions}")
    check_digests([r], [ps], name)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_every_cell_config4_batch(vor, prec):
    """Config 4, all 4096 sets in one batched call, every cell with vertices."""
    _, sets = golden_digests.config_sets("config4")
    say(f"config4 {prec}: {len(sets)} sets, {sum(s.n for s in sets)} sites")
    with vor.Context(precision=precision_of(vor, prec)) as ctx:
        rc, res = ctx.compute_batch([(s.x, s.y, s.box) for s in sets])
    assert rc == vor.VOR_OK
    say(f"  device {res[0].device_ms:.1f} ms")
    check_digests(res, sets, "config4")


@pytest.mark.parametrize("prec", PRECISIONS)
def test_every_cell_config5_requests(vor, prec):
    """Config 5: the requests with n <= 2^16 of the 200-request stream, submitted in stream
    order to the request loop (continuous batching), every cell with vertices."""
    import time
    reqs = golden_digests.config5_requests()
    sets = [ps for _, ps in reqs]
    say(f"config5 {prec}: {len(sets)} requests, {sum(s.n for s in sets)} sites")
    with vor.Context(precision=precision_of(vor, prec)) as ctx:
        tickets = [ctx.submit(ps.x, ps.y, ps.box) for ps in sets]
        out = {}
        t0 = time.time()
        while len(out) < len(tickets):
            for t in tickets:
                if t not in out:
                    st, r = ctx.poll(t)
                    if st != vor.VOR_PENDING:
                        assert st == vor.VOR_OK, st
                        out[t] = r
            assert time.time() - t0 < 100
            time.sleep(0.001)
    check_digests([out[t] for t in tickets], sets, "config5")
