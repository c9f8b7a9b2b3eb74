"""Batched sets in one launch and the continuous-batching request loop, through the C ABI."""
import time

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


def same(a, b):
    assert np.array_equal(a.cell_off, b.cell_off)
    assert np.array_equal(a.nbr, b.nbr)
    assert np.array_equal(a.dele, b.dele)
    if a.vtx is not None or b.vtx is not None:
        assert a.vtx.tobytes() == b.vtx.tobytes()


def uneven_sets(k, seed, lo=32, hi=4096):
    sizes = sitegen.batch_sizes(k, seed, lo, hi)
    return sitegen.batch_sets(k, seed, B=1 << 20, lo=lo, hi=hi, sizes=sizes)


def test_batch_matches_oracle_and_single(vor):
    sets = uneven_sets(48, seed=4)
    say(f"batch of {len(sets)} sets, total {sum(s.n for s in sets)} sites")
    with vor.Context() as ctx:
        rc, res = ctx.compute_batch([(s.x, s.y, s.box) for s in sets])
        assert rc == vor.VOR_OK
        for s, r in zip(sets, res):
            assert r.status == vor.VOR_OK
            assert_matches_oracle(r, s)
        for s, r in zip(sets[:8], res[:8]):
            same(r, ctx.compute(s.x, s.y, s.box))


def test_batch_mixed_boxes_and_distributions(vor):
    sets = [sitegen.uniform(700, 1 << 16, 11), sitegen.clustered(900, 1 << 24, 12),
            sitegen.lattice(400, 1 << 24, 13), sitegen.small_integer_set(60, 12, 14),
            sitegen.uniform(1, 1 << 10, 15)]
    with vor.Context() as ctx:
        rc, res = ctx.compute_batch([(s.x, s.y, s.box) for s in sets])
        assert rc == vor.VOR_OK
        for s, r in zip(sets, res):
            assert_matches_oracle(r, s)


def test_batch_with_a_bad_set(vor):
    good = sitegen.uniform(300, 1 << 12, 21)
    bad_x = np.array([5, 5, 9], np.int32)
    bad_y = np.array([6, 6, 9], np.int32)
    with vor.Context() as ctx:
        rc, res = ctx.compute_batch([(good.x, good.y, good.box), (bad_x, bad_y, (0, 0, 20, 20)),
                                     (good.x, good.y, good.box)])
        assert rc == vor.VOR_E_DUPLICATE
        assert res[1].status == vor.VOR_E_DUPLICATE
        assert res[0].status == vor.VOR_OK and res[2].status == vor.VOR_OK
        assert_matches_oracle(res[0], good)
        same(res[0], res[2])


def test_batch_repeated_calls_replay(vor):
    """A new shape launches kernel by kernel; the same shape again is captured as a graph and
    replayed from then on; the results of all three calls are identical."""
    sets = uneven_sets(16, seed=5, hi=2048)
    args = [(s.x, s.y, s.box) for s in sets]
    with vor.Context() as ctx:
        _, r1 = ctx.compute_batch(args)
        _, r2 = ctx.compute_batch(args)
        _, r3 = ctx.compute_batch(args)
        for a, b, c in zip(r1, r2, r3):
            same(a, b)
            same(a, c)
        assert r1[0].graph_replayed == 0
        assert r2[0].graph_replayed == 1 and r3[0].graph_replayed == 1


def wait_all(ctx, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            st, r = ctx.poll(t)
            if st != 1:   # VOR_PENDING
                out[t] = (st, r)
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return out


def test_serving_results_identical_alone_and_in_mix(vor):
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(24):
        kind = i % 4
        n = int(rng.integers(100, 6000))
        if kind == 0:
            reqs.append(sitegen.uniform(n, 1 << 24, 100 + i))
        elif kind == 1:
            reqs.append(sitegen.clustered(n, 1 << 24, 100 + i))
        elif kind == 2:
            reqs.append(sitegen.lattice(n, 1 << 24, 100 + i))
        else:
            reqs.append(sitegen.uniform(n, 1 << 16, 100 + i))
    with vor.Context() as ctx:
        tickets = [ctx.submit(r.x, r.y, r.box) for r in reqs]
        say(f"submitted {len(tickets)} requests")
        done = wait_all(ctx, tickets)
        for t, r in zip(tickets, reqs):
            st, res = done[t]
            assert st == vor.VOR_OK, (t, st)
            assert 0 < res.t_submit <= res.t_admit <= res.t_done
            alone = ctx.compute(r.x, r.y, r.box)
            same(res, alone)
        for r, t in list(zip(reqs, tickets))[:6]:
            assert_matches_oracle(done[t][1], r)
        # a consumed ticket
        st, _ = ctx.poll(tickets[0])
        assert st == vor.VOR_E_TICKET
        st, _ = ctx.poll(123456789)
        assert st == vor.VOR_E_TICKET


def test_serving_bad_request_and_budget(vor):
    good = sitegen.uniform(2000, 1 << 20, 31)
    # a budget that holds one such request at a time: admission queues, never fails
    with vor.Context(hbm_budget_bytes=4 << 20) as ctx:
        tickets = [ctx.submit(good.x, good.y, good.box) for _ in range(5)]
        bad = ctx.submit(np.array([1, 1], np.int32), np.array([2, 2], np.int32), (0, 0, 8, 8))
        done = wait_all(ctx, tickets + [bad])
        ref = None
        for t in tickets:
            st, r = done[t]
            assert st == vor.VOR_OK
            if ref is None:
                ref = r
                assert_matches_oracle(r, good)
            else:
                same(r, ref)
        assert done[bad][0] == vor.VOR_E_DUPLICATE
        big = sitegen.uniform(60000, 1 << 24, 32)
        t = ctx.submit(big.x, big.y, big.box)
        st, _ = wait_all(ctx, [t])[t]
        assert st == vor.VOR_E_NOMEM


def test_destroy_with_pending_requests(vor):
    ctx = vor.Context()
    ps = sitegen.uniform(20000, 1 << 24, 41)
    for _ in range(4):
        ctx.submit(ps.x, ps.y, ps.box)
    ctx.close()   # cancels pending requests, joins the loop, frees results


def test_consumed_tickets_leave_nothing_behind(vor):
    """A served request is forgotten once polled: the context's ticket map stays bounded."""
    sets = [sitegen.uniform(300 + 7 * i, 1 << 20, 500 + i) for i in range(60)]
    with vor.Context(flags=vor.VOR_NO_VERTICES) as ctx:
        for rnd in range(4):
            tickets = [ctx.submit(s.x, s.y, s.box) for s in sets]
            assert ctx.ticket_count() == len(sets)
            done = wait_all(ctx, tickets)
            assert all(st == vor.VOR_OK for st, _ in done.values())
            assert ctx.ticket_count() == 0, rnd
        with pytest.raises(vor.VorError):
            ctx.times(tickets[0])
        st, _ = ctx.poll(tickets[0])
        assert st == vor.VOR_E_TICKET


def test_admission_keeps_the_budget_across_workspaces(vor):
    """Two requests, each larger than half the budget: the second is admitted only after the
    first is done, although a second workspace is free."""
    a = sitegen.uniform(200000, 1 << 24, 41)
    b = sitegen.uniform(180000, 1 << 24, 42)
    with vor.Context() as c0:
        fa, fb = c0.footprint(a.x, a.y, a.box), c0.footprint(b.x, b.y, b.box)
    budget = int(1.5 * max(fa, fb))
    assert fa > budget // 2 and fb > budget // 2 and fa + fb > budget
    with vor.Context(hbm_budget_bytes=budget) as ctx:
        ta = ctx.submit(a.x, a.y, a.box)
        tb = ctx.submit(b.x, b.y, b.box)
        done = wait_all(ctx, [ta, tb])
    (sa, ra), (sb, rb) = done[ta], done[tb]
    assert sa == vor.VOR_OK and sb == vor.VOR_OK
    say(f"a: admit {ra.t_admit:.4f} done {ra.t_done:.4f}; b: admit {rb.t_admit:.4f}")
    assert rb.t_admit >= ra.t_done


def test_size_tuning_changes_no_result(vor):
    """Per-set grid parameters by size class (vor_set_size_tuning) change speed only: a batch of
    sets of several sizes gives the same bytes with two different tables and with none."""
    sizes = [40, 300, 1000, 5000, 20000, 70]
    sets = [sitegen.uniform(n, 1 << 20, 900 + i) for i, n in enumerate(sizes)]
    args = [(s.x, s.y, s.box) for s in sets]
    out = []
    tables = [[], [(6, 0.7, 1, 0), (10, 2.0, 2, 0), (14, 1.0, 3, 1)],
              [(5, 3.0, 1, 2), (12, 0.5, 2, 0)]]
    with vor.Context() as ctx:
        for t in tables:
            ctx.size_tuning(t)
            rc, res = ctx.compute_batch(args)
            assert rc == vor.VOR_OK
            out.append(res)
        with pytest.raises(vor.VorError):
            ctx.size_tuning([(5, 100.0, 1, 0)])   # sites per bucket out of range
    for res in out[1:]:
        for a, b in zip(out[0], res):
            same(a, b)
    assert_matches_oracle(out[1][3], sets[3])


def snapshot(r):
    """Copies of a result's arrays (which view library memory)."""
    return (r.cell_off.copy(), r.nbr.copy(), None if r.vtx is None else r.vtx.copy(),
            r.dele.copy())


def unchanged(r, snap):
    off, nbr, vtx, dele = snap
    assert np.array_equal(r.cell_off, off) and np.array_equal(r.nbr, nbr)
    assert np.array_equal(r.dele, dele)
    assert (vtx is None) == (r.vtx is None)
    if vtx is not None:
        assert r.vtx.tobytes() == vtx.tobytes()


def test_held_results_survive_later_calls_and_the_context(vor):
    """Results point into pooled host blocks: a block still held by results is never handed to
    a later run, and results outlive the context that made them."""
    a_sets = uneven_sets(24, seed=31, hi=3000)
    b_sets = uneven_sets(24, seed=32, hi=3000)
    ctx = vor.Context()
    _, ra = ctx.compute_batch([(s.x, s.y, s.box) for s in a_sets])
    snaps = [snapshot(r) for r in ra]
    one = ctx.compute(a_sets[0].x, a_sets[0].y, a_sets[0].box)
    one_snap = snapshot(one)
    for _ in range(3):   # later runs of other shapes and of the same shape, results dropped
        ctx.compute_batch([(s.x, s.y, s.box) for s in b_sets])
        ctx.compute_batch([(s.x, s.y, s.box) for s in a_sets])
        ctx.compute(b_sets[1].x, b_sets[1].y, b_sets[1].box)
    for r, sn in zip(ra, snaps):
        unchanged(r, sn)
    unchanged(one, one_snap)
    ctx.close()
    for r, sn in zip(ra, snaps):   # after the context is gone
        unchanged(r, sn)
    for s, r in zip(a_sets[:4], ra[:4]):
        assert_matches_oracle(r, s)
    del ra, one


def test_held_request_results_survive_later_requests(vor):
    """The request loop's results stay intact while later batches run."""
    sets = [sitegen.uniform(n, 1 << 20, 40 + i) for i, n in enumerate((500, 2000, 800, 5000))]
    with vor.Context() as ctx:
        first = wait_all(ctx, [ctx.submit(s.x, s.y, s.box) for s in sets])
        held = [first[t][1] for t in sorted(first)]
        snaps = [snapshot(r) for r in held]
        for _ in range(3):
            wait_all(ctx, [ctx.submit(s.x, s.y, s.box) for s in reversed(sets)])
        for r, sn in zip(held, snaps):
            unchanged(r, sn)
        for s, r in zip(sets, held):
            assert_matches_oracle(r, s)
