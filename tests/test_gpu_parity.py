"""Parity of the HIP path with the oracle (element by element), through the C ABI."""
import numpy as np
import pytest

import sitegen
from oracle import cdiagram, paper_forms
from tests.gpu_util import assert_matches_oracle, say, symmetric

pytestmark = pytest.mark.gpu

MODES = ["filtered", "exact"]


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


@pytest.fixture(scope="module", params=MODES)
def ctx(request, vor):
    prec = vor.VOR_FP32_FILTERED if request.param == "filtered" else vor.VOR_EXACT_ONLY
    c = vor.Context(device=0, precision=prec)
    c.mode = request.param
    yield c
    c.close()


def run(ctx, ps, name):
    say(f"[{ctx.mode}] {name}: n={ps.n} box={ps.box}")
    return ctx.compute(ps.x, ps.y, ps.box)


@pytest.mark.parametrize("seed", range(40))
def test_tiny_tie_heavy_sets(ctx, seed):
    n = 1 + seed % 8
    ps = sitegen.small_integer_set(n, 3 + seed % 6, seed=5000 + seed)
    r = run(ctx, ps, f"tiny seed={seed}")
    assert_matches_oracle(r, ps)


def test_single_site(ctx):
    ps = sitegen.PointSet(np.array([3], np.int32), np.array([5], np.int32), (0, 0, 10, 10))
    r = run(ctx, ps, "single site")
    assert r.lines(0) == [-4, -1, -2, -3]
    assert_matches_oracle(r, ps)


def test_two_sites(ctx):
    ps = sitegen.PointSet(np.array([2, 8], np.int32), np.array([5, 5], np.int32), (0, 0, 10, 10))
    assert_matches_oracle(run(ctx, ps, "two sites"), ps)


def test_collinear_row(ctx):
    xs = np.array([3, 7, 15, 16, 30, 31, 33], np.int32)
    ps = sitegen.PointSet(xs, np.full(xs.shape, 20, np.int32), (0, 0, 40, 40))
    assert_matches_oracle(run(ctx, ps, "collinear row"), ps)


def test_collinear_column_and_diagonal(ctx):
    ys = np.array([1, 5, 6, 20, 38], np.int32)
    ps = sitegen.PointSet(np.full(ys.shape, 11, np.int32), ys, (0, 0, 40, 40))
    assert_matches_oracle(run(ctx, ps, "collinear column"), ps)
    d = np.array([2, 5, 9, 14, 30], np.int32)
    ps = sitegen.PointSet(d, d, (0, 0, 40, 40))
    assert_matches_oracle(run(ctx, ps, "diagonal"), ps)


def test_twelve_cocircular(ctx):
    offs = [(3, 4), (4, 3), (5, 0), (4, -3), (3, -4), (0, -5), (-3, -4), (-4, -3), (-5, 0),
            (-4, 3), (-3, 4), (0, 5)]
    x = np.array([50 + a for a, _ in offs], np.int32)
    y = np.array([50 + b for _, b in offs], np.int32)
    ps = sitegen.PointSet(x, y, (0, 0, 100, 100))
    r = run(ctx, ps, "12 cocircular")
    assert_matches_oracle(r, ps)
    assert r.dele.shape[0] == 12


@pytest.mark.parametrize("ring", [40, 300, 3000])
def test_hub_cell_with_many_edges(ctx, ring):
    """A site at the centre of `ring` sites on a circle: its cell has one edge per ring site.
    40 edges exceed the filtered pass's 24 line slots (the cell moves to the exact pass and its
    lines to the overflow pool), 300 exceed the exact pass's 128 (deep pass), 3000 exceed the
    2048 entries that the output kernel stages per block of 256 cells."""
    R, c = 1 << 20, 1 << 21
    ang = 2 * np.pi * (np.arange(ring) + 0.25) / ring
    x = np.concatenate([[c], np.rint(c + R * np.cos(ang))]).astype(np.int32)
    y = np.concatenate([[c], np.rint(c + R * np.sin(ang))]).astype(np.int32)
    order = np.random.default_rng(ring).permutation(ring + 1)   # the hub at a random id
    ps = sitegen.PointSet(x[order], y[order], (0, 0, 1 << 22, 1 << 22))
    r = run(ctx, ps, f"hub with {ring} ring sites")
    hub = int(np.flatnonzero(order == 0)[0])
    assert len(r.lines(hub)) == ring
    assert_matches_oracle(r, ps)
    assert symmetric(r)


@pytest.mark.parametrize("name", ["jittered lattice", "dense small box", "perfect lattice"])
def test_near_ties_in_the_filtered_pass(ctx, name):
    """Sets above the small-set threshold (the one-lane-per-cell pass runs) full of near-ties
    and exact ties: the FP32 filter leaves rays undecided and those cells reach the exact pass."""
    if name == "jittered lattice":
        ps = sitegen.lattice(30000, 176 * 1024, seed=44)   # the lattice fills the box
    elif name == "dense small box":
        ps = sitegen.uniform(30000, 1 << 9, seed=45)
    else:
        k, h = 180, 256
        ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
        ps = sitegen.PointSet((h // 2 + h * ii.ravel()).astype(np.int32),
                              (h // 2 + h * jj.ravel()).astype(np.int32), (0, 0, k * h, k * h))
    r = run(ctx, ps, f"{name} n={ps.n}")
    assert_matches_oracle(r, ps)
    assert symmetric(r)
    if ctx.mode == "filtered":
        assert r.stats.deferred_cells > 0


@pytest.mark.parametrize("k", [1, 2, 7, 16])
def test_perfect_lattice(ctx, k):
    h = 64
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    x = (h // 2 + h * ii.ravel()).astype(np.int32)
    y = (h // 2 + h * jj.ravel()).astype(np.int32)
    ps = sitegen.PointSet(x, y, (0, 0, k * h, k * h))
    r = run(ctx, ps, f"lattice {k}x{k}")
    assert_matches_oracle(r, ps)
    assert r.dele.shape[0] == 2 * k * (k - 1)


def test_config1_uniform_1000(ctx):
    """n = 1000 uniform in [1, 2^16)^2, X = [0, 2^16]^2, seed 1."""
    ps = sitegen.uniform(1000, 1 << 16, seed=1)
    r = run(ctx, ps, "config1")
    assert_matches_oracle(r, ps)


@pytest.mark.parametrize("gen,n", [("uniform", 20000), ("clustered", 20000),
                                   ("lattice", 20000)])
def test_moderate_full(ctx, gen, n):
    if gen == "uniform":
        ps = sitegen.uniform(n, 1 << 20, seed=41)
    elif gen == "clustered":
        ps = sitegen.clustered(n, 1 << 24, seed=42)
    else:
        ps = sitegen.lattice(n, 1 << 24, seed=43)
    r = run(ctx, ps, f"{gen} {n}")
    assert_matches_oracle(r, ps)


def test_small_box_dense(ctx):
    """Many sites in a small box: most coordinates collide with cocircular quadruples."""
    ps = sitegen.small_integer_set(600, 40, seed=77)
    r = run(ctx, ps, "dense small box")
    assert_matches_oracle(r, ps)


def test_negative_box_origin(ctx):
    ps = sitegen.uniform(3000, 1 << 18, seed=9)
    x = ps.x - (1 << 17) - 12345
    y = ps.y - 77777
    box = (-(1 << 17) - 12345, -77777, (1 << 18) - (1 << 17) - 12345, (1 << 18) - 77777)
    ps2 = sitegen.PointSet(x.astype(np.int32), y.astype(np.int32), box)
    assert_matches_oracle(run(ctx, ps2, "negative origin"), ps2)


def test_paper_counter_bounds(ctx):
    """Lemma on shot rays: sum rho_k <= (|X_e| + 7) n = 11 n; nodes <= 2 e_k per cell summed;
    sum e_k <= 10 n (rectangle X)."""
    ps = sitegen.uniform(50000, 1 << 24, seed=2)
    r = run(ctx, ps, "counters")
    E = int(r.cell_off[-1])
    assert E <= 10 * ps.n
    assert r.stats.edges == E
    # counters include the abandoned attempt of each cell that was deferred to the exact pass
    # or handed to the adaptive pass
    slack = 64 * (r.stats.deferred_cells + r.stats.adaptive_cells)
    assert r.stats.rays <= 11 * ps.n + slack
    assert r.stats.nodes <= 2 * E + slack
    # the projector confirms each vertex of a cell once: one test per stored vertex
    assert r.stats.vertex_tests <= E + slack
    say(f"  rays/cell={r.stats.rays / ps.n:.3f} nodes/cell={r.stats.nodes / ps.n:.3f} "
        f"evals/cell={r.stats.evals / ps.n:.1f} exact={r.stats.exact_decisions} "
        f"deferred={r.stats.deferred_cells}")


def test_input_error_on_the_first_call(vor):
    """A fresh context whose first call has a site outside X: the grid is built, the
    refinement is skipped because the error is already flagged, and no later kernel may walk the
    unwritten refinement slots; the call reports VOR_E_DOMAIN and the next call is exact."""
    for box, x, y in [((0, 0, 100, 100), [-1, 5, 7], [6, 7, 8]),
                      ((0, 0, 1 << 20, 1 << 20), [3, (1 << 20) + 1, 9], [4, 5, 1 << 19])]:
        with vor.Context(device=0) as c:
            say(f"first call with a site outside {box}")
            with pytest.raises(vor.VorError) as e:
                c.compute(np.array(x, np.int32), np.array(y, np.int32), box)
            assert e.value.status == vor.VOR_E_DOMAIN
            ps = sitegen.clustered(3000, 1 << 20, seed=5)
            assert_matches_oracle(c.compute(ps.x, ps.y, ps.box), ps)


def test_errors(vor):
    with vor.Context() as c:
        box = (0, 0, 100, 100)
        for x, y, code in [([5, 5], [6, 6], vor.VOR_E_DUPLICATE),
                           ([-1, 5], [6, 7], vor.VOR_E_DOMAIN),
                           ([101, 5], [6, 7], vor.VOR_E_DOMAIN),
                           ([5, 50], [6, 101], vor.VOR_E_DOMAIN)]:
            say(f"error case {x} {y}")
            with pytest.raises(vor.VorError) as e:
                c.compute(np.array(x, np.int32), np.array(y, np.int32), box)
            assert e.value.status == code
        with pytest.raises(vor.VorError) as e:
            c.compute(np.array([], np.int32), np.array([], np.int32), box)
        assert e.value.status == vor.VOR_E_INVAL
        with pytest.raises(vor.VorError) as e:
            c.compute(np.array([1], np.int32), np.array([1], np.int32), (0, 0, 1 << 25, 10))
        assert e.value.status == vor.VOR_E_DOMAIN
        # the context still works after errors
        ps = sitegen.uniform(100, 1 << 10, seed=3)
        assert_matches_oracle(c.compute(ps.x, ps.y, ps.box), ps)


def test_site_limit_per_run(vor):
    """Entry offsets are 32-bit: a batch whose sets hold more than 2^27 sites together is
    refused with VOR_E_NOMEM before any device work (the sets here share one host array, which
    is never read), and the context still works afterwards."""
    n = 1 << 21
    x = np.arange(1, n + 1, dtype=np.int32)
    box = (0, 0, 1 << 24, 1 << 24)
    with vor.Context() as c:
        say("batch of 65 sets of 2^21 sites (2^27 + 2^21 in all)")
        with pytest.raises(vor.VorError) as e:
            c.compute_batch([(x, x, box)] * 65)
        assert e.value.status == vor.VOR_E_NOMEM
        ps = sitegen.uniform(500, 1 << 12, seed=4)
        rc, res = c.compute_batch([(ps.x, ps.y, ps.box)] * 2)
        assert rc == vor.VOR_OK
        for r in res:
            assert_matches_oracle(r, ps)
