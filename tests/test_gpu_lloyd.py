"""Lloyd iterations on the device (vor_lloyd) against the oracle's step definition
(oracle/lloyd.py): identical sites after every step and identical moved counts, for boxes and
polygons, uniform and clustered sets, both precisions, and a dense set where the collision rule
sends a site back."""
import numpy as np
import pytest

import sitegen
from oracle import lloyd as olloyd
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


@pytest.fixture(scope="module", params=["filtered", "exact"])
def ctx(request, vor):
    prec = vor.VOR_FP32_FILTERED if request.param == "filtered" else vor.VOR_EXACT_ONLY
    c = vor.Context(device=0, precision=prec)
    c.mode = request.param
    yield c
    c.close()


def sets():
    yield "uniform box", sitegen.uniform(3000, 1 << 16, seed=21)
    yield "clustered box", sitegen.clustered(6000, 1 << 20, seed=22)
    reg = sitegen.convex_polygon(9, 1 << 18, seed=23)
    yield "polygon", sitegen.in_polygon(2500, reg, seed=24)
    yield "dense", sitegen.uniform(300, 40, seed=3)
    yield "collision", sitegen.small_integer_set(18, 11, seed=30)
    yield "fast path", sitegen.uniform(20000, 1 << 20, seed=25)


@pytest.mark.parametrize("name", [n for n, _ in sets()])
def test_lloyd_matches_oracle(ctx, name):
    ps = dict(sets())[name]
    iters = 3
    say(f"[{ctx.mode}] lloyd {name}: n={ps.n} iters={iters}")
    gx, gy, gm = ctx.lloyd(ps.x, ps.y, ps.box, iters, region=ps.region)
    ox, oy, om = olloyd.iterate(ps.x, ps.y, ps.box, iters, region=ps.region)
    assert gm == om
    assert np.array_equal(gx, ox) and np.array_equal(gy, oy)


def test_lloyd_errors(vor):
    with vor.Context(device=0) as c:
        x = np.array([5, 5], np.int32)
        y = np.array([5, 5], np.int32)
        with pytest.raises(vor.VorError) as e:
            c.lloyd(x, y, (0, 0, 10, 10), 2)
        assert e.value.status == vor.VOR_E_DUPLICATE
