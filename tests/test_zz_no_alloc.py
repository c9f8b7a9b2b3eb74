"""vor_compute_noalloc, the entry point that allocates nothing (its working memory is a fixed
device array of the library), against vor_compute on the same sets: identical offsets,
neighbour lists, pair-form vertices and Delaunay pairs, on consecutive calls of decreasing
size (the array keeps the previous call's contents), in both precisions, with device and host
inputs, for the box and a polygon X."""
import numpy as np
import pytest

import sitegen
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vor():
    import paper_1212_1095_amd as v
    return v


def run_noalloc(vor, ps, prec, device_in):
    import torch
    dev = torch.device("cuda:0")
    n = ps.n
    K = len(ps.region[0]) if ps.region is not None else 4
    cap, dcap = 6 * n + K + 16, 3 * n + 8
    # outputs prefilled with junk: everything read back must have been written by the call
    off = torch.full((n + 1,), -1, dtype=torch.int32, device=dev)
    nbr = torch.full((cap,), -77, dtype=torch.int32, device=dev)
    vtx = torch.full((cap * 5,), 12345, dtype=torch.int64, device=dev)
    dl = torch.full((2 * dcap,), -1, dtype=torch.int32, device=dev)
    if device_in:
        xd = torch.from_numpy(ps.x).to(dev)
        yd = torch.from_numpy(ps.y).to(dev)
        x, y = (xd.data_ptr(), n), (yd.data_ptr(), n)
    else:
        x, y = ps.x, ps.y
    torch.cuda.synchronize()
    E, m, st = vor.vor_compute_noalloc(x, y, ps.box, off.data_ptr(), nbr.data_ptr(),
                                       vtx.data_ptr(), cap, dl.data_ptr(), dcap, precision=prec,
                                       stream=torch.cuda.current_stream().cuda_stream,
                                       device_ptrs=device_in, region=ps.region)
    torch.cuda.synchronize()
    return (off.cpu().numpy().view(np.uint32), nbr[:E].cpu().numpy(),
            vtx[:5 * E].cpu().numpy().tobytes(), dl[:2 * m].cpu().numpy().view(np.uint32), st)


def reference(vor, ps, prec):
    with vor.Context(precision=prec) as ctx:
        return ctx.compute(ps.x, ps.y, ps.box, region=ps.region)


@pytest.mark.parametrize("prec", ["filtered", "exact"])
def test_noalloc_equals_compute_on_consecutive_calls(vor, prec):
    p = vor.VOR_FP32_FILTERED if prec == "filtered" else vor.VOR_EXACT_ONLY
    reg = sitegen.convex_polygon(12, 1 << 20, seed=9)
    sets = [("uniform 30000", sitegen.uniform(30000, 1 << 24, seed=61), True),
            ("clustered 3000", sitegen.clustered(3000, 1 << 24, seed=62), False),
            ("polygon 1500", sitegen.in_polygon(1500, reg, seed=63), True),
            ("uniform 200", sitegen.uniform(200, 1 << 16, seed=64), False)]
    for name, ps, device_in in sets:
        say(f"[{prec}] {name} (device input {device_in})")
        off, nbr, vtx, dl, st = run_noalloc(vor, ps, p, device_in)
        r = reference(vor, ps, p)
        assert np.array_equal(off, r.cell_off), name
        assert np.array_equal(nbr, r.nbr), name
        assert vtx == r.vtx.tobytes(), name
        assert np.array_equal(dl, r.dele.reshape(-1)), name
        assert st.edges == int(r.cell_off[-1])


def test_noalloc_rejects_what_it_cannot_hold(vor):
    import torch
    dev = torch.device("cuda:0")
    big = sitegen.uniform(vor.VOR_NOALLOC_MAX_SITES + 1, 1 << 24, seed=65)
    buf = torch.zeros(16, dtype=torch.int32, device=dev)
    with pytest.raises(vor.VorError) as e:
        vor.vor_compute_noalloc(big.x, big.y, big.box, buf.data_ptr(), buf.data_ptr(), 0,
                                1 << 30, buf.data_ptr(), 1 << 30)
    assert e.value.status == vor.VOR_E_INVAL
    ps = sitegen.uniform(100, 1 << 16, seed=66)
    with pytest.raises(vor.VorError):   # neighbour capacity below 6n + 4 + 16
        vor.vor_compute_noalloc(ps.x, ps.y, ps.box, buf.data_ptr(), buf.data_ptr(), 0,
                                6 * 100 + 19, buf.data_ptr(), 3 * 100 + 8)
