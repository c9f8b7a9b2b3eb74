"""ctypes binding of include/vor.h.  Argument marshalling only: every step of the path runs in
the HIP library."""
from __future__ import annotations

import ctypes as C
import gc
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libvor.so")

VOR_OK, VOR_PENDING = 0, 1
VOR_E_INVAL, VOR_E_DOMAIN, VOR_E_DUPLICATE, VOR_E_NOMEM = -1, -2, -3, -4
VOR_E_DEVICE, VOR_E_TICKET, VOR_E_CAPACITY = -5, -6, -7
VOR_SET_DEVICE, VOR_RESULT_DEVICE, VOR_NO_VERTICES, VOR_CHECK_SYMMETRY = 0x1, 0x2, 0x4, 0x8
VOR_TIME_KERNELS = 0x10
VOR_PATH_GRID_FIRST, VOR_PATH_TREE = 0, 1
VOR_EXACT_ONLY, VOR_FP32_FILTERED = 0, 1


class vor_box(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32)]


class vor_set(C.Structure):
    _fields_ = [("n", C.c_uint32), ("x", C.c_void_p), ("y", C.c_void_p), ("box", vor_box),
                ("flags", C.c_uint32), ("nregion", C.c_uint32), ("region_x", C.c_void_p),
                ("region_y", C.c_void_p)]


class vor_opts(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget_bytes", C.c_uint64), ("precision", C.c_int32),
                ("flags", C.c_uint32)]


class vor_rat(C.Structure):
    _fields_ = [("x_lo", C.c_uint64), ("x_hi", C.c_int64), ("y_lo", C.c_uint64),
                ("y_hi", C.c_int64), ("d", C.c_int64)]


class vor_stats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("rays", "nodes", "evals", "exact_decisions",
                                           "deferred_cells", "asym_pairs", "shells", "edges",
                                           "vertex_tests", "adaptive_cells",
                                           "adaptive_evals", "fallback_cmp",
                                           "fallback_incircle", "vertex_rays")]


class vor_result(C.Structure):
    _fields_ = [("n", C.c_uint32), ("cell_off", C.c_void_p), ("nbr", C.c_void_p),
                ("vtx", C.c_void_p), ("m", C.c_uint64), ("del_", C.c_void_p),
                ("stats", vor_stats), ("device_ms", C.c_float), ("cells_ms", C.c_float),
                ("exact_ms", C.c_float), ("grid_ms", C.c_float), ("emit_ms", C.c_float),
                ("graph_replayed", C.c_int32), ("status", C.c_int32),
                ("adaptive_ms", C.c_float), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


class vor_size_tuning(C.Structure):
    _fields_ = [("log2n", C.c_int32), ("sites_per_bucket", C.c_float),
                ("block_halfwidth", C.c_int32), ("leaf_halfwidth", C.c_int32)]


class vor_tuning(C.Structure):
    _fields_ = [("sites_per_bucket", C.c_float), ("block", C.c_int32),
                ("block_halfwidth", C.c_int32), ("leaf_halfwidth", C.c_int32),
                ("scan_path", C.c_int32)]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libvor.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is not built: run __graft_entry__.build()")
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        L.vor_create.argtypes = [P(vor_opts), P(C.c_void_p)]
        L.vor_destroy.argtypes = [C.c_void_p]
        L.vor_compute.argtypes = [C.c_void_p, P(vor_set), P(P(vor_result))]
        L.vor_compute_batch.argtypes = [C.c_void_p, P(vor_set), C.c_uint32, P(P(vor_result))]
        L.vor_submit.argtypes = [C.c_void_p, P(vor_set), P(C.c_uint64)]
        L.vor_poll.argtypes = [C.c_void_p, C.c_uint64, P(P(vor_result))]
        L.vor_ticket_times.argtypes = [C.c_void_p, C.c_uint64, P(C.c_double), P(C.c_double),
                                       P(C.c_double)]
        L.vor_ticket_count.argtypes = [C.c_void_p, P(C.c_uint64)]
        L.vor_footprint.argtypes = [C.c_void_p, P(vor_set), P(C.c_uint64)]
        L.vor_result_free.argtypes = [P(vor_result)]
        L.vor_result_to_host.argtypes = [C.c_void_p, P(vor_result), P(P(vor_result))]
        L.vor_result_layout.argtypes = [P(P(vor_result)), C.c_uint32, P(C.c_uint64)]
        L.vor_result_free.restype = None
        L.vor_strerror.argtypes = [C.c_int]
        L.vor_strerror.restype = C.c_char_p
        L.vor_set_tuning.argtypes = [C.c_void_p, P(vor_tuning)]
        L.vor_get_tuning.argtypes = [C.c_void_p, P(vor_tuning)]
        L.vor_set_size_tuning.argtypes = [C.c_void_p, P(vor_size_tuning), C.c_uint32]
        L.vor_version.argtypes = []
        L.vor_lloyd.argtypes = [C.c_void_p, P(vor_set), C.c_uint32, P(C.c_int32),
                                P(C.c_int32), P(C.c_uint32)]
        L.vor_filter_keys.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int32),
                                      P(C.c_int32), P(C.c_int64), P(C.c_int64), P(C.c_float),
                                      P(C.c_int32)]
        L.vor_compute_noalloc.argtypes = [C.c_int32, C.c_void_p, P(vor_set), C.c_int32,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                          C.c_void_p, C.c_uint64, P(C.c_uint64), P(C.c_uint64),
                                          P(vor_stats)]
        L.vor_region_diag.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), P(C.c_int64),
                                      P(C.c_float), P(C.c_int32), P(C.c_int32), P(C.c_float),
                                      P(C.c_int32), P(C.c_int32), P(C.c_float)]
        L.vor_peak_fp32.argtypes = [C.c_int32, P(C.c_double)]
        L.vor_peak_copy.argtypes = [C.c_int32, C.c_uint64, P(C.c_double)]
        L.vor_version.restype = C.c_char_p
        for f in ("vor_create", "vor_destroy", "vor_compute", "vor_result_to_host", "vor_compute_batch", "vor_submit",
                  "vor_poll", "vor_ticket_times", "vor_ticket_count", "vor_footprint",
                  "vor_set_tuning", "vor_get_tuning", "vor_set_size_tuning",
                  "vor_filter_keys", "vor_region_diag", "vor_compute_noalloc", "vor_lloyd",
                  "vor_peak_fp32",
                  "vor_peak_copy"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class VorError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {vor_strerror(status)} ({status})")


def vor_strerror(status: int) -> str:
    return lib().vor_strerror(int(status)).decode()


def vor_version() -> str:
    return lib().vor_version().decode()


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise VorError(rc, where)
    return rc


def vor_create(device: int = 0, precision: int = VOR_FP32_FILTERED, flags: int = 0,
               hbm_budget_bytes: int = 0):
    o = vor_opts(device, hbm_budget_bytes, precision, flags)
    h = C.c_void_p()
    _check(lib().vor_create(C.byref(o), C.byref(h)), "vor_create")
    return h


def vor_destroy(ctx) -> None:
    _check(lib().vor_destroy(ctx), "vor_destroy")


def _make_set(x, y, box, device_ptrs=False, region=None):
    """x, y: int32 numpy arrays (host) or (ptr, ptr) device addresses with device_ptrs=True.
    region: None (X = box) or (vx, vy), the vertices of a convex polygon X, counter-clockwise."""
    rn, rx, ry, rkeep = 0, None, None, None
    if region is not None:
        vx = np.ascontiguousarray(region[0], dtype=np.int32)
        vy = np.ascontiguousarray(region[1], dtype=np.int32)
        if vx.shape != vy.shape or vx.ndim != 1:
            raise ValueError("region: vx and vy must be 1-D arrays of the same length")
        rn, rx, ry, rkeep = vx.shape[0], vx.ctypes.data, vy.ctypes.data, (vx, vy)
    if device_ptrs:
        xp, yp, n = x[0], y[0], x[1]
        return vor_set(n, xp, yp, vor_box(*box), VOR_SET_DEVICE, rn, rx, ry), rkeep
    x = np.ascontiguousarray(x, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    keep = (x, y, rkeep)
    return vor_set(x.shape[0], x.ctypes.data, y.ctypes.data, vor_box(*[int(v) for v in box]),
                   0, rn, rx, ry), keep


@dataclass(frozen=True)
class Stats:
    rays: int
    nodes: int
    evals: int
    exact_decisions: int
    deferred_cells: int
    asym_pairs: int
    shells: int
    edges: int
    vertex_tests: int
    adaptive_cells: int
    adaptive_evals: int
    fallback_cmp: int
    fallback_incircle: int
    vertex_rays: int

    def fallback_rates(self):
        """Exact fallbacks per filtered decision of each kind: (ray order, vertex-in-cell)."""
        plain = self.rays + self.vertex_tests - self.vertex_rays
        return (self.fallback_cmp / plain if plain else 0.0,
                self.fallback_incircle / self.vertex_rays if self.vertex_rays else 0.0)


@dataclass
class Result:
    n: int
    cell_off: np.ndarray        # uint32 [n+1]
    nbr: np.ndarray             # int32
    vtx: np.ndarray | None      # structured (x_lo, x_hi, y_lo, y_hi, d)
    dele: np.ndarray            # uint32 [m, 2]
    stats: Stats
    device_ms: float
    status: int
    cells_ms: float = 0.0
    exact_ms: float = 0.0
    grid_ms: float = 0.0
    emit_ms: float = 0.0
    graph_replayed: int = 0
    adaptive_ms: float = 0.0
    t_submit: float = 0.0      # request loop: latency stamps (seconds, monotonic clock)
    t_admit: float = 0.0
    t_done: float = 0.0

    def lines(self, k: int) -> list:
        return self.nbr[self.cell_off[k]:self.cell_off[k + 1]].tolist()

    def vertices_int(self):
        """Pair-form vertices as Python ints (X, Y, D) per entry."""
        v = self.vtx
        X = [int(h) * (1 << 64) + int(l) for l, h in zip(v["x_lo"], v["x_hi"])]
        Y = [int(h) * (1 << 64) + int(l) for l, h in zip(v["y_lo"], v["y_hi"])]
        return X, Y, [int(d) for d in v["d"]]


_RAT = np.dtype([("x_lo", "<u8"), ("x_hi", "<i8"), ("y_lo", "<u8"), ("y_hi", "<i8"), ("d", "<i8")])


class _Owned:
    """Holds a library result: vor_result_free runs once neither this object nor any array that
    views the result's memory is referenced."""
    __slots__ = ("rp",)

    def __init__(self, rp):
        self.rp = rp

    def __del__(self):
        try:
            lib().vor_result_free(self.rp)
        except Exception:
            pass


def _view(owner, addr, dtype, count):
    """count items of dtype at a library-owned host address, without a copy; the array keeps
    `owner` (and so the memory) alive."""
    dt = np.dtype(dtype)
    buf = (C.c_char * (count * dt.itemsize)).from_address(addr)
    buf._owner = owner
    return np.frombuffer(buf, dtype=dt)


def _stats(raw: vor_stats, cache: dict | None = None) -> Stats:
    """Stats of a vor_stats; `cache` shares one object among the results of a batch, which carry
    the run's counters alike."""
    if cache is None:
        return Stats(*[int(getattr(raw, f)) for f, _ in vor_stats._fields_])
    key = bytes(raw)
    st = cache.get(key)
    if st is None:
        st = cache[key] = Stats(*[int(getattr(raw, f)) for f, _ in vor_stats._fields_])
    return st


def _to_result(rp, device: bool = False, owner: _Owned | None = None,
               stats_cache: dict | None = None) -> Result:
    """Result of a vor_result.  With `owner` (host results), the arrays view the library's memory
    and keep it alive; without, they are copies."""
    r = rp.contents
    n = int(r.n)
    st = _stats(r.stats, stats_cache)
    if device:
        # arrays live in device memory: hand back their addresses, never dereference them here
        res = Result(n, np.zeros(0, np.uint32), np.zeros(0, np.int32), None,
                     np.zeros((0, 2), np.uint32), st, float(r.device_ms), int(r.status),
                     float(r.cells_ms), float(r.exact_ms), float(r.grid_ms),
                     float(r.emit_ms), int(r.graph_replayed), float(r.adaptive_ms))
        res.device_ptrs = {"cell_off": r.cell_off, "nbr": r.nbr, "vtx": r.vtx, "del": r.del_,
                           "m": int(r.m)}
        return res
    if r.status != VOR_OK or not r.cell_off:
        return Result(n, np.zeros(0, np.uint32), np.zeros(0, np.int32), None,
                      np.zeros((0, 2), np.uint32), st, float(r.device_ms), int(r.status),
                      float(r.cells_ms), float(r.exact_ms), float(r.grid_ms), float(r.emit_ms),
                      int(r.graph_replayed), float(r.adaptive_ms))

    def arr(addr, dtype, count):
        if owner is not None:
            return _view(owner, addr, dtype, count)
        dt = np.dtype(dtype)
        return np.frombuffer((C.c_char * (count * dt.itemsize)).from_address(addr), dt).copy()

    off = arr(r.cell_off, np.uint32, n + 1)
    E = int(off[-1])
    nbr = arr(r.nbr, np.int32, E) if E else np.zeros(0, np.int32)
    vtx = arr(r.vtx, _RAT, E) if (r.vtx and E) else None
    m = int(r.m)
    dele = arr(r.del_, np.uint32, 2 * m).reshape(m, 2) if m else np.zeros((0, 2), np.uint32)
    return Result(n, off, nbr, vtx, dele, st, float(r.device_ms), int(r.status),
                  float(r.cells_ms), float(r.exact_ms), float(r.grid_ms), float(r.emit_ms),
                  int(r.graph_replayed), float(r.adaptive_ms), float(r.t_submit),
                  float(r.t_admit), float(r.t_done))


class _OwnedMany:
    """Holds the library results that share one host block: vor_result_free runs for each of
    them once no array that views the block is referenced."""
    __slots__ = ("rps",)

    def __init__(self):
        self.rps = []

    def __del__(self):
        try:
            for rp in self.rps:
                lib().vor_result_free(rp)
        except Exception:
            pass


def _own_batch(outs, k: int) -> list:
    """Results of a batch call whose ownership passes to Python.  The results of one run share
    one library block: one buffer per block, each result's arrays are views at their offsets in
    it (no ctypes structure read per result), and the block's results are freed together once
    none of those arrays is referenced.  Results outside a block (error status) go one by one."""
    tab = np.zeros((k, 8), np.uint64)
    _check(lib().vor_result_layout(outs, k, tab.ctypes.data_as(C.POINTER(C.c_uint64))),
           "vor_result_layout")
    rows = tab.tolist()
    res = [None] * k
    cache, groups = {}, {}
    for i in range(k):
        o = outs[i]
        if not o:
            continue
        n, m, a_off, a_nbr, a_vtx, a_del, base, size = rows[i]
        if not base:
            res[i] = _own_result(o, cache)
            continue
        g = groups.get(base)
        if g is None:
            owner = _OwnedMany()
            buf = (C.c_char * size).from_address(base)
            buf._owner = owner
            r0 = o.contents   # every result of one run carries the run's counters and times
            figs = (float(r0.device_ms), int(r0.status), float(r0.cells_ms), float(r0.exact_ms),
                    float(r0.grid_ms), float(r0.emit_ms), int(r0.graph_replayed),
                    float(r0.adaptive_ms), float(r0.t_submit), float(r0.t_admit),
                    float(r0.t_done))
            g = groups[base] = (owner, buf, _stats(r0.stats, cache), figs)
        owner, buf, st, figs = g
        owner.rps.append(o)
        off = np.frombuffer(buf, np.uint32, n + 1, a_off - base)
        E = int(off[-1])
        nbr = np.frombuffer(buf, np.int32, E, a_nbr - base) if E else np.zeros(0, np.int32)
        vtx = np.frombuffer(buf, _RAT, E, a_vtx - base) if (a_vtx and E) else None
        dele = (np.frombuffer(buf, np.uint32, 2 * m, a_del - base).reshape(m, 2) if m
                else np.zeros((0, 2), np.uint32))
        res[i] = Result(n, off, nbr, vtx, dele, st, *figs)
    return res


def _own_result(rp, stats_cache: dict | None = None) -> Result:
    """Result of a host vor_result whose ownership passes to Python: its arrays view the
    library's memory, freed when the last of them (and the Result) is gone."""
    return _to_result(rp, owner=_Owned(rp), stats_cache=stats_cache)


def vor_result_free(rp) -> None:
    lib().vor_result_free(rp)


def vor_compute(ctx, x, y, box, device_ptrs=False, keep_raw=False, device_result=False,
                region=None):
    """x, y: int32 host arrays, or (device address, n) pairs with device_ptrs=True.
    device_result must match the context's VOR_RESULT_DEVICE flag.  region: (vx, vy) of a
    convex polygon X (counter-clockwise), or None for X = box."""
    s, keep = _make_set(x, y, box, device_ptrs, region)
    rp = C.POINTER(vor_result)()
    _check(lib().vor_compute(ctx, C.byref(s), C.byref(rp)), "vor_compute")
    if keep_raw:
        return rp
    if not device_result:
        return _own_result(rp)
    try:
        return _to_result(rp, True)
    finally:
        lib().vor_result_free(rp)


def vor_result_to_host(ctx, res: Result) -> Result:
    """Host copy of a device-resident result (compute with VOR_RESULT_DEVICE); call it before
    the context's next call, while the device arrays are valid."""
    dp = res.device_ptrs
    r = vor_result()
    r.n = res.n
    r.cell_off, r.nbr, r.vtx, r.del_ = dp["cell_off"], dp["nbr"], dp["vtx"], dp["del"]
    r.m = dp["m"]
    r.status = res.status
    rp = C.POINTER(vor_result)()
    _check(lib().vor_result_to_host(ctx, C.byref(r), C.byref(rp)), "vor_result_to_host")
    out = _own_result(rp)
    out.stats, out.device_ms, out.cells_ms = res.stats, res.device_ms, res.cells_ms
    out.exact_ms, out.grid_ms, out.emit_ms = res.exact_ms, res.grid_ms, res.emit_ms
    out.graph_replayed, out.adaptive_ms = res.graph_replayed, res.adaptive_ms
    return out


VOR_NOALLOC_MAX_SITES = 32768


def vor_compute_noalloc(x, y, box, cell_off, nbr, vtx, nbr_cap, dele, del_cap,
                        precision=VOR_FP32_FILTERED, device=0, stream=0, device_ptrs=False,
                        region=None):
    """vor_compute_noalloc (see include/vor.h): x, y host arrays, or (device address, n) pairs
    with device_ptrs=True; cell_off, nbr, vtx (or 0), dele: device addresses of the caller's
    output buffers.  Returns (entries, m, Stats)."""
    s, keep = _make_set(x, y, box, device_ptrs, region)
    e, m, st = C.c_uint64(), C.c_uint64(), vor_stats()
    _check(lib().vor_compute_noalloc(int(device), C.c_void_p(stream or None), C.byref(s),
                                     int(precision), C.c_void_p(cell_off), C.c_void_p(nbr),
                                     C.c_void_p(vtx or None), int(nbr_cap), C.c_void_p(dele),
                                     int(del_cap), C.byref(e), C.byref(m), C.byref(st)),
           "vor_compute_noalloc")
    return int(e.value), int(m.value), Stats(*[int(getattr(st, f)) for f, _ in vor_stats._fields_])


def vor_compute_batch(ctx, sets):
    """sets: list of (x, y, box) or (x, y, box, region).  Returns (status, [Result])."""
    k = len(sets)
    arr = (vor_set * k)()
    keep = []
    for i, t in enumerate(sets):
        x, y, box = t[:3]
        if len(t) > 3 and t[3] is not None:
            s, kp = _make_set(x, y, box, region=t[3])
            arr[i] = s
            keep.append(kp)
            continue
        # the plain case field by field (no intermediate structure)
        x = np.ascontiguousarray(x, dtype=np.int32)
        y = np.ascontiguousarray(y, dtype=np.int32)
        e = arr[i]
        e.n = x.shape[0]
        e.x = x.ctypes.data
        e.y = y.ctypes.data
        bx = e.box
        bx.x0, bx.y0, bx.x1, bx.y1 = (int(v) for v in box)
        keep.append((x, y))
    outs = (C.POINTER(vor_result) * k)()
    rc = lib().vor_compute_batch(ctx, arr, k, outs)
    if rc < 0 and not any(bool(o) for o in outs):
        raise VorError(rc, "vor_compute_batch")
    # thousands of small objects at once: the cyclic collector's passes over them (none of
    # them is garbage yet) would cost more than the conversion itself
    was = gc.isenabled()
    gc.disable()
    try:
        res = _own_batch(outs, k)
    finally:
        if was:
            gc.enable()
    return rc, res


def vor_submit(ctx, x, y, box, region=None) -> int:
    s, keep = _make_set(x, y, box, region=region)
    t = C.c_uint64()
    _check(lib().vor_submit(ctx, C.byref(s), C.byref(t)), "vor_submit")
    return int(t.value)


def vor_poll(ctx, ticket: int):
    """Returns (status, Result | None); status VOR_PENDING while running."""
    rp = C.POINTER(vor_result)()
    rc = lib().vor_poll(ctx, C.c_uint64(ticket), C.byref(rp))
    if rc == VOR_OK:
        return rc, _own_result(rp)
    return rc, None


def vor_ticket_times(ctx, ticket: int):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(lib().vor_ticket_times(ctx, C.c_uint64(ticket), C.byref(a), C.byref(b), C.byref(c)),
           "vor_ticket_times")
    return a.value, b.value, c.value


def vor_ticket_count(ctx) -> int:
    v = C.c_uint64()
    _check(lib().vor_ticket_count(ctx, C.byref(v)), "vor_ticket_count")
    return int(v.value)


def vor_footprint(ctx, x, y, box, region=None) -> int:
    s, keep = _make_set(x, y, box, region=region)
    v = C.c_uint64()
    _check(lib().vor_footprint(ctx, C.byref(s), C.byref(v)), "vor_footprint")
    return int(v.value)


def vor_set_tuning(ctx, sites_per_bucket: float, block: int, block_halfwidth: int = 0,
                   leaf_halfwidth: int = 0, scan_path: int = 0) -> None:
    t = vor_tuning(sites_per_bucket, block, block_halfwidth, leaf_halfwidth, scan_path)
    _check(lib().vor_set_tuning(ctx, C.byref(t)), "vor_set_tuning")


def vor_set_size_tuning(ctx, entries) -> None:
    """entries: [(log2n, sites_per_bucket, block_halfwidth, leaf_halfwidth)] (see include/vor.h);
    [] clears the table."""
    arr = (vor_size_tuning * max(1, len(entries)))()
    for i, (k, rho, h, ht) in enumerate(entries):
        arr[i] = vor_size_tuning(int(k), float(rho), int(h), int(ht))
    _check(lib().vor_set_size_tuning(ctx, arr, len(entries)), "vor_set_size_tuning")


def vor_get_tuning(ctx):
    t = vor_tuning()
    _check(lib().vor_get_tuning(ctx, C.byref(t)), "vor_get_tuning")
    return (float(t.sites_per_bucket), int(t.block), int(t.block_halfwidth),
            int(t.leaf_halfwidth), int(t.scan_path))


def vor_lloyd(ctx, x, y, box, iters: int, region=None):
    """`iters` Lloyd steps on the device (see include/vor.h for the exact step).  Returns
    (x, y, moved): the final sites (int32 [n]) and the number of sites moved per step."""
    s, keep = _make_set(x, y, box, region=region)
    n = int(s.n)
    ox = np.zeros(n, np.int32)
    oy = np.zeros(n, np.int32)
    mv = np.zeros(max(int(iters), 1), np.uint32)
    P = C.POINTER
    _check(lib().vor_lloyd(ctx, C.byref(s), int(iters), ox.ctypes.data_as(P(C.c_int32)),
                           oy.ctypes.data_as(P(C.c_int32)), mv.ctypes.data_as(P(C.c_uint32))),
           "vor_lloyd")
    return ox, oy, mv[:int(iters)].tolist()


def vor_filter_keys(kind, nx, ny, c, dx, dy, device: int = 0):
    """FP32 filter keys of single (line, ray) instances on the device (diagnostic entry).

    kind/nx/ny/c: per-instance arrays (see include/vor.h); dx, dy: Python ints, the exact ray
    direction (|.| < 2^100).  Returns (out [n, 8] float32, sigma [n] int32)."""
    n = len(kind)
    if not len(dx) == len(dy) == n:
        raise ValueError("vor_filter_keys: per-instance arrays of different lengths")
    M = (1 << 64) - 1

    def split(v):
        v = int(v)
        hi = v >> 64                      # floor: the low word is the unsigned remainder
        lo = v & M
        return hi, lo - (1 << 64) if lo >= 1 << 63 else lo

    d = np.zeros((n, 4), np.int64)
    for i in range(n):
        d[i, 0], d[i, 1] = split(dx[i])
        d[i, 2], d[i, 3] = split(dy[i])
    return vor_filter_keys_words(kind, nx, ny, c, d, device)


def vor_filter_keys_words(kind, nx, ny, c, d, device: int = 0):
    """Same as vor_filter_keys with the directions given as int64 words [n, 4]
    (x_hi, x_lo, y_hi, y_lo), the layout of the C entry point."""
    kind = np.ascontiguousarray(kind, np.int32)
    nx = np.ascontiguousarray(nx, np.int32)
    ny = np.ascontiguousarray(ny, np.int32)
    c = np.ascontiguousarray(c, np.int64)
    d = np.ascontiguousarray(d, np.int64).reshape(-1, 4)
    n = kind.shape[0]
    if not nx.shape == ny.shape == c.shape == (n,) or d.shape[0] != n:
        raise ValueError("vor_filter_keys: per-instance arrays of different lengths")
    out = np.zeros((n, 8), np.float32)
    sigma = np.zeros(n, np.int32)
    P = C.POINTER
    _check(lib().vor_filter_keys(int(device), n, kind.ctypes.data_as(P(C.c_int32)),
                                 nx.ctypes.data_as(P(C.c_int32)),
                                 ny.ctypes.data_as(P(C.c_int32)),
                                 c.ctypes.data_as(P(C.c_int64)), d.ctypes.data_as(P(C.c_int64)),
                                 out.ctypes.data_as(P(C.c_float)),
                                 sigma.ctypes.data_as(P(C.c_int32))), "vor_filter_keys")
    return out, sigma


def _dir_words(dx, dy):
    """Exact directions (Python ints) as int64 words [n, 4]: x_hi, x_lo, y_hi, y_lo."""
    M = (1 << 64) - 1

    def split(v):
        v = int(v)
        lo = v & M
        return v >> 64, lo - (1 << 64) if lo >= 1 << 63 else lo

    d = np.zeros((len(dx), 4), np.int64)
    for i in range(len(dx)):
        d[i, 0], d[i, 1] = split(dx[i])
        d[i, 2], d[i, 3] = split(dy[i])
    return d


def vor_region_diag(geom, dx, dy, T, z, device: int = 0):
    """Candidate regions of single ray bounds on the device (diagnostic entry, see
    include/vor.h).  geom [n, 7] (px, py, W, H, s, gx, gy); dx, dy: exact directions as Python
    ints; T [n] float32; z [n, 2] test points.  Returns a dict of arrays: bucket_rect [n, 4],
    coord_rect [n, 4], disk [n, 3], inside [n], sigma [n], ds [n, 2]."""
    geom = np.ascontiguousarray(geom, np.int32).reshape(-1, 7)
    n = geom.shape[0]
    d = _dir_words(dx, dy)
    T = np.ascontiguousarray(T, np.float32)
    z = np.ascontiguousarray(z, np.int32).reshape(-1, 2)
    if d.shape[0] != n or T.shape != (n,) or z.shape[0] != n:
        raise ValueError("vor_region_diag: per-instance arrays of different lengths")
    rects = np.zeros((n, 8), np.int32)
    disk = np.zeros((n, 3), np.float32)
    inside = np.zeros(n, np.int32)
    sigma = np.zeros(n, np.int32)
    ds = np.zeros((n, 2), np.float32)
    P = C.POINTER
    _check(lib().vor_region_diag(int(device), n, geom.ctypes.data_as(P(C.c_int32)),
                                 d.ctypes.data_as(P(C.c_int64)), T.ctypes.data_as(P(C.c_float)),
                                 z.ctypes.data_as(P(C.c_int32)),
                                 rects.ctypes.data_as(P(C.c_int32)),
                                 disk.ctypes.data_as(P(C.c_float)),
                                 inside.ctypes.data_as(P(C.c_int32)),
                                 sigma.ctypes.data_as(P(C.c_int32)),
                                 ds.ctypes.data_as(P(C.c_float))), "vor_region_diag")
    return {"bucket_rect": rects[:, :4], "coord_rect": rects[:, 4:], "disk": disk,
            "inside": inside, "sigma": sigma, "ds": ds}


def vor_peak_fp32(device: int = 0) -> float:
    """Measured FP32 FMA rate of the device in TFLOP/s (see include/vor.h)."""
    v = C.c_double(0.0)
    _check(lib().vor_peak_fp32(int(device), C.byref(v)), "vor_peak_fp32")
    return v.value


def vor_peak_copy(nbytes: int = 1 << 30, device: int = 0) -> float:
    """Measured device-to-device copy rate in GB/s, read plus written (see include/vor.h)."""
    v = C.c_double(0.0)
    _check(lib().vor_peak_copy(int(device), int(nbytes), C.byref(v)), "vor_peak_copy")
    return v.value


class Context:
    """Owning wrapper: ``with Context() as ctx: ctx.compute(x, y, box)``."""

    def __init__(self, device=0, precision=VOR_FP32_FILTERED, flags=0, hbm_budget_bytes=0):
        self.h = None
        self.flags = flags
        self.h = vor_create(device, precision, flags, hbm_budget_bytes)

    def compute(self, x, y, box, **kw):
        kw.setdefault("device_result", bool(self.flags & VOR_RESULT_DEVICE))
        return vor_compute(self.h, x, y, box, **kw)

    def compute_batch(self, sets):
        return vor_compute_batch(self.h, sets)

    def to_host(self, res):
        return vor_result_to_host(self.h, res)

    def lloyd(self, x, y, box, iters, region=None):
        return vor_lloyd(self.h, x, y, box, iters, region)

    def submit(self, x, y, box, region=None):
        return vor_submit(self.h, x, y, box, region)

    def poll(self, ticket):
        return vor_poll(self.h, ticket)

    def times(self, ticket):
        return vor_ticket_times(self.h, ticket)

    def ticket_count(self):
        return vor_ticket_count(self.h)

    def footprint(self, x, y, box, region=None):
        return vor_footprint(self.h, x, y, box, region)

    def tune(self, sites_per_bucket, block, block_halfwidth=0, leaf_halfwidth=0, scan_path=0):
        vor_set_tuning(self.h, sites_per_bucket, block, block_halfwidth, leaf_halfwidth,
                       scan_path)

    def size_tuning(self, entries):
        vor_set_size_tuning(self.h, entries)

    def close(self):
        if self.h:
            vor_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
