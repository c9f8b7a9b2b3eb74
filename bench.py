"""Benchmark: Voronoi cells per second (bit-exact) of the projector-algorithm engine on MI355X.

Workload (default): one set of n = 2^20 distinct sites uniform in [1, 2^24)^2, X = [0, 2^24]^2,
seed 2, FP32-filtered predicates with exact fallback.  Inputs are resident in HBM (torch
tensors) when the timed region starts; one step = the whole device pipeline (validation, grid,
projector cells, CSR neighbour lists, pair-form vertices, Delaunay edges) through the C ABI.

Prints ONE JSON line.  Also measured, outside the timed steps:
  * every cell of the last timed step's own output, copied to the host after the timed region,
    against the oracle's stored digests of the workload (bit_exact);
  * roofline of the dominant kernel (the filtered cell pass), timed with HIP events on the
    library's stream during the timed steps;
  * the oracle (C, exact half-plane clipping) on a bounded sample of the same cells, on the
    host cores (cpu_baseline), which also checks the sampled cells bit for bit;
  * "modes" (each with its own steps and timings, and its own outputs checked against the
    oracle's digests): the exact-only GPU path on the same set; 4096 config-4 sets in one
    batched call; 4096 sets of the small single-set shape in one batched call, with the
    roofline of its filtered cell kernel; the config-5 request stream served by the request
    loop (capacity, then p50 / p99 latency at 0.5 and 0.8 of it);
  * with --peaks only: the measured FP32 FMA rate and device copy rate of the card.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Per candidate evaluation the FP32 filter executes these floating-point operations:
# 2 sub (delta), mul + fma (q: 3 flops), 2 mul (delta.d products), add (den), add (|.| sum),
# fma (upper den bound: 2 flops), rcp, mul (key) = 13 flops; the compiled inner loop has exactly
# these 11 FP32 instructions per candidate (2 of them FMAs).
FLOPS_PER_EVAL = 13
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector (spec sheet)
PEAK_FP32_NONPACKED = 78.6    # without packed FP32 (the build disables packed FP32 ops)
HBM_PEAK_GBS = 8000.0
ALL_MODES = ("exact", "batched", "batched1", "served")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_1212_1095_amd/csrc/vor_cell.hpp", "paper_1212_1095_amd/csrc/vor_device.hpp",
                  "paper_1212_1095_amd/csrc/vor_kernels.hip", "paper_1212_1095_amd/csrc/vor_internal.h",
                  "paper_1212_1095_amd/csrc/vor_local.hpp", "paper_1212_1095_amd/csrc/vor_tree.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, tag):
    """HBM bytes per launch of `kernel` from the committed counter summary of this workload
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration), or None when there is no
    summary or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{tag}.md")
    try:
        text = open(path).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_hash") != kernel_source_hash():
        return None
    return int(rec["bytes_per_launch"])


def make_workload(n, B, seed, dist="uniform", sides=0):
    """The box [0, B]^2, or (sides > 0) a random convex polygon with at most that many vertices
    inside it, with n sites of the distribution strictly inside."""
    import sitegen
    if sides > 0:
        reg = sitegen.convex_polygon(sides, B, seed=seed)
        return sitegen.in_polygon(n, reg, seed=seed, kind=dist)
    gen = {"uniform": sitegen.uniform, "clustered": sitegen.clustered,
           "lattice": sitegen.lattice}[dist]
    return gen(n, B, seed=seed)


def golden_record(name):
    """The stored oracle digests of a workload (tests/golden/fullsize_digests.json)."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize_digests.json")
    try:
        with open(path) as f:
            return json.load(f)["configs"].get(name)
    except (OSError, ValueError, KeyError):
        return None


def digest_check(results, name):
    """Every cell of `results` against the oracle's stored digests of workload `name`:
    (checked cells, mismatch description or None); (0, reason) when nothing is stored."""
    from oracle import golden_digests
    gold = golden_record(name)
    if gold is None:
        return 0, f"no stored digests for {name}"
    if gold["sets"] != len(results):
        return 0, f"{name}: {len(results)} diagrams, {gold['sets']} stored"
    dg = golden_digests.Digest()
    for r in results:
        vw = None if r.vtx is None else np.frombuffer(r.vtx.tobytes(), "<u8").reshape(-1, 5)
        dg.add(r.cell_off, r.nbr, vw, r.dele)
    got = dg.result()["sha256"]
    kinds = [k for k in ("cell_off", "nbr", "vtx", "del")
             if results[0].vtx is not None or k != "vtx"]
    bad = [k for k in kinds if got[k] != gold["sha256"][k]]
    cells = int(sum(r.n for r in results))
    return (cells, None) if not bad else (0, f"{name}: {bad} differ from the oracle's digests")


def bench_exact_only(vor, torch, xd, yd, ps, steps):
    """The plain exact-only GPU path on the same HBM-resident set (every decision exact)."""
    with vor.Context(device=0, precision=vor.VOR_EXACT_ONLY,
                     flags=vor.VOR_RESULT_DEVICE) as ectx:
        def step():
            return ectx.compute((xd.data_ptr(), ps.n), (yd.data_ptr(), ps.n), ps.box,
                                device_ptrs=True, region=ps.region)
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            er = step()
        torch.cuda.synchronize()
        ew = (time.perf_counter() - t0) / steps
        host = ectx.to_host(er)
    return ew, host, er.device_ms


def batch_size_table():
    """The autotuner's per-set table for uniform batches (empty when none is stored)."""
    from paper_1212_1095_amd import autotune
    return autotune.size_table("uniform")


def bench_batched(vor, sets, name, steps=3, flags=0, kernel_roofline=False):
    """Sets in one call (one launch per stage, graph replayed), host inputs and host results as
    the batch API takes them, per-set grid parameters from the autotuner's batch table; the last
    step's results are checked against the oracle's digests."""
    args = [(s.x, s.y, s.box) for s in sets]
    total = int(sum(s.n for s in sets))
    table = batch_size_table()
    with vor.Context(flags=flags) as ctx:
        ctx.size_tuning(table)
        # warm-up and graph capture (a shape's second call captures it); two calls, the first
        # one's results held meanwhile, so that the library's pinned pool holds the two host
        # blocks of a caller that keeps one batch's results while the next one runs
        held = ctx.compute_batch(args)
        ctx.compute_batch(args)
        del held
        dev, cells, walls = [], [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            rc, res = ctx.compute_batch(args)
            walls.append(time.perf_counter() - t0)
            assert rc == vor.VOR_OK, rc
            dev.append(res[0].device_ms)
            cells.append(res[0].cells_ms)
    checked, err = digest_check(res, name)
    st = res[0].stats
    wall = float(np.mean(walls))
    out = {"sets": len(sets), "sites": total, "steps": steps,
           "ms_per_step_end_to_end": round(1000 * wall, 3),
           "device_ms_per_step": round(float(np.mean(dev)), 3),
           "cells_per_s_end_to_end": round(total / wall, 1),
           "cells_per_s_device": round(total / (np.mean(dev) / 1000.0), 1),
           "vertices": not (flags & vor.VOR_NO_VERTICES),
           "bit_exact_cells": checked, "bit_exact_error": err,
           "fallback_rates": dict(zip(("ray_order", "vertex_in_cell"),
                                      [round(v, 8) for v in st.fallback_rates()])),
           "exact_decisions": st.exact_decisions,
           "tuning": {"per_set_size_classes": len(table),
                      "source": "autotuner batch table (tuning.json)" if table
                      else "library default"}}
    if kernel_roofline:
        evals = st.evals - st.adaptive_evals
        kern_s = float(np.mean(cells)) / 1000.0
        achieved = evals * FLOPS_PER_EVAL / kern_s / 1e12
        out["roofline"] = {"bound": "alu", "achieved": round(achieved, 4),
                           "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(achieved / PEAK_FP32_TFLOPS, 6), "traffic": None,
                           "kernel": "vor::k_cells_fast<256, false>",
                           "kernel_ms": round(1000 * kern_s, 4),
                           "flops_per_eval": FLOPS_PER_EVAL, "evals_per_launch": int(evals),
                           "evals_per_cell": round(evals / total, 2),
                           "frac_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED, 6)}
    return out


def bench_served(vor, count=200, seed=5, hi=1 << 20):
    """Poisson request stream (sizes log-uniform in [100, hi], 45/45/10 uniform / clustered /
    lattice, in [1, 2^24)^2), with vertices: capacity (back to back), then p50 / p99 latency
    from submission to result at 0.5 and 0.8 of it.  Failed requests are counted, not timed.
    The requests with n <= 2^16 are checked against the oracle's digests on every pass."""
    import sitegen
    from oracle import golden_digests
    reqs = sitegen.request_stream(count, 1.0, seed=seed, hi=hi)
    gold = golden_record("config5")
    watch = set(gold.get("stream_index", [])) if gold else set()
    total = int(sum(r.n for _, r in reqs))

    def run(arrivals):
        """Submit at the given offsets (None: all at once); returns (latencies of the OK
        requests in s, failures, wall s, results of the watched requests in stream order)."""
        lat, fails, kept = [], 0, {}
        pending = {}
        i = 0
        t_start = time.perf_counter()
        while i < count or pending:
            now = time.perf_counter() - t_start
            while i < count and (arrivals is None or arrivals[i] <= now):
                r = reqs[i][1]
                pending[ctx.submit(r.x, r.y, r.box)] = i
                i += 1
            for t in list(pending):
                st, res = ctx.poll(t)
                if st == vor.VOR_PENDING:
                    continue
                if st == vor.VOR_OK:
                    lat.append(res.t_done - res.t_submit)
                    if pending[t] in watch:
                        kept[pending[t]] = res
                else:
                    fails += 1
                del pending[t]
            time.sleep(0.0002)
        return lat, fails, time.perf_counter() - t_start, [kept[k] for k in sorted(kept)]

    def verify(kept):
        if not watch or len(kept) != len(watch):
            return 0, "not every watched request returned"
        return digest_check(kept, "config5")

    out = {"requests": count, "sites": total, "max_request_sites": hi, "vertices": True}
    table = batch_size_table()
    out["tuning"] = {"per_set_size_classes": len(table),
                     "source": "autotuner batch table (tuning.json)" if table else "library default"}
    with vor.Context() as ctx:
        ctx.size_tuning(table)
        run(None)   # warm-up: the request loop's workspaces and the pinned result pool
        _, fails, cap_s, kept = run(None)
        rate = count / cap_s
        out["capacity_req_per_s"] = round(rate, 1)
        out["capacity_cells_per_s"] = round(total / cap_s, 1)
        out["capacity_failed"] = fails
        ok_cells, err = verify(kept)
        for rho in (0.5, 0.8):
            arrivals = np.array([a for a, _ in reqs]) / (rho * rate)
            lat, fails, wall, kept = run(arrivals)
            lat_ms = 1000 * np.array(lat) if lat else np.zeros(1)
            c, e = verify(kept)
            ok_cells, err = min(ok_cells, c), err or e
            out[f"load_{rho}"] = {"qps": round(rho * rate, 1),
                                  "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                                  "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                                  "cells_per_s": round(total / wall, 1), "failed": fails,
                                  "completed": len(lat)}
    out["bit_exact_cells_per_pass"] = ok_cells
    out["bit_exact_error"] = err
    return out


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(ps, res, budget_s=12.0, threads=None):
    """Oracle on a bounded sample of cells; returns (cells/s, cores, sample, sample_cells)."""
    from oracle import cdiagram
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(12345)
    probe = np.sort(rng.choice(ps.n, size=min(ps.n, max(64, 8 * threads)),
                               replace=False)).astype(np.int32)
    # a first probe pays the one-time costs (threads, library); a second one sizes the sample
    cdiagram.cells(ps.x, ps.y, ps.box, which=probe, threads=threads, vertices=False,
                   region=ps.region)
    probe = np.sort(rng.choice(ps.n, size=min(ps.n, max(1024, 256 * threads)),
                               replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    cdiagram.cells(ps.x, ps.y, ps.box, which=probe, threads=threads, vertices=False,
                   region=ps.region)
    t_probe = time.perf_counter() - t0
    per_cell = t_probe / probe.shape[0]
    m = int(min(ps.n, max(probe.shape[0], budget_s / max(per_cell, 1e-9))))
    which = np.sort(rng.choice(ps.n, size=m, replace=False)).astype(np.int32)
    t0 = time.perf_counter()
    oc = cdiagram.cells(ps.x, ps.y, ps.box, which=which, threads=threads, vertices=True,
                        region=ps.region)
    dt = time.perf_counter() - t0
    # bit-exact check of the sampled cells (neighbour lists and pair-form vertices)
    bad = 0
    if res is not None:
        for i, k in enumerate(which):
            lo, hi = int(res.cell_off[k]), int(res.cell_off[k + 1])
            if res.nbr[lo:hi].tolist() != oc.lines(i):
                bad += 1
                continue
            if res.vtx is not None:
                v = res.vtx[lo:hi]
                o0, o1 = int(oc.off[i]), int(oc.off[i + 1])
                X = [int(h) * (1 << 64) + int(l) for l, h in zip(v["x_lo"], v["x_hi"])]
                if X != list(oc.vx[o0:o1]) or [int(d) for d in v["d"]] != [int(d) for d in oc.vd[o0:o1]]:
                    bad += 1
    return m / dt, threads, m, bad, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--box", type=int, default=1 << 24)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--dist", default="uniform", choices=["uniform", "clustered", "lattice"])
    ap.add_argument("--region-sides", type=int, default=0, metavar="K",
                    help="X a random convex polygon with at most K sides (0: the box)")
    ap.add_argument("--lloyd", type=int, default=0, metavar="K",
                    help="also time K Lloyd steps on the workload (vor_lloyd)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--modes", default=",".join(ALL_MODES),
                    help="comma list of the further modes timed after the plain set: exact "
                         "(exact-only path, same set), batched (config 4), batched1 (4096 "
                         "config-1 shaped sets), served (config 5 stream); '' for none")
    ap.add_argument("--cpu-budget", type=float, default=10.0,
                    help="wall seconds of the oracle's all-core sample (single thread: a quarter)")
    ap.add_argument("--path", default=None, choices=["grid", "tree"],
                    help="scan path (default: the library's)")
    ap.add_argument("--sites-per-bucket", type=float, default=None)
    ap.add_argument("--block-halfwidth", type=int, default=None)
    ap.add_argument("--leaf-halfwidth", type=int, default=None)
    ap.add_argument("--peaks", action="store_true",
                    help="measure the FP32 FMA rate and the device copy rate, print them, exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes (counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)
        return

    if args.peaks:
        import paper_1212_1095_amd as vor
        fma = vor.vor_peak_fp32(0)
        copy = vor.vor_peak_copy(1 << 30, 0)
        print(json.dumps({"peak_fp32_tflops_measured": round(fma, 2),
                          "peak_fp32_tflops_published_nonpacked": PEAK_FP32_NONPACKED,
                          "peak_fp32_tflops_published_packed": PEAK_FP32_TFLOPS,
                          "copy_GBps_measured": round(copy, 1),
                          "hbm_GBps_published": 8000.0,
                          "note": "FMA loop without packed FP32 (as the cell kernels are built); "
                                  "copy of 1 GiB, bytes read plus written"}), flush=True)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the path shards by "
                                   "cell ranges or sets (see the design notes), but no "
                                   "multi-GPU run is provided", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    modes = [m for m in args.modes.split(",") if m]
    for m in modes:
        if m not in ALL_MODES:
            raise SystemExit(f"unknown mode {m}; choose from {','.join(ALL_MODES)}")

    import torch
    import paper_1212_1095_amd as vor

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    ps = make_workload(args.n, args.box, args.seed, args.dist, args.region_sides)
    log(f"workload: n={ps.n} box={ps.box} seed={args.seed}")
    xd = torch.from_numpy(ps.x).to(dev)
    yd = torch.from_numpy(ps.y).to(dev)
    torch.cuda.synchronize()

    ctx = vor.Context(device=0, precision=vor.VOR_FP32_FILTERED,
                      flags=vor.VOR_RESULT_DEVICE | vor.VOR_TIME_KERNELS)
    tuning = list(vor.vor_get_tuning(ctx.h))
    tuning_source = "library default"
    from paper_1212_1095_amd import autotune
    tuned = autotune.best_params(ps.n, args.dist)
    if tuned is not None:
        tuning = list(tuned)
        tuning_source = "autotuner table (" + os.path.basename(autotune.TABLE) + ")"
    for i, v in ((0, args.sites_per_bucket), (2, args.block_halfwidth), (3, args.leaf_halfwidth),
                 (4, None if args.path is None else (1 if args.path == "tree" else 0))):
        if v is not None:
            tuning[i] = v
            tuning_source = "command line"
    ctx.tune(*tuning)
    log(f"tuning (sites/bucket, block, h, leaf h, path): {tuning}")

    def step():
        return ctx.compute((xd.data_ptr(), ps.n), (yd.data_ptr(), ps.n), ps.box,
                           device_ptrs=True, region=ps.region)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    cells_ms, adapt_ms, dev_ms, last = [], [], [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        last = step()
        cells_ms.append(last.cells_ms)
        adapt_ms.append(last.adaptive_ms)
        dev_ms.append(last.device_ms)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    value = ps.n / (wall / args.steps)
    st = last.stats
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, device {np.mean(dev_ms):.3f} ms, "
        f"grid {last.grid_ms:.3f} cells {np.mean(cells_ms):.3f} adaptive {np.mean(adapt_ms):.3f} "
        f"exact {last.exact_ms:.3f} "
        f"emit {last.emit_ms:.3f} ms, graph {last.graph_replayed}; stats {st}")
    # the last timed step's own output, copied to the host after the timed region: every cell
    # against the oracle's digests of this workload (when stored), and the oracle sample below
    res = ctx.to_host(last)
    ctx.close()
    default_cfg = {(1 << 20, 1 << 24, 2, "uniform", 0): "config2",
                   (1 << 20, 1 << 24, 3, "clustered", 0): "config3",
                   (1000, 1 << 16, 1, "uniform", 0): "config1"}
    wname = default_cfg.get((ps.n, args.box, args.seed, args.dist, args.region_sides))
    exact_cells, exact_err = digest_check([res], wname) if wname else (0, "no stored digests")
    log(f"timed output vs oracle digests: {exact_cells} cells bit-exact, {exact_err or 'ok'}")

    # roofline of the dominant kernel: algorithmic flops per launch / mean launch duration.
    # The filtered grid pass runs as one kernel, the adaptive pass as two (the local grids,
    # then the tree scans for the cells they hand on); the evaluations of the exact pass (a few
    # hundred cells) count with the grid pass.
    if float(np.mean(adapt_ms)) > float(np.mean(cells_ms)):
        evals = st.adaptive_evals
        kern_s = float(np.mean(adapt_ms)) / 1000.0
        kname = "vor::k_cells_local + vor::k_cells_tree<128>"
    else:
        evals = st.evals - st.adaptive_evals
        kern_s = float(np.mean(cells_ms)) / 1000.0
        kname = ("vor::k_cells_fast<256, true>" if ps.region is not None
                 else "vor::k_cells_fast<256, false>")
    achieved = evals * FLOPS_PER_EVAL / kern_s / 1e12
    traffic = (measured_traffic(kname, f"{args.dist}_n{ps.n}")
               if (args.box, args.seed, args.region_sides) == (1 << 24, 2, 0) else None)
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 6),
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "traffic_GBps": (round(traffic / kern_s / 1e9, 1) if traffic else None),
                "kernel": kname, "kernel_ms": round(1000 * kern_s, 4),
                "flops_per_eval": FLOPS_PER_EVAL, "evals_per_launch": int(evals),
                "frac_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED, 6)}

    cpu = None
    if not args.no_cpu:
        v, cores, m, bad, dt = cpu_baseline(ps, res, args.cpu_budget)
        v1, _, m1, _, dt1 = cpu_baseline(ps, None, min(3.0, args.cpu_budget / 4), threads=1)
        cpu = {"value": round(v, 2), "unit": "cells/s", "cores": cores, "kind": "oracle",
               "sample": f"{m} cells sampled uniformly from the same n={ps.n} set "
                         f"(exact half-plane clipping, {dt:.1f} s wall)",
               "sampled_cells_bit_exact": m - bad, "sampled_cells_mismatch": bad,
               "single_thread_value": round(v1, 2),
               "single_thread_sample": f"{m1} cells, {dt1:.1f} s wall",
               "host_cpu": host_cpu_model(), "host_threads_available": os.cpu_count()}
        log(f"oracle sample: {m} cells in {dt:.2f} s on {cores} threads, mismatches {bad}")
        if bad:
            log("ERROR: sampled cells differ from the oracle")

    out_modes = {}
    if "exact" in modes:
        k = max(3, args.steps // 4)
        ew, ehost, edev = bench_exact_only(vor, torch, xd, yd, ps, k)
        c, e = digest_check([ehost], wname) if wname else (0, "no stored digests")
        out_modes["exact_only"] = {"steps": k, "ms_per_step": round(1000 * ew, 3),
                                   "device_ms": round(edev, 3),
                                   "cells_per_s": round(ps.n / ew, 1),
                                   "bit_exact_cells": c, "bit_exact_error": e,
                                   "filtered_speedup": round((ps.n / (wall / args.steps)) /
                                                             (ps.n / ew), 2)}
        log(f"exact-only: {out_modes['exact_only']}")
    if "batched" in modes:
        import sitegen
        sets = sitegen.batch_sets(4096, 4, B=1 << 20, lo=32, hi=65536)
        log("batched config 4 ...")
        out_modes["batched_config4"] = bench_batched(vor, sets, "config4")
        out_modes["batched_config4"]["workload"] = (
            "4096 sets, sizes log-uniform in [32,65536], uniform in [1,2^20)^2, X=[0,2^20]^2, "
            "seed 4, FP32 filter + exact fallback, vertices and Delaunay edges")
        log(f"batched config 4: {out_modes['batched_config4']}")
        del sets
    if "batched1" in modes:
        from oracle import golden_digests
        sets = golden_digests.config1_batch_sets()
        log("batched config-1 shape ...")
        out_modes["batched_config1_shape"] = bench_batched(
            vor, sets, "config1_batch", flags=vor.VOR_TIME_KERNELS, kernel_roofline=True)
        out_modes["batched_config1_shape"]["workload"] = (
            "4096 sets of n=1000 uniform in [1,2^16)^2, X=[0,2^16]^2, seeds 1001..5096, FP32 "
            "filter + exact fallback, vertices and Delaunay edges")
        log(f"batched config-1 shape: {out_modes['batched_config1_shape']}")
        del sets
    if "served" in modes:
        log("served config 5 ...")
        out_modes["served_config5"] = bench_served(vor)
        log(f"served config 5: {out_modes['served_config5']}")

    extra = {}
    if args.lloyd > 0:
        with vor.Context(device=0) as lctx:
            lctx.tune(*tuning)
            lctx.lloyd(ps.x, ps.y, ps.box, 1, region=ps.region)   # warm-up, graph capture
            t0 = time.perf_counter()
            _, _, mv = lctx.lloyd(ps.x, ps.y, ps.box, args.lloyd, region=ps.region)
            lw = (time.perf_counter() - t0) / args.lloyd
        extra["lloyd"] = {"steps": args.lloyd, "ms_per_step": round(1000 * lw, 3),
                          "cells_per_s": round(ps.n / lw, 1), "moved": mv,
                          "note": "host sites in and out once per call; every step runs the "
                                  "whole pipeline with vertices, the centroid and collision "
                                  "kernels, and one host round trip"}
        log(f"lloyd: {extra['lloyd']}")

    fr = st.fallback_rates()
    out = {
        "metric": "Voronoi cells/sec (bit-exact) plain vs batched; p50/p99 latency per request",
        "value": round(value, 1),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+i128",
        "data": "synthetic",
        "config": {"workload": (f"single set, n={ps.n} {args.dist} sites in [1,{args.box})^2, "
                                f"X=[0,{args.box}]^2, seed {args.seed}, FP32 filter + exact "
                                f"fallback, vertices and Delaunay edges"
                                if ps.region is None else
                                f"single set, n={ps.n} {args.dist} sites in a convex polygon X "
                                f"with {len(ps.region[0])} sides inside [0,{args.box}]^2, seed "
                                f"{args.seed}, FP32 filter + exact fallback, vertices and "
                                f"Delaunay edges"),
                   "n": ps.n, "box": args.box, "mode": "plain (single set)"},
        "bit_exact": {"cells": exact_cells, "error": exact_err,
                      "what": "the last timed step's own output, every cell, against the "
                              "oracle's stored digests (tests/golden/fullsize_digests.json)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": out_modes,
        "stats": {"evals_per_cell": round(st.evals / ps.n, 2),
                  "rays_per_cell": round(st.rays / ps.n, 3),
                  "nodes_per_cell": round(st.nodes / ps.n, 3),
                  "shells_per_cell": round(st.shells / ps.n, 3),
                  "exact_decisions": st.exact_decisions, "deferred_cells": st.deferred_cells,
                  "fallback_cmp": st.fallback_cmp, "fallback_incircle": st.fallback_incircle,
                  "fallback_rate_ray_order": round(fr[0], 9),
                  "fallback_rate_vertex_in_cell": round(fr[1], 9),
                  "edges_per_cell": round(st.edges / ps.n, 3),
                  "device_ms": round(float(np.mean(dev_ms)), 4),
                  "adaptive_cells": st.adaptive_cells,
                  "tuning": {"sites_per_bucket": tuning[0], "block": tuning[1],
                             "block_halfwidth": tuning[2], "leaf_halfwidth": tuning[3],
                             "path": "tree" if tuning[4] == 1 else "grid-first",
                             "source": tuning_source},
                  "stage_ms": {"grid": round(last.grid_ms, 4), "cells": round(last.cells_ms, 4),
                               "adaptive": round(last.adaptive_ms, 4),
                               "exact": round(last.exact_ms, 4), "emit": round(last.emit_ms, 4)},
                  "graph_replayed": bool(last.graph_replayed)},
    }
    if extra:
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
