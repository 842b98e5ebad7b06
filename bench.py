"""Benchmark: point-iterations/s of the CVD mesher hot path on one MI355X.

Workload: the unit square minus 20 seeded disks, a 4096^2 float32 sdf grid,
10^6 points drawn from the density rho = 1 + 4 sum_k exp(-|x - c_k|^2/0.01)
over 5 seeded centres, CVD (Lloyd) iterations.  One step = one iteration
of the whole hot path: binning, bounded Voronoi cells, Delaunay extraction
with validity tests and quality statistics, adaptive-quadrature centroids
and point treatment, over all points.  The headline runs FP32 arithmetic
with FP64 replay of undecided points; plain FP64 is timed beside it, and the
CPU oracle is timed on a bounded sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "point-iterations/s at 1e6 pts (FP32+FP64-fallback vs FP64); % of roofline"
PEAK_FP32 = 157.3e12  # MI355X vector FP32 FLOP/s (published)
PEAK_HBM = 8.0e12     # MI355X HBM3E bytes/s (published)

# Algorithmic work of the fused cell kernel (cells, triangles with Tests 1-3
# and quality, CVD centroid, treatment) per point and iteration, as the method
# counts it (not the kernel's own instruction stream): the event counts come
# from the CPU oracle's instrumented run of the same iteration (neighbours
# tested n_c, vertex margins evaluated, cuts n_k, quadrature leaves n_q,
# triangles), priced per event as follows (FMA = 2 flops, add/mul/div/sqrt =
# 1, compares free):
#   cells (a2):      5 per candidate (offset, |q - p|^2, range test), 4 per
#                    vertex margin (n . v - s), 20 per cut (two new vertices by
#                    Cramer's rule), 3 per final vertex (n_v = 3 T / N)
#   extraction (a3): 180 (two owned triangles: centroid, midpoints, AND tests,
#                    mu at 3 midpoints)
#   CVD (a5):        27 per quadrature leaf (area, centroid, bilinear mu,
#                    weight, three sums)
#   stats (a7):      60 (alpha, beta, q and the histogram of ~2 triangles)
FLOPS_PER_EVENT = {"candidates": 5, "clip_tests": 4, "cuts": 20, "vertices": 3, "quad_points": 27}
FLOPS_PER_POINT_FIXED = 180 + 60

# Algorithmic bytes per point of the fused kernel in CVD mode (each position
# and grid node counted once per pass, no re-reads): the positions read once
# per tile plus the octagon span (a2: 12 + 4 in FP32 mode, 16 + 4 in FP64),
# triangles, CSR and the grid values of the validity tests (a3: 101), the
# distinct mu nodes of the cell (a5: ~16 x 4 = 64) and the point state read
# and written by the treatment (a6: 37).
BYTES_PER_POINT = {"fp32": 16 + 101 + 64 + 37, "fp64": 20 + 101 + 64 + 37}

# HBM traffic of one launch of the fused kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (the mean of its last two launches in a short run: the timed
# CVD iteration 2 and the next one; scaled by a 1 GiB copy: FETCH x 2.0,
# WRITE x 1.0), valid for the kernel sources with this digest only.
TRAFFIC = {"sha1": "63db500238238aecf79a8ff6a761f832047ad13e", "bytes_per_launch": 437414752.9}
# counted flops per point of the DistMesh force gather (edge forces over the
# adjacency row, forward Euler, treatment checks)
DM_FLOPS_PER_POINT = 150
# the same price list applied to the cell kernels' own work counters (the
# non-headline workloads, which have no oracle run in the bench)
FLOPS_PER = {"candidates": 7, "margins": 6, "cuts": 154, "leaves": 57, "point": 1088}

# XCD runs (blocks of the fused cell kernel one L2 takes in a row) the
# autotuner tries with each bin density
XCD_RUNS = (1, 4, 8, 16)

# CVD iterations from the seeded points before the autotuner's timing
TUNE_FROM = 10
KERNEL_SOURCES = ["cells_k.hpp", "cells.hip", "trime_dev.hpp", "geom_dev.hpp", "exact_dev.hpp", "launch.hpp"]


def kernel_digest():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_13824_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1000000)
    ap.add_argument("--grid", type=int, default=4096)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--tune", type=str, default="1.4,2.0,2.4,2.8,3.2,3.6",
                    help="bin densities (points per bin) the autotuner tries before the timed run; "
                         "empty for the default 3.3")
    ap.add_argument("--xcd-runs", type=str, default=",".join(str(r) for r in XCD_RUNS),
                    help="XCD runs (blocks of the fused cell kernel one L2 takes in a row) the autotuner "
                         "tries with each density; one value pins it (the HBM counters depend on it)")
    ap.add_argument("--workload", default="holes20",
                    choices=["holes20", "stars", "disk", "annulus", "ellipses", "coast"],
                    help="holes20: the headline CVD run; stars: the batch of 512 star polygons "
                         "(DistMesh), one launch per kernel for all shapes, against a graph of per-shape "
                         "launches and per-shape launches; disk, annulus, ellipses, coast (segment input): "
                         "their fixed schedules, one JSON line each")
    ap.add_argument("--shapes", type=int, default=512)
    ap.add_argument("--persistent", action="store_true",
                    help="stars: also time the persistent batch kernel (only in a library built with "
                         "TRIME_PERSIST_ENABLE; switched off otherwise)")
    ap.add_argument("--batch-only", action="store_true",
                    help="stars: time only the batch with one launch per kernel (no per-shape or graph runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib, log):
    """A plain device-to-device copy of known size, three times: the reference
    the FETCH_SIZE / WRITE_SIZE counters of the cell kernel are scaled by."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: %d MiB read + %d MiB written per copy, 3 copies" % (mib, mib))
    print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)


def gpu_run(wl, precision, steps, warmup, log, tune=(), xcd_runs=XCD_RUNS):
    """The timed run: `steps` CVD iterations from the seeded points, captured
    in one HIP graph and replayed (positions reloaded before each replay,
    outside the timed region), timed with events on the stream the graph runs
    on.  The fused cell kernel's average duration comes from an eager pass of
    the same iterations with a pair of events around that kernel in every
    iteration, recorded on the stream the kernel is launched on (events
    recorded inside the graph do not time the kernels between them)."""
    import torch
    from paper_2309_13824_amd import trime as T
    from paper_2309_13824_amd.mesher import Mesher

    m = Mesher(wl, precision=precision)
    name = "fp32" if precision == T.FP32 else "fp64"
    density = 3.3
    if tune:
        # tuned on the positions after a few iterations: the seeded points'
        # first iterations scan differently from the rest of the run
        m.load()
        m.step_cvd(TUNE_FROM)
        px, py, _ = m.points()
        density, ms = m.autotune(tune, n_iter=4, x=px, y=py, xcd_runs=xcd_runs)
        log("  autotune (%s): %s -> %.2f points per bin, XCD run %d" % (
            name, ", ".join("%.2f/%d: %.3f ms" % (d, r, t) for (d, r), t in sorted(ms.items())), density,
            m.state.xcd_run))
    m.load()
    for _ in range(warmup):
        m.step_cvd(1)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    # eager pass: the fused kernel's duration in every iteration
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:  # materialise the events (the library records them again below)
        a.record(s)
        b.record(s)
    m.load()
    torch.cuda.synchronize()
    for a, b in ev:
        m.state.ev_cells[0] = a.cuda_event
        m.state.ev_cells[1] = b.cuda_event
        T.step_cvd(m.state, 1, stream=s)
    torch.cuda.synchronize()
    m.state.ev_cells[0] = None
    m.state.ev_cells[1] = None
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    # the timed region: the whole loop as one graph
    m.load()  # the graph starts from buffer set 0, as every load leaves it
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    t = time.perf_counter()
    with torch.cuda.graph(g, stream=s):
        T.step_cvd(m.state, steps, stream=s)
    log("  %s: %d iterations captured in one graph in %.2f s" % (name, steps, time.perf_counter() - t))
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    reps = []
    for rep in range(2):  # a warm-up replay, then the timed one
        m.load()
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        with torch.cuda.stream(s):  # replay() launches on the current stream
            t0.record()
            g.replay()
            t1.record()
        torch.cuda.synchronize()
        reps.append((t0.elapsed_time(t1), time.perf_counter() - wall0))
    total_ms, wall = reps[-1]
    m.state.cur_pos = m.state.cur_ord = steps & 1  # the buffers the last iteration wrote
    st = m.stats()
    del g
    log("  precision %s: %d steps in %.2f ms (warm-up replay %.2f ms, wall %.2f ms), fused cell kernel avg "
        "%.3f ms (eager pass), replays %d %s" % (name, steps, total_ms, reps[0][0], wall * 1e3,
                                                 float(np.mean(kern_ms)), st["fp64_replays"], m.replay_reasons()))
    pts = float(wl.n * steps)
    log("  kernel work per point-iteration: candidates %.2f margins %.2f cuts %.2f leaves %.2f; level cap "
        "hits %d, exact points %d" % (st["work_candidates"] / pts, st["work_margins"] / pts,
                                      st["work_cuts"] / pts, st["work_leaves"] / pts, st["level_cap_hits"],
                                      st["exact_points"]))
    return m, total_ms, float(np.mean(kern_ms)), st, density


def cpu_info():
    """Model of the host CPU, the cores this process may use, and the
    thread count the oracle's all-core runs take (at most 16: the host's
    share per GPU)."""
    # the model name, and the family, model and stepping numbers that tell
    # apart CPUs a virtual machine reports under a generic name
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break
                k, _, v = line.partition(":")
                fields[k.strip()] = v.strip()
    except OSError:
        pass
    model = fields.get("model name", "unknown")
    cpu_id = " ".join("%s %s" % (k, fields[k]) for k in ("cpu family", "model", "stepping") if k in fields)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:
        phys = None
    return {"model": model, "cpu_id": cpu_id, "cpus_available": avail, "physical_cores_machine": phys,
            "threads_all": max(1, min(16, avail))}


CPU_SAMPLE_1T = 100000  # points of the single-thread sample (same recipe)


def oracle_iteration(orc, og, x, y, cats, dprev, threads):
    """One CVD iteration of the oracle (triangulation with Tests 1-3 and
    quality, centroids, treatment); its time and the method's event counts
    per point."""
    t = time.perf_counter()
    mesh = orc.triangulate(og, x, y, nthreads=threads)
    orc.quality(x, y, mesh.tri, mesh.valid)
    xn, yn, cn, dn, _, cnt = orc.cvd_step(og, x, y, cats, dprev, nthreads=threads)
    secs = time.perf_counter() - t
    n = float(len(x))
    counts = {k: cnt[k] / n for k in ("candidates", "clip_tests", "cuts", "quad_points")}
    counts["vertices"] = 3.0 * len(mesh.tri) / n
    return secs, (xn, yn, cn, dn), counts


def flops_per_point(counts):
    return FLOPS_PER_POINT_FIXED + sum(FLOPS_PER_EVENT[k] * counts[k] for k in FLOPS_PER_EVENT)


def cpu_baseline(wl, log, bin_density=0.0, end_state=None):
    """The oracle as it stands, on the host: one CVD iteration from the
    seeded start over all points on every core of this process's share
    (<= 16 threads), and the same iteration of the same recipe at
    CPU_SAMPLE_1T points on one thread.  The all-core iteration also gives
    the position error of one GPU CVD step in each precision (the oracle's
    grid uploaded, so both sides see the same inputs) and the method's event
    counts per point; with end_state (the GPU's positions, categories and
    movements after the timed run) the counts are also taken there."""
    from oracle import oracle as orc
    from paper_2309_13824_amd import inputs as I
    info = cpu_info()
    threads = info["threads_all"]
    t = time.perf_counter()
    og = orc.build_grid(wl)
    cats = orc.initial_categories(og, wl.x, wl.y)
    log("  cpu oracle setup (grid, categories) %.1f s; cpu %s (%s), %d cpus available" % (
        time.perf_counter() - t, info["model"], info["cpu_id"], info["cpus_available"]))
    secs, first, counts0 = oracle_iteration(orc, og, wl.x, wl.y, cats, np.full(wl.n, -1.0), threads)
    log("  cpu oracle, one iteration over %d points: %.2f s on %d threads" % (wl.n, secs, threads))
    counts = {"start": counts0}
    if end_state is not None:
        xe, ye, ce, de = end_state
        _, _, counts["end"] = oracle_iteration(orc, og, xe, ye, ce, de, threads)
    small = I.holes20(n=CPU_SAMPLE_1T, grid_n=wl.grid.nx, iters=1)
    og1 = orc.build_grid(small)
    c1 = orc.initial_categories(og1, small.x, small.y)
    secs1, _, _ = oracle_iteration(orc, og1, small.x, small.y, c1, np.full(small.n, -1.0), 1)
    log("  cpu oracle, one iteration over %d points: %.2f s on 1 thread" % (small.n, secs1))
    cpu = {"value": wl.n / secs, "unit": "point-iterations/s", "cores": threads, "kind": "oracle",
           "sample": "one CVD iteration (cells, triangles with Tests 1-3 and quality, centroids, treatment) "
                     "from the seeded start over all %d points of the holes20 workload, FP64 with exact "
                     "predicates" % wl.n,
           "single_thread": {"value": small.n / secs1, "unit": "point-iterations/s", "cores": 1,
                             "sample": "the same iteration of the same recipe at %d points" % small.n},
           "cpu_model": info["model"], "cpu_id": info["cpu_id"], "cpus_available": info["cpus_available"],
           "physical_cores_machine": info["physical_cores_machine"]}
    return cpu, counts, position_error(wl, og, first[:3], bin_density, log)


def position_error(wl, og, ref, bin_density, log):
    """Max and mean |p_gpu - p_oracle| / h after one CVD step from the seeded
    start, FP32 + FP64 replay and plain FP64; categories compared too."""
    import torch
    from paper_2309_13824_amd import trime as T
    from paper_2309_13824_amd.mesher import Mesher
    xr, yr, cr = ref
    fx = np.floor((xr - og.x0) * (1.0 / og.dx)).astype(int)
    fy = np.floor((yr - og.y0) * (1.0 / og.dy)).astype(int)
    h = og.hcell[fy * (og.nx - 1) + fx].astype(np.float64)
    out = {}
    for prec, name in ((T.FP32, "fp32"), (T.FP64, "fp64")):
        m = Mesher(wl, precision=prec, grid=og, bin_density=bin_density)
        m.load()
        m.step_cvd(1)
        gx, gy, gc = m.points()
        err = np.hypot(gx - xr, gy - yr) / h
        out[name] = {"max_h": float(err.max()), "mean_h": float(err.mean()),
                     "categories_equal": bool(np.array_equal(gc, cr))}
        log("  %s position error against the oracle after one CVD step: max %.3g h, mean %.3g h"
            % (name, err.max(), err.mean()))
        del m
        torch.cuda.empty_cache()
    out["what"] = "one CVD step from the seeded start, every point, |p - p_oracle| / h"
    return out


def stars_run(args, log):
    """The star-polygon batch: every shape on its own 512^2 grid, 60
    DistMesh iterations.  The headline runs each kernel of an iteration once
    for all shapes (trime_batch_create; FP32 + FP64 replay, and FP64), the
    60 iterations' launches issued eagerly and captured in one HIP graph (the
    line reports the faster); also timed: the batch re-triangulating every
    iteration,
    one graph of the shapes' own launches per two iterations (FP32), and
    per-shape launches (FP32 and FP64)."""
    import torch
    from paper_2309_13824_amd import inputs as I
    from paper_2309_13824_amd import trime as T
    from paper_2309_13824_amd.mesher import Batch, Mesher
    iters = 60
    t = time.perf_counter()
    wls = I.stars(count=args.shapes, grid_n=512, iters=iters)
    total = sum(w.n for w in wls)
    log("stars: %d shapes, %d points in total (%.1f s to sample)" % (len(wls), total, time.perf_counter() - t))

    def timed(fn, stream=None):
        """GPU time of fn's work, with the events on the stream it runs on."""
        stream = stream or torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    out = {}
    for prec, name in ((T.FP32, "fp32"), (T.FP64, "fp64")):
        t = time.perf_counter()
        ms = [Mesher(w, precision=prec) for w in wls]
        for m in ms:
            m.load()
        torch.cuda.synchronize()
        log("  %s: %d grids built and states loaded in %.1f s" % (name, len(ms), time.perf_counter() - t))

        def per_shape():
            for m in ms:
                T.step_dm(m.state, iters, fresh=False)
        if not args.batch_only:
            per_ms = timed(per_shape)
            out["per_shape_" + name] = total * iters / (per_ms * 1e-3)
            log("  %s per-shape launches: %.1f ms for %d iterations" % (name, per_ms, iters))
        for m in ms:
            m.load()
        t = time.perf_counter()
        b = Batch(ms, method="dm", n_iter=2, kind="kernels")
        log("  one launch per kernel for %d shapes: tables built in %.1f s" % (len(ms), time.perf_counter() - t))
        b.run(2)  # warm-up
        for m in ms:
            m.load()
        torch.cuda.synchronize()
        bat_ms = timed(lambda: b.run(iters), b.stream)
        out["batched_eager_" + name] = total * iters / (bat_ms * 1e-3)
        log("  %s batched kernels: %.1f ms for %d iterations" % (name, bat_ms, iters))
        # the same launches captured as one HIP graph of all the iterations
        # (capture runs nothing: the states stay as loaded)
        for m in ms:
            m.load()
        torch.cuda.synchronize()
        t = time.perf_counter()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=b.stream):
            T.batch_run(b.batch, iters, b.stream)
        torch.cuda.synchronize()
        log("  %s: %d iterations of the batch captured in one graph in %.2f s" % (name, iters, time.perf_counter() - t))

        def replay():
            with torch.cuda.stream(b.stream):
                g.replay()
        replay()  # warm-up (the first replay uploads the graph)
        torch.cuda.synchronize()
        for m in ms:
            m.load()
        torch.cuda.synchronize()
        gb_ms = timed(replay, b.stream)
        del g
        b.close()
        out["batched_graph_" + name] = total * iters / (gb_ms * 1e-3)
        log("  %s batched kernels, one captured graph: %.1f ms for %d iterations" % (name, gb_ms, iters))
        # the line reports the faster of the two ways to issue the launches
        best_ms = min(bat_ms, gb_ms)
        out["batched_" + name] = total * iters / (best_ms * 1e-3)
        out["batched_ms_" + name] = best_ms
        out["batched_how_" + name] = "one captured graph" if gb_ms <= bat_ms else "eager launches"
        # the same batch as one persistent launch (work items of `tiles` =
        # fast-cell tiles, blocks of the other bulk kernels)
        for tiles in (PERSIST_TILES if not args.batch_only else PERSIST_TILES[:1]) if args.persistent else ():
            for m in ms:
                m.load()
            t = time.perf_counter()
            b = Batch(ms, method="dm", n_iter=2, kind="persistent", tiles=tiles)
            log("  persistent batch, items of %s tiles: tables built in %.1f s" % (tiles, time.perf_counter() - t))
            b.run(2)  # warm-up
            for m in ms:
                m.load()
            torch.cuda.synchronize()
            p_ms = timed(lambda: b.run(iters), b.stream)
            b.close()
            errs = sum(m.stats_raw().error != 0 for m in ms)
            key = "persistent_%s_%dx%d" % (name, tiles[0], tiles[1])
            out[key] = total * iters / (p_ms * 1e-3)
            log("  %s persistent batch (%s): %.1f ms for %d iterations, %d shapes with errors" %
                (name, tiles, p_ms, iters, errs))
        # the same batch re-triangulating every iteration
        for m in ms:
            m.load()
        b = Batch(ms, method="dm_always", n_iter=2, kind="kernels")
        b.run(2)  # warm-up
        for m in ms:
            m.load()
        torch.cuda.synchronize()
        alw_ms = timed(lambda: b.run(iters), b.stream)
        b.close()
        out["batched_always_" + name] = total * iters / (alw_ms * 1e-3)
        log("  %s batched kernels, re-triangulating every iteration: %.1f ms for %d iterations" %
            (name, alw_ms, iters))
        for m in ms:  # the flag-mode run's statistics for the roofline below
            m.load()
        b = Batch(ms, method="dm", n_iter=2, kind="kernels")
        torch.cuda.synchronize()
        b.run(iters)
        torch.cuda.synchronize()
        b.close()
        if prec == T.FP32:  # whole-iteration HBM roofline of the timed batch run
            nbytes = 0
            for m in ms:
                tri = m.stats_raw().triangulations
                nbytes += m.n * (tri * ITER_BYTES["dm_tri"] + (iters - tri) * ITER_BYTES["dm"])
            bw = nbytes / (bat_ms * 1e-3)
            out["hbm"] = {"bound": "hbm", "achieved": bw / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                          "frac": bw / PEAK_HBM, "algorithmic_bytes": nbytes, "kernel": "whole iteration"}
        if prec == T.FP32 and not args.batch_only:
            for m in ms:
                m.load()
            t = time.perf_counter()
            b = Batch(ms, method="dm", n_iter=2, nstreams=8, kind="graph")
            log("  graph of 2 iterations x %d shapes captured and instantiated in %.1f s" % (len(ms), time.perf_counter() - t))
            b.run(2)  # warm-up launch
            for m in ms:
                m.load()
            torch.cuda.synchronize()
            gr_ms = timed(lambda: b.run(iters), b.stream)
            b.close()
            out["graph_fp32"] = total * iters / (gr_ms * 1e-3)
            log("  fp32 graph of per-shape launches: %.1f ms for %d iterations" % (gr_ms, iters))
        del ms
        torch.cuda.empty_cache()
    line = {
        "metric": "point-iterations/s, batch of %d star polygons, DistMesh" % len(wls),
        "value": out["batched_fp32"], "unit": "point-iterations/s", "n_gpus": 1, "steps": iters, "warmup": 2,
        "ms_per_step": out["batched_ms_fp32"] / iters, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stars: %d star polygons (8-64 vertices, radii U[0.5,1]) on 512^2 f32 grids, "
                               "log-uniform point counts in [1e3, 1e5], %d points in total, 60 DistMesh "
                               "iterations" % (len(wls), total), "shapes": len(wls), "total_points": total,
                   "seed": 1005,
                   "timing": "one launch per kernel for all shapes; the faster of the 60 iterations' launches "
                             "issued eagerly and of the same launches captured in one HIP graph and replayed: %s"
                             % out["batched_how_fp32"]},
        "batched_fp64": out["batched_fp64"],
        "batched_eager_fp32": out["batched_eager_fp32"], "batched_eager_fp64": out["batched_eager_fp64"],
        "batched_graph_fp32": out["batched_graph_fp32"], "batched_graph_fp64": out["batched_graph_fp64"],
        "batched_always_fp32": out["batched_always_fp32"], "batched_always_fp64": out["batched_always_fp64"],
        "batched_fp32_over_batched_fp64": out["batched_fp32"] / out["batched_fp64"],
        "persistent": {k[len("persistent_"):]: v for k, v in out.items() if k.startswith("persistent_")},
        "whole_iteration_hbm": out["hbm"],
    }
    if not args.no_cpu_baseline:
        # the oracle beside it: the first DistMesh iteration of 8 of the shapes
        threads = args.cpu_threads or cpu_info()["threads_all"]
        secs, errs, npts = 0.0, [], 0
        for w in wls[:8]:
            s_, e_ = oracle_first_step(w, "dm", (T.FP32, T.FP64), threads, lambda _: None)
            secs += s_
            npts += w.n
            errs.append(e_)
        line["cpu_baseline"] = {"value": npts / secs, "unit": "point-iterations/s", "cores": threads,
                                "kind": "oracle", "sample": "the first DistMesh iteration of the first 8 "
                                "shapes (%d points), FP64 with exact predicates" % npts}
        line["position_error"] = {
            "what": "one DistMesh step from the seeded start, every point of the first 8 shapes, "
                    "|p - p_oracle| / h",
            "fp32": {"max_h": max(e["fp32"]["max_h"] for e in errs),
                     "categories_equal": all(e["fp32"]["categories_equal"] for e in errs)},
            "fp64": {"max_h": max(e["fp64"]["max_h"] for e in errs),
                     "categories_equal": all(e["fp64"]["categories_equal"] for e in errs)}}
        log("  cpu oracle: first DistMesh iteration of 8 shapes (%d points) %.2f s; fp32 max error %.3g h"
            % (npts, secs, line["position_error"]["fp32"]["max_h"]))
    if not args.batch_only:
        line.update({"graph_fp32": out["graph_fp32"], "per_shape_fp32": out["per_shape_fp32"],
                     "per_shape_fp64": out["per_shape_fp64"],
                     "batched_over_per_shape_fp32": out["batched_fp32"] / out["per_shape_fp32"],
                     "batched_fp32_over_per_shape_fp64": out["batched_fp32"] / out["per_shape_fp64"]})
    print(json.dumps(line), flush=True)


# Work items of the persistent batch timed beside the one-launch-per-kernel
# batch: (fast-cell tiles, blocks of the other bulk kernels) per item.
PERSIST_TILES = ((1, 4), (2, 8), (4, 16))

# Algorithmic HBM bytes per point-iteration of a whole iteration (every
# kernel), counting each position, grid node and connectivity entry once per
# pass: binning 2 x 49 + 12, the cells with triangles and statistics 156
# (the fused kernel's figure above), the DistMesh force step over a sorted
# row (6 neighbours x 4 + 6 mu samples x 16 + own state 50 = 170) and the
# re-triangulation test's last-triangulation positions 16.
ITER_BYTES = {"cvd": 110 + 156, "dm_tri": 110 + 156 + 170 + 16, "dm": 170 + 16}


def oracle_first_step(wl, method, precs, threads, log):
    """The oracle's first iteration of `method` from the seeded start over
    every point (timed), and the GPU's first iteration in each precision on
    the oracle's grid against it: max and mean |p - p_oracle| / h."""
    from oracle import oracle as orc
    from paper_2309_13824_amd import trime as T
    from paper_2309_13824_amd.mesher import Mesher
    og = orc.build_grid(wl)
    cats = orc.initial_categories(og, wl.x, wl.y)
    t = time.perf_counter()
    mesh = orc.triangulate(og, wl.x, wl.y, nthreads=threads)
    orc.quality(wl.x, wl.y, mesh.tri, mesh.valid)
    if method == "cvd":
        xr, yr, cr, _, _, _ = orc.cvd_step(og, wl.x, wl.y, cats, np.full(wl.n, -1.0), nthreads=threads)
    else:
        xr, yr, cr, _, _, _ = orc.dm_step(og, wl.x, wl.y, cats, mesh)
    secs = time.perf_counter() - t
    fx = np.floor((xr - og.x0) * (1.0 / og.dx)).astype(int)
    fy = np.floor((yr - og.y0) * (1.0 / og.dy)).astype(int)
    h = og.hcell[fy * (og.nx - 1) + fx].astype(np.float64)
    err = {"what": "one %s step from the seeded start, every point, |p - p_oracle| / h" % method}
    for prec in precs:
        name = "fp32" if prec == T.FP32 else "fp64"
        m = Mesher(wl, precision=prec, grid=og)
        m.load()
        if method == "cvd":
            m.step_cvd(1)
        else:
            m.step_dm(1)
        gx, gy, gc = m.points()
        e = np.hypot(gx - xr, gy - yr) / h
        err[name] = {"max_h": float(e.max()), "mean_h": float(e.mean()), "categories_equal": bool(np.array_equal(gc, cr))}
        log("  %s position error against the oracle after one %s step: max %.3g h, mean %.3g h"
            % (name, method, e.max(), e.mean()))
    return secs, err


def grid_build_times(wl, log):
    """Geometry grid of a segment-input workload, built on the GPU from its
    loop (Sec. 3.2): with the workload's sizing, and with the automatic
    sizing field (Eq. 8, K = 0.05) on the same loop; the median of three
    builds each, Mesher setup (workspace allocation) included."""
    import copy

    import torch
    from paper_2309_13824_amd import inputs as I
    from paper_2309_13824_amd.mesher import Mesher
    out = {}
    auto = copy.copy(wl)
    auto.sizing = I.Sizing(I.SZ_AUTO, 0.05, 0.5)
    for name, w in (("segments_%d_uniform" % len(wl.prims[0].poly), wl),
                    ("segments_%d_auto_sizing" % len(wl.prims[0].poly), auto)):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m = Mesher(w)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
            del m
        out[name] = sorted(ts)[1]
        log("  grid build %s on %d^2 nodes: %.1f ms" % (name, wl.grid.nx, out[name]))
    return out


def schedule_run(args, log):
    """disk (DistMesh, FP64, CPU oracle timed beside it), annulus (30 CVD then
    70 DistMesh as configured, and the paper's order 70 DistMesh then 30
    CVD; FP32 + FP64 replay vs FP64), ellipses (70 DistMesh then 30 CVD,
    10^7 points, autotuned bin size, FP32 + FP64 replay) or coast (a
    4096-segment loop minus a disk, 10^5 points, 50 CVD; also the time of
    its grid build from segments, with and without automatic sizing)."""
    import torch
    from paper_2309_13824_amd import inputs as I
    from paper_2309_13824_amd import trime as T
    from paper_2309_13824_amd.mesher import Mesher
    which = args.workload
    t = time.perf_counter()
    wl = {"disk": I.disk, "annulus": I.annulus, "ellipses": I.ellipses, "coast": I.coast}[which]()
    log("workload %s: %d points (%.1f s to sample)" % (wl.name, wl.n, time.perf_counter() - t))
    builds = grid_build_times(wl, log) if which == "coast" else None
    schedules = [wl.schedule]
    if which == "annulus":
        schedules.append([("dm", 70), ("cvd", 30)])
    precs = [T.FP64] if which == "disk" else [T.FP32, T.FP64]
    res = {}
    for prec in precs:
        pname = "fp32" if prec == T.FP32 else "fp64"
        m = Mesher(wl, precision=prec)
        dens = 3.3
        if which == "ellipses":
            dens, ms = m.autotune((1.4, 2.0, 2.4, 2.8, 3.2, 3.6), n_iter=2)
            log("  autotune (%s): %s -> %.2f" % (pname, ", ".join("%.1f: %.2f ms" % kv for kv in sorted(ms.items())), dens))
        variants = [(sch, False) for sch in schedules]
        # DistMesh schedules also as "always": re-triangulating every iteration
        variants += [(sch, True) for sch in schedules if any(meth == "dm" for meth, _ in sch)]
        for sch, always in variants:
            iters = sum(k for _, k in sch)
            m.load()
            m.step_hybrid([(sch[0][0], 2)])  # warm-up
            m.load()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            w0 = time.perf_counter()
            a.record()
            if always:
                for meth, k in sch:
                    if meth == "dm":
                        m.step_dm(k, fresh=True, always=True)
                    else:
                        m.step_cvd(k)
            else:
                m.step_hybrid(sch)
            b.record()
            torch.cuda.synchronize()
            wall = time.perf_counter() - w0
            ms_ = a.elapsed_time(b)
            st = m.stats()
            key = "%s %s%s" % (pname, "+".join("%d %s" % (k, meth) for meth, k in sch),
                               " (DistMesh re-triangulating every iteration)" if always else "")
            n_cvd = sum(k for meth, k in sch if meth == "cvd")
            n_dm = iters - n_cvd
            n_dm_tri = min(max(st["triangulations"] - n_cvd, 0), n_dm)
            nbytes = wl.n * (n_cvd * ITER_BYTES["cvd"] + n_dm_tri * ITER_BYTES["dm_tri"]
                             + (n_dm - n_dm_tri) * ITER_BYTES["dm"])
            bw = nbytes / (ms_ * 1e-3)
            # counted arithmetic of the whole run: the cell kernels' work
            # counters (every triangulation and CVD iteration) and the
            # DistMesh force gather per DistMesh iteration
            cell_pts = float(wl.n) * st["triangulations"]
            flops = (FLOPS_PER["point"] * cell_pts + sum(FLOPS_PER[c] * st["work_" + c]
                                                          for c in ("candidates", "margins", "cuts", "leaves"))
                     + DM_FLOPS_PER_POINT * wl.n * n_dm)
            fl = flops / (ms_ * 1e-3)
            res[key] = {"value": wl.n * iters / (ms_ * 1e-3), "ms_per_step": ms_ / iters, "wall_s": wall,
                        "triangulations": st["triangulations"], "fp64_replays": st["fp64_replays"],
                        "bin_density": dens, "mean_q": st["mean_q"], "min_q": st["min_q"],
                        "whole_iteration_hbm": {"bound": "hbm", "achieved": bw / 1e9, "peak": PEAK_HBM / 1e9,
                                                "unit": "GB/s", "frac": bw / PEAK_HBM,
                                                "algorithmic_bytes": nbytes},
                        "whole_iteration_valu": {"bound": "alu", "achieved": fl / 1e12, "peak": PEAK_FP32 / 1e12,
                                                 "unit": "TFLOP/s", "frac": fl / PEAK_FP32,
                                                 "counted_flops": flops}}
            log("  %s: %.1f ms for %d iterations (%d triangulations), mean q %.4f" % (
                key, ms_, iters, st["triangulations"], st["mean_q"]))
        del m
        torch.cuda.empty_cache()
    first = res[next(iter(res))]
    cpu = None
    perr = None
    threads = args.cpu_threads or cpu_info()["threads_all"]
    if which == "disk" and not args.no_cpu_baseline:
        from oracle import oracle as orc
        og = orc.build_grid(wl)
        t = time.perf_counter()
        orc.run(og, wl.x, wl.y, wl.schedule, nthreads=threads)
        secs = time.perf_counter() - t
        cpu = {"value": wl.n * 50 / secs, "unit": "point-iterations/s", "cores": threads, "kind": "oracle",
               "sample": "the full 50-iteration DistMesh run of the disk workload (2000 points), FP64 with "
                         "exact predicates"}
        log("  cpu oracle: full run %.2f s on %d threads" % (secs, threads))
        _, perr = oracle_first_step(wl, "dm", precs, threads, log)
    elif which == "ellipses" and not args.no_cpu_baseline:
        # the oracle needs minutes at 10^7 points on the 8192^2 grid: the same
        # recipe at 2 10^6 points on a 1024^2 grid, the first DistMesh step
        sample = I.ellipses(n=2000000, grid_n=1024)
        secs, perr = oracle_first_step(sample, "dm", precs, threads, log)
        perr["what"] = ("one DistMesh step from the seeded start, every point of the same recipe at %d points on a "
                        "1024^2 grid, |p - p_oracle| / h" % sample.n)
        cpu = {"value": sample.n / secs, "unit": "point-iterations/s", "cores": threads, "kind": "oracle",
               "sample": "the first DistMesh iteration (triangulation with quality, then the step) of the ellipses "
                         "recipe at %d points on a 1024^2 grid, FP64 with exact predicates" % sample.n}
        log("  cpu oracle: first DistMesh iteration at %d points %.2f s on %d threads" % (sample.n, secs, threads))
    elif which in ("annulus", "coast") and not args.no_cpu_baseline:
        secs, perr = oracle_first_step(wl, wl.schedule[0][0], precs, threads, log)
        cpu = {"value": wl.n / secs, "unit": "point-iterations/s", "cores": threads, "kind": "oracle",
               "sample": "the first %s iteration (triangulation with quality, then the step) from the seeded "
                         "start over all %d points, FP64 with exact predicates" % (wl.schedule[0][0], wl.n)}
        log("  cpu oracle: first iteration %.2f s on %d threads" % (secs, threads))
    line = {"metric": "point-iterations/s, %s workload" % wl.name, "value": first["value"],
            "unit": "point-iterations/s", "n_gpus": 1, "steps": sum(k for _, k in wl.schedule), "warmup": 2,
            "ms_per_step": first["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if which == "disk" else "f32", "data": "synthetic",
            "config": {"workload": "%s, %d points, %d^2 grid, schedule %s" % (
                wl.name, wl.n, wl.grid.nx, wl.schedule), "seed": wl.seed},
            "runs": res, "cpu_baseline": cpu, "position_error": perr}
    if builds:
        line["grid_build_ms"] = builds
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe, log)
        return
    if args.workload == "stars":
        stars_run(args, log)
        return
    if args.workload in ("disk", "annulus", "ellipses", "coast"):
        schedule_run(args, log)
        return
    import torch
    from paper_2309_13824_amd import inputs as I
    from paper_2309_13824_amd import trime as T

    t = time.perf_counter()
    wl = I.holes20(n=args.n, grid_n=args.grid, iters=args.steps)
    log("workload %s: %d points, %d^2 grid (%.1f s to sample)" % (wl.name, wl.n, wl.grid.nx, time.perf_counter() - t))

    tune = tuple(float(v) for v in args.tune.split(",") if v.strip())
    xruns = tuple(int(v) for v in args.xcd_runs.split(",") if v.strip()) or XCD_RUNS
    m32, ms32, k32, st32, dens32 = gpu_run(wl, T.FP32, args.steps, args.warmup, log, tune, xruns)
    # the state the timed run ends in, with the movement of one more step
    # (the CVD error bound of the next iteration), for the oracle's counts there
    xe, ye, _ = m32.points()
    m32.step_cvd(1)
    xe2, ye2, ce2 = m32.points()
    end_state = (xe2, ye2, ce2, np.hypot(xe2 - xe, ye2 - ye))
    run32 = m32.state.xcd_run
    out = {"metric": METRIC}
    pit = wl.n * args.steps / (ms32 * 1e-3)
    fp64 = None
    if not args.no_fp64:
        m64, ms64, k64, st64, dens64 = gpu_run(wl, T.FP64, args.steps, args.warmup, log, tune, xruns)
        fp64 = {"value": wl.n * args.steps / (ms64 * 1e-3), "ms_per_step": ms64 / args.steps,
                "kernel_ms": k64, "fp32_over_fp64": ms64 / ms32, "bin_density": dens64,
                "xcd_run": m64.state.xcd_run}
        del m64
        torch.cuda.empty_cache()
    del m32
    torch.cuda.empty_cache()

    cpu = perr = counts = None
    if not args.no_cpu_baseline:
        cpu, counts, perr = cpu_baseline(wl, log, dens32, end_state)

    # roofline of the fused cell kernel against both ceilings: algorithmic
    # bytes per point and algorithmic flops per point (the oracle's event
    # counts, mean of the start and the end of the run), over the kernel's
    # average duration in the timed graph; the bound is the ceiling that
    # takes longer at peak
    if counts:
        keys = list(counts["start"])
        cmean = {k: float(np.mean([c[k] for c in counts.values()])) for k in keys}
        flops_pt = flops_per_point(cmean)
    else:
        cmean, flops_pt = None, None
    bytes_pt = BYTES_PER_POINT["fp32"]
    hbm_bw = bytes_pt * wl.n / (k32 * 1e-3)
    hbm = {"achieved": hbm_bw / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": hbm_bw / PEAK_HBM,
           "bytes_per_point": bytes_pt}
    valu = None
    if flops_pt is not None:
        fl = flops_pt * wl.n / (k32 * 1e-3)
        valu = {"achieved": fl / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": fl / PEAK_FP32,
                "flops_per_point": flops_pt}
    hbm_bound = flops_pt is None or bytes_pt / PEAK_HBM >= flops_pt / PEAK_FP32
    main_roof = hbm if hbm_bound else valu
    traffic = TRAFFIC["bytes_per_launch"] if kernel_digest() == TRAFFIC["sha1"] else None
    roof = {"bound": "hbm" if hbm_bound else "alu", "achieved": main_roof["achieved"], "peak": main_roof["peak"],
            "unit": main_roof["unit"], "frac": main_roof["frac"], "traffic": traffic,
            "kernel": "k_cells<float, float, CVD> (cells, triangles, validity, quality, centroid, treatment)",
            "kernel_ms": k32, "hbm": hbm, "valu": valu,
            "oracle_counts_per_point": {"mean": cmean, **(counts or {})}}

    out.update({
        "value": pit, "unit": "point-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms32 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "holes20: unit square minus 20 disks, %d^2 f32 sdf grid, %d points, "
                               "Gaussian density, CVD iterations" % (args.grid, args.n),
                   "n_points": wl.n, "grid": args.grid, "method": "cvd",
                   "precision": "fp32 cut and octagon margins (fp64 re-evaluation inside their error bound, fp64 replay of points left undecided); vertices, positions and centroid sums in fp64", "seed": wl.seed, "bin_density": dens32, "xcd_run": run32,
                   "timing": "one HIP graph of all timed iterations, replayed; the fused kernel's duration "
                             "from an eager pass of the same iterations"},
        "roofline": roof, "cpu_baseline": cpu, "fp64": fp64,
        "position_error": perr,
        "fp64_replays_per_step": st32["fp64_replays"] / max(args.steps, 1),
        "kernel_work_per_point": {k: st32["work_" + k] / float(wl.n * args.steps)
                                  for k in ("candidates", "margins", "cuts", "leaves")},
        "quality": {k: st32[k] for k in ("half_mean_alpha", "half_mean_beta", "min_q", "mean_q", "nvalid")},
    })
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
