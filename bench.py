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

# Algorithmic FP operations per counted event of the fused cell kernel
# (FMA = 2, add/mul/div/sqrt/rcp = 1, compares and selects free), read off the
# arithmetic of each step; the event counts are the kernel's own work counters
# over the timed iterations.
#   candidate: offset (2), |q-p|^2 (3), range test (2)
#   margin:    n.v - s (4), its error bound (2)
#   cut:       two vertices by Cramer's rule with bounds (2 x 32), the rows of
#              the neighbouring constraints (10), the radius bound over ~8
#              vertices (8 x 10), the record shifts (0)
#   leaf:      area (5), centroid (6), grid coordinates (8), bilinear mu (11),
#              weight mu^-2 (3), three sums (5), its share of the bisections
#              (longest edge 15 + midpoint 4)
#   point:     octagon tests of ~6 vertices at two neighbours (6 x 2 x 8 x 8),
#              validity of ~2 triangles (2 x 60), quality of ~2 (2 x 45), area
#              and level loop (~40), treatment (~40), setup (~30)
FLOPS_PER = {"candidates": 7, "margins": 6, "cuts": 154, "leaves": 57, "point": 1088}

# Algorithmic bytes per point of the fused kernel: its own state read once
# (x, y, dprev 24 + cat 1 + id 4 + span 4 + order 4), the new state written
# (x, y, dprev 24 + cat 1), ~2 owned triangles (2 x 13) + count 4, and the
# distinct mu nodes of its cell (~16 x 4); neighbour positions are counted
# once, with the point that owns them.
BYTES_PER_POINT = 37 + 25 + 30 + 64

# HBM traffic of one launch of the fused kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (first two CVD iterations, scaled by a 1 GiB copy: FETCH x 2.0,
# WRITE x 1.0), valid for the kernel sources with this digest only.
TRAFFIC = {"sha1": "05db16e10958f712c6a7a92bb2cd27bb3d4934d3", "bytes_per_launch": 341257508.3}
# counted flops per point of the DistMesh force gather (edge forces over the
# adjacency row, forward Euler, treatment checks)
DM_FLOPS_PER_POINT = 150

# CVD iterations from the seeded points before the autotuner's timing
TUNE_FROM = 10
KERNEL_SOURCES = ["cells.hip", "trime_dev.hpp", "geom_dev.hpp", "exact_dev.hpp", "launch.hpp"]


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
    ap.add_argument("--tune", type=str, default="1.0,1.4,2.0,2.8",
                    help="bin densities (points per bin) the autotuner tries before the timed run; "
                         "empty for the default 3.3")
    ap.add_argument("--workload", default="holes20",
                    choices=["holes20", "stars", "disk", "annulus", "ellipses", "coast"],
                    help="holes20: the headline CVD run; stars: the batch of 512 star polygons "
                         "(DistMesh), one launch per kernel for all shapes, against a graph of per-shape "
                         "launches and per-shape launches; disk, annulus, ellipses, coast (segment input): "
                         "their fixed schedules, one JSON line each")
    ap.add_argument("--shapes", type=int, default=512)
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


def gpu_run(wl, precision, steps, warmup, log, tune=()):
    import torch
    from paper_2309_13824_amd import trime as T
    from paper_2309_13824_amd.mesher import Mesher

    m = Mesher(wl, precision=precision)
    density = 3.3
    if tune:
        # tuned on the positions after a few iterations: the seeded points'
        # first iterations scan differently from the rest of the run
        m.load()
        m.step_cvd(TUNE_FROM)
        px, py, _ = m.points()
        density, ms = m.autotune(tune, n_iter=4, x=px, y=py)
        log("  autotune (%s): %s -> %.2f points per bin" % (
            "fp32" if precision == T.FP32 else "fp64",
            ", ".join("%.2f: %.3f ms" % (d, t) for d, t in sorted(ms.items())), density))
    m.load()
    for _ in range(warmup):
        m.step_cvd(1)
    torch.cuda.synchronize()
    m.load()  # timed run starts from the seeded initial points
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:  # materialise the events
        a.record(stream)
        b.record(stream)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for a, b in ev:
        m.state.ev_cells[0] = a.cuda_event
        m.state.ev_cells[1] = b.cuda_event
        T.step_cvd(m.state, 1)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    m.state.ev_cells[0] = None
    m.state.ev_cells[1] = None
    total_ms = t0.elapsed_time(t1)
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    st = m.stats()
    log("  precision %s: %d steps in %.2f ms (wall %.2f ms), fused cell kernel avg %.3f ms, replays %d %s"
        % ("fp32" if precision == T.FP32 else "fp64", steps, total_ms, wall * 1e3, float(np.mean(kern_ms)),
           st["fp64_replays"], m.replay_reasons()))
    pts = float(wl.n * steps)
    log("  work per point-iteration: candidates %.2f margins %.2f cuts %.2f leaves %.2f; level cap hits %d, "
        "exact points %d" % (st["work_candidates"] / pts, st["work_margins"] / pts, st["work_cuts"] / pts,
                             st["work_leaves"] / pts, st["level_cap_hits"], st["exact_points"]))
    return m, total_ms, float(np.mean(kern_ms)), st, density


CPU_ITERS = 3


def cpu_baseline(wl, threads, log, bin_density=0.0):
    """The oracle as it stands: the first CPU_ITERS CVD iterations from the
    seeded start (triangulation with validity and quality, centroids,
    treatment) over every point, on the host cores; setup not timed.  Its
    first iteration also gives the position error of one GPU CVD step in
    each precision (the oracle's grid uploaded, so both sides see the same
    inputs), in units of the local h, over every point."""
    from oracle import oracle as orc
    t = time.perf_counter()
    og = orc.build_grid(wl)
    x, y = wl.x, wl.y
    cats = orc.initial_categories(og, x, y)
    dprev = np.full(wl.n, -1.0)
    log("  cpu oracle setup (grid, categories) %.1f s" % (time.perf_counter() - t))
    secs = 0.0
    first = None
    for it in range(CPU_ITERS):
        t = time.perf_counter()
        mesh = orc.triangulate(og, x, y, nthreads=threads)
        orc.quality(x, y, mesh.tri, mesh.valid)
        x, y, cats, dprev, _, _ = orc.cvd_step(og, x, y, cats, dprev, nthreads=threads)
        dt = time.perf_counter() - t
        secs += dt
        if it == 0:
            first = (x, y, cats)
        log("  cpu oracle iteration %d: %.2f s on %d threads" % (it + 1, dt, threads))
    return secs, position_error(wl, og, first, bin_density, log)


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
    for all shapes (trime_batch_create; FP32 + FP64 replay, and FP64); also
    timed: one graph of the shapes' own launches per two iterations (FP32),
    and per-shape launches (FP32 and FP64)."""
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
        b.close()
        out["batched_" + name] = total * iters / (bat_ms * 1e-3)
        out["batched_ms_" + name] = bat_ms
        log("  %s batched kernels: %.1f ms for %d iterations" % (name, bat_ms, iters))
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
                   "seed": 1005},
        "batched_fp64": out["batched_fp64"],
        "batched_always_fp32": out["batched_always_fp32"], "batched_always_fp64": out["batched_always_fp64"],
        "batched_fp32_over_batched_fp64": out["batched_fp32"] / out["batched_fp64"],
        "whole_iteration_hbm": out["hbm"],
    }
    if not args.no_cpu_baseline:
        # the oracle beside it: the first DistMesh iteration of 8 of the shapes
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
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
            dens, ms = m.autotune((1.4, 2.0, 2.8), n_iter=2)
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
    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
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
    m32, ms32, k32, st32, dens32 = gpu_run(wl, T.FP32, args.steps, args.warmup, log, tune)
    out = {"metric": METRIC}
    pit = wl.n * args.steps / (ms32 * 1e-3)
    fp64 = None
    if not args.no_fp64:
        m64, ms64, k64, st64, dens64 = gpu_run(wl, T.FP64, args.steps, args.warmup, log, tune)
        fp64 = {"value": wl.n * args.steps / (ms64 * 1e-3), "ms_per_step": ms64 / args.steps,
                "kernel_ms": k64, "fp32_over_fp64": ms64 / ms32, "bin_density": dens64}
        del m64
        torch.cuda.empty_cache()

    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    cpu = None
    perr = None
    if not args.no_cpu_baseline:
        del m32
        torch.cuda.empty_cache()
        secs, perr = cpu_baseline(wl, threads, log, dens32)
        cpu = {"value": wl.n * CPU_ITERS / secs, "unit": "point-iterations/s", "cores": threads, "kind": "oracle",
               "sample": "the first %d CVD iterations from the seeded start (cells, triangles with Tests 1-3 "
                         "and quality, centroids, treatment) over all %d points of the holes20 workload, "
                         "FP64 with exact predicates" % (CPU_ITERS, wl.n)}

    # roofline of the fused cell kernel: algorithmic flops from its own work
    # counters, algorithmic bytes from the per-point model; the larger time
    # names the bound
    pts = float(wl.n * args.steps)
    per_pt = {k: st32["work_" + k] / pts for k in ("candidates", "margins", "cuts", "leaves")}
    flops_pt = FLOPS_PER["point"] + sum(FLOPS_PER[k] * per_pt[k] for k in per_pt)
    t_alu = flops_pt * wl.n / PEAK_FP32
    t_hbm = BYTES_PER_POINT * wl.n / PEAK_HBM
    traffic = TRAFFIC["bytes_per_launch"] if kernel_digest() == TRAFFIC["sha1"] else None
    if t_alu >= t_hbm:
        achieved = flops_pt * wl.n / (k32 * 1e-3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32}
    else:
        achieved = BYTES_PER_POINT * wl.n / (k32 * 1e-3)
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": achieved / PEAK_HBM}
    roof.update({"traffic": traffic, "kernel": "k_cells<float, float, CVD> (cells, extraction, centroid, "
                 "treatment)", "kernel_ms": k32, "flops_per_point": flops_pt,
                 "bytes_per_point": BYTES_PER_POINT, "counts_per_point": per_pt})

    out.update({
        "value": pit, "unit": "point-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms32 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "holes20: unit square minus 20 disks, %d^2 f32 sdf grid, %d points, "
                               "Gaussian density, CVD iterations" % (args.grid, args.n),
                   "n_points": wl.n, "grid": args.grid, "method": "cvd",
                   "precision": "fp32 + fp64 replay", "seed": wl.seed, "bin_density": dens32},
        "roofline": roof, "cpu_baseline": cpu, "fp64": fp64,
        "position_error": perr,
        "fp64_replays_per_step": st32["fp64_replays"] / max(args.steps, 1),
        "quality": {k: st32[k] for k in ("half_mean_alpha", "half_mean_beta", "min_q", "mean_q", "nvalid")},
    })
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
