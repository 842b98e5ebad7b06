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
PEAK = {"f32": 157.3e12, "f64": 78.6e12}  # MI355X vector FP32 / FP64 FLOP/s

# Algorithmic FP operations per counted event of the fused cell kernel
# (FMA = 2, add/mul/div/sqrt = 1, compares free); counts per point come from
# the instrumented oracle on the same workload.
FLOPS_PER = {"candidates": 7, "clip_tests": 6, "cuts": 130, "quad_points": 45, "point": 900}


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
    return ap.parse_args()


def gpu_run(wl, precision, steps, warmup, log):
    import torch
    from paper_2309_13824_amd import trime as T
    from paper_2309_13824_amd.mesher import Mesher

    m = Mesher(wl, precision=precision)
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
    return m, total_ms, float(np.mean(kern_ms)), st


def cpu_baseline(wl, threads, log):
    """The oracle as it stands: one CVD iteration (triangulation + centroids
    + treatment) over every point, on the host cores."""
    from oracle import oracle as orc
    t = time.perf_counter()
    og = orc.build_grid(wl)
    x0, y0 = wl.x, wl.y
    cats = orc.initial_categories(og, x0, y0)
    log("  cpu oracle setup (grid, categories) %.1f s" % (time.perf_counter() - t))
    t = time.perf_counter()
    mesh = orc.triangulate(og, x0, y0, nthreads=threads)
    t_tri = time.perf_counter() - t
    t = time.perf_counter()
    xr, yr, cr, dr, lev, cnt = orc.cvd_step(og, x0, y0, cats, np.full(wl.n, -1.0), nthreads=threads)
    t_cvd = time.perf_counter() - t
    secs = t_tri + t_cvd
    log("  cpu oracle: triangulate %.2f s + cvd %.2f s on %d threads" % (t_tri, t_cvd, threads))
    per_pt = {k: cnt[k] / wl.n for k in ("candidates", "clip_tests", "cuts", "quad_points")}
    return secs, per_pt, mesh, (xr, yr)


def main():
    args = parse()
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2309_13824_amd import inputs as I
    from paper_2309_13824_amd import trime as T

    t = time.perf_counter()
    wl = I.holes20(n=args.n, grid_n=args.grid, iters=args.steps)
    log("workload %s: %d points, %d^2 grid (%.1f s to sample)" % (wl.name, wl.n, wl.grid.nx, time.perf_counter() - t))

    m32, ms32, k32, st32 = gpu_run(wl, T.FP32, args.steps, args.warmup, log)
    out = {"metric": METRIC}
    pit = wl.n * args.steps / (ms32 * 1e-3)
    fp64 = None
    if not args.no_fp64:
        m64, ms64, k64, st64 = gpu_run(wl, T.FP64, args.steps, args.warmup, log)
        fp64 = {"value": wl.n * args.steps / (ms64 * 1e-3), "ms_per_step": ms64 / args.steps,
                "kernel_ms": k64, "fp32_over_fp64": ms64 / ms32}
        del m64
        torch.cuda.empty_cache()

    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    cpu = None
    per_pt = None
    if not args.no_cpu_baseline:
        del m32
        torch.cuda.empty_cache()
        secs, per_pt, _, _ = cpu_baseline(wl, threads, log)
        cpu = {"value": wl.n / secs, "unit": "point-iterations/s", "cores": threads, "kind": "oracle",
               "sample": "one CVD iteration (cells, triangles + Tests 1-3, centroids, treatment) over all "
                         "%d points of the holes20 workload, FP64 with exact predicates" % wl.n}

    roof = None
    if per_pt is not None:
        flops_pt = (FLOPS_PER["point"] + sum(FLOPS_PER[k] * per_pt[k] for k in per_pt))
        achieved = flops_pt * wl.n / (k32 * 1e-3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK["f32"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["f32"], "traffic": None,
                "kernel": "k_cells<float,float,CVD> (fused cells+extraction+centroid)",
                "kernel_ms": k32, "flops_per_point": flops_pt, "counts_per_point": per_pt}

    out.update({
        "value": pit, "unit": "point-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms32 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "holes20: unit square minus 20 disks, %d^2 f32 sdf grid, %d points, "
                               "Gaussian density, CVD iterations" % (args.grid, args.n),
                   "n_points": wl.n, "grid": args.grid, "method": "cvd",
                   "precision": "fp32 + fp64 replay", "seed": wl.seed},
        "roofline": roof, "cpu_baseline": cpu, "fp64": fp64,
        "fp64_replays_per_step": st32["fp64_replays"] / max(args.steps, 1),
        "quality": {k: st32[k] for k in ("half_mean_alpha", "half_mean_beta", "min_q", "mean_q", "nvalid")},
    })
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
