"""Writes the oracle's mesh quality after full fixed-schedule runs of two
seeded workloads, the expected values of the full-run GPU quality tests.

Only the oracle computes them (FP64, exact predicates): the seeded points of
the workload, the oracle's own grid, the workload's whole schedule (CVD with
a triangulation every iteration, Alg. 2; DistMesh re-triangulating when a
point moved more than fac_retria h, Alg. 1), then the triangulation of the
final points and its quality (Eq. 10-11: M_1/2 of alpha and beta, min and
mean q = 1/alpha, max alpha, the beta histogram with 40 bins on [1, 3)).

    python tests/golden/make_fullrun.py [holes20|annulus ...]

Runs take about 25 minutes (holes20, 1e6 points, 100 CVD iterations) and
3 minutes (annulus, 1e5 points, 30 CVD then 70 DistMesh) on 8 threads.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2309_13824_amd import inputs as I  # noqa: E402

WORKLOADS = {
    "holes20": lambda: I.holes20(),   # 1e6 points, 4096^2, 100 CVD
    "annulus": lambda: I.annulus(),   # 1e5 points, 1024^2, 30 CVD -> 70 DM
}


def run(name, nthreads):
    wl = WORKLOADS[name]()
    t0 = time.time()
    og = orc.build_grid(wl)
    sched = [(m, int(k)) for m, k in wl.schedule]
    x, y, cat, fin, info = orc.run(og, wl.x, wl.y, sched, nthreads=nthreads)
    q = orc.quality(x, y, fin.tri, fin.valid)
    out = {
        "workload": name, "n": int(wl.n), "seed": int(wl.seed), "grid_n": int(wl.grid.nx),
        "schedule": sched,
        "triangulations": int(sum(1 for i in info if i["triangulated"])),
        "ntri": int(len(fin.tri)), "nvalid": int(fin.valid.sum()),
        "min_q": q["min_q"], "mean_q": q["mean_q"],
        "half_mean_alpha": q["half_mean_alpha"], "half_mean_beta": q["half_mean_beta"],
        "max_alpha": q["max_alpha"], "hist_beta": [float(v) for v in q["hist_beta"]],
        "oracle_seconds": round(time.time() - t0, 1), "threads": nthreads,
    }
    path = os.path.join(HERE, "fullrun_%s.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["min_q"], out["mean_q"], out["oracle_seconds"], flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    for nm in names:
        run(nm, int(os.environ.get("ORC_THREADS", "8")))
