"""Mesh quality after the full fixed schedules of two workloads at their
full size, against the oracle's runs of the same schedules from the same
seeded points (tests/golden/fullrun_*.json, written by
tests/golden/make_fullrun.py from the oracle alone).

Iterated DistMesh and Lloyd steps are chaotic: after many iterations the
point sets differ by far more than rounding, and several final meshes are
equally correct.  The comparison is therefore statistical (Eq. 10-11 over
the final triangulation): M_1/2(alpha), M_1/2(beta), mean q and min q within
1%, the normalised beta histograms within an L1 distance of 0.01.
"""
import json
import os

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def T():
    from paper_2309_13824_amd import trime
    trime.lib()
    return trime


def final_quality(wl, prec, og):
    from paper_2309_13824_amd.mesher import Mesher
    m = Mesher(wl, precision=prec, grid=og)
    m.load()
    for method, iters in wl.schedule:
        if method == "cvd":
            m.step_cvd(iters)
        else:
            m.step_dm(iters, fresh=True)
    m.bin()
    m.extract()
    st = m.stats()
    assert st["error"] == 0
    return st


def compare(st, gold, label):
    hist = st["hist_beta"] / max(st["nq"], 1)
    l1 = float(np.abs(hist - np.array(gold["hist_beta"])).sum())
    rel = {k: abs(st[k] - gold[k]) / gold[k] for k in ("half_mean_alpha", "half_mean_beta", "mean_q", "min_q")}
    print("%s: valid %d (oracle %d), rel. differences %s, histogram L1 %.4f" % (
        label, st["nvalid"], gold["nvalid"], {k: "%.2e" % v for k, v in rel.items()}, l1), flush=True)
    for k in ("half_mean_alpha", "half_mean_beta", "mean_q", "min_q"):
        assert rel[k] <= 0.01, (k, st[k], gold[k])
    assert l1 <= 0.01


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("name", ["annulus", "holes20"])
def test_full_schedule_quality_matches_oracle(orc, T, name, prec):
    gold = json.load(open(os.path.join(GOLDEN, "fullrun_%s.json" % name)))
    wl = I.annulus() if name == "annulus" else I.holes20()
    assert (wl.n, wl.seed, wl.grid.nx) == (gold["n"], gold["seed"], gold["grid_n"])
    assert [(m, k) for m, k in wl.schedule] == [tuple(v) for v in gold["schedule"]]
    og = orc.build_grid(wl)
    st = final_quality(wl, prec, og)
    compare(st, gold, "%s %s" % (name, "fp64" if prec == FP64 else "fp32"))
