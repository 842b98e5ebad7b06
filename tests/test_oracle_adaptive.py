"""Pins of the oracle's adaptive run (termination tests, Sec. 6; hybrid
switch, Sec. 4.2; thresholds in Table 8): special cases whose outcome the
definitions fix, and the recorded relative changes against the measured
statistics."""
import math

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I

INF = math.inf


@pytest.fixture(scope="module")
def disk(orc):
    wl = I.disk()
    return wl, orc.build_grid(wl)


def test_quality_test_passes_on_the_first_comparison(orc, disk):
    """Infinite quality thresholds and fac_end = 0 (every point counts as
    moving): a CVD run stops on quality at iteration 1, the first one with a
    previous iteration to compare with."""
    wl, og = disk
    prm = orc.default_params(fac_end=0.0)
    _, _, _, info = orc.run_adaptive(og, wl.x, wl.y, "cvd", 10, t_quality=INF, t_amax=INF, params=prm,
                                     nthreads=8)
    assert info["stop_iter"] == 1 and info["reason"] == orc.STOP_QUALITY and info["iters"] == 2


def test_zero_thresholds_never_stop(orc, disk):
    wl, og = disk
    prm = orc.default_params(fac_end=0.0)
    _, _, _, info = orc.run_adaptive(og, wl.x, wl.y, "dm", 6, t_quality=0.0, t_amax=0.0, params=prm, nthreads=8)
    assert info["stop_iter"] == -1 and info["reason"] == 0 and info["iters"] == 6
    assert all(h["method"] == "dm" for h in info["history"])


def test_movement_test_ends_the_first_iteration(orc, disk):
    """With fac_end so large that no point can move that far, the movement
    test ends the run after iteration 0 (no quality comparison exists yet)."""
    wl, og = disk
    prm = orc.default_params(fac_end=1e9)
    x, y, _, info = orc.run_adaptive(og, wl.x, wl.y, "cvd", 10, t_quality=0.0, t_amax=0.0, params=prm,
                                     nthreads=8)
    assert info["stop_iter"] == 0 and info["reason"] == orc.STOP_MOVEMENT and info["iters"] == 1
    # the stopping iteration's update is kept: one CVD step from the start
    x1, y1, _, _, _, _ = orc.cvd_step(og, wl.x, wl.y, orc.initial_categories(og, wl.x, wl.y),
                                      np.full(wl.n, -1.0), 8)
    assert np.array_equal(x, x1) and np.array_equal(y, y1)


def test_hybrid_switches_then_runs_cvd(orc, disk):
    """An infinite switch threshold switches the hybrid run after iteration 1;
    the quality and movement tests are not applied in the DistMesh phase, so
    a run with infinite quality thresholds still switches before it stops."""
    wl, og = disk
    prm = orc.default_params(fac_end=0.0)
    _, _, _, info = orc.run_adaptive(og, wl.x, wl.y, "hybrid", 8, t_quality=0.0, t_amax=0.0, t_switch=INF,
                                     params=prm, nthreads=8)
    assert info["switch_iter"] == 1 and info["stop_iter"] == -1
    assert [h["method"] for h in info["history"]] == ["dm", "dm"] + ["cvd"] * 6
    _, _, _, info = orc.run_adaptive(og, wl.x, wl.y, "hybrid", 8, t_quality=INF, t_amax=INF, t_switch=INF,
                                     params=prm, nthreads=8)
    assert info["switch_iter"] == 1 and info["stop_iter"] == 2 and info["reason"] == orc.STOP_QUALITY


def test_recorded_changes_follow_the_measured_statistics(orc, disk):
    """The relative changes are |M_k - M_k-1| / M_k-1 of the recorded
    statistics; each CVD iteration's statistics are those of the
    triangulation of the positions it starts from, so the last recorded
    entry equals the quality of the mesh rebuilt from the positions the last
    iteration started from (recomputed here by one fewer iteration)."""
    wl, og = disk
    prm = orc.default_params(fac_end=0.0)
    _, _, _, info = orc.run_adaptive(og, wl.x, wl.y, "cvd", 4, t_quality=0.0, t_amax=0.0, params=prm, nthreads=8)
    h = info["history"]
    assert h[0]["rel"] is None
    for k in range(1, 4):
        for q in range(3):
            want = abs(h[k]["quality"][q] - h[k - 1]["quality"][q]) / h[k - 1]["quality"][q]
            assert h[k]["rel"][q] == pytest.approx(want, rel=1e-12, abs=0)
    x3, y3, _, _ = orc.run_adaptive(og, wl.x, wl.y, "cvd", 3, t_quality=0.0, t_amax=0.0, params=prm,
                                    nthreads=8)
    mesh = orc.triangulate(og, x3, y3, 8, prm)
    q = orc.quality(x3, y3, mesh.tri, mesh.valid)
    assert h[3]["quality"] == (q["half_mean_alpha"], q["half_mean_beta"], q["max_alpha"])
