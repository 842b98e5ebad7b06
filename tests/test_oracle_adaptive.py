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


# ------------------------------------------------------- point addition --

def circumradius_bisectors(ax, ay, bx, by, cx, cy):
    """Circumradius as the distance from a to the intersection of the
    perpendicular bisectors of ab and ac (Cramer's rule, a at the origin)."""
    bx, by, cx, cy = bx - ax, by - ay, cx - ax, cy - ay
    d = 2.0 * (bx * cy - by * cx)
    b2, c2 = bx * bx + by * by, cx * cx + cy * cy
    ux = (cy * b2 - by * c2) / d
    uy = (bx * c2 - cx * b2) / d
    return math.hypot(ux, uy)


def test_added_points_are_the_centroids_of_the_largest_circumradii(orc, disk):
    """Uniform sizing (one h over the disk's grid): the selection is the
    n_add valid triangles of largest circumradius, found by brute force over
    the triangles with an independent circumradius formula, returned in the
    order of (owner id, second id) at their centroids."""
    wl, og = disk
    assert len(np.unique(og.hcell)) == 1
    mesh = orc.triangulate(og, wl.x, wl.y, 8)
    tris = [tuple(int(v) for v in t) for t, ok in zip(mesh.tri, mesh.valid) if ok]
    R = [circumradius_bisectors(wl.x[a], wl.y[a], wl.x[b], wl.y[b], wl.x[c], wl.y[c]) for a, b, c in tris]
    order = sorted(range(len(tris)), key=lambda i: (-R[i], tris[i][0], tris[i][1]))
    for k in (1, 37, 600):
        # a clear gap at the cut, so rounding differences cannot move it
        assert R[order[k - 1]] - R[order[k]] > 1e-9 * R[order[k]]
        chosen = sorted(order[:k], key=lambda i: (tris[i][0], tris[i][1]))
        gx = np.array([(wl.x[tris[i][0]] + wl.x[tris[i][1]] + wl.x[tris[i][2]]) / 3 for i in chosen])
        gy = np.array([(wl.y[tris[i][0]] + wl.y[tris[i][1]] + wl.y[tris[i][2]]) / 3 for i in chosen])
        px, py = orc.added_points(og, wl.x, wl.y, mesh, k)
        assert len(px) == k
        assert np.allclose(px, gx, rtol=0, atol=1e-15) and np.allclose(py, gy, rtol=0, atol=1e-15)


def lattice_mesh(orc, m):
    """An m x m lattice of spacing 1/8 (exact binary coordinates), each
    square cut along the same diagonal: congruent right isosceles triangles,
    whose circumradii are exactly equal in FP64.  Rows of tri start at the
    smallest id and run CCW."""
    ids = lambda i, j: j * m + i  # noqa: E731
    x = np.array([(i - m / 2) / 8 for j in range(m) for i in range(m)], np.float64)
    y = np.array([(j - m / 2) / 8 for j in range(m) for i in range(m)], np.float64)
    tri = []
    for j in range(m - 1):
        for i in range(m - 1):
            for t in ((ids(i, j), ids(i + 1, j), ids(i + 1, j + 1)), (ids(i, j), ids(i + 1, j + 1), ids(i, j + 1))):
                r = t.index(min(t))
                tri.append(t[r:] + t[:r])
    tri = np.array(tri, np.int32)
    mesh = orc.Mesh(tri, np.ones(len(tri), np.uint8), np.zeros(m * m + 1, np.int64), np.zeros(0, np.int32), {})
    return x, y, mesh


def test_added_points_break_ratio_ties_by_owner_then_second_id(orc, disk):
    """All ratios equal (lattice triangles under one h): the selection is the
    n_add triangles of smallest (owner id, second id)."""
    _, og = disk
    x, y, mesh = lattice_mesh(orc, 5)
    tri = mesh.tri
    d1x, d1y = x[tri[:, 1]] - x[tri[:, 0]], y[tri[:, 1]] - y[tri[:, 0]]
    d2x, d2y = x[tri[:, 2]] - x[tri[:, 0]], y[tri[:, 2]] - y[tri[:, 0]]
    assert np.all(d1x * d2y - d1y * d2x > 0)  # CCW
    keys = sorted((int(a), int(b), k) for k, (a, b, _) in enumerate(tri))
    for n_add in (1, 7, 20):
        want = [k for _, _, k in keys[:n_add]]
        gx = np.array([x[tri[k]].sum() / 3 for k in want])
        gy = np.array([y[tri[k]].sum() / 3 for k in want])
        px, py = orc.added_points(og, x, y, mesh, n_add)
        assert np.allclose(px, gx, rtol=0, atol=1e-15) and np.allclose(py, gy, rtol=0, atol=1e-15)


def test_scaled_grid_scales_h_and_nothing_else(orc, disk):
    _, og = disk
    g1 = orc.scaled_grid(og, 1.0)
    assert np.array_equal(g1.hcell, og.hcell) and g1.h_avg == og.h_avg
    g2 = orc.scaled_grid(og, 2.0)  # a power of two: exact
    assert np.array_equal(g2.hcell, 2 * og.hcell) and g2.h_avg == 2 * og.h_avg
    assert np.array_equal(g2.sdf, og.sdf) and np.array_equal(g2.mu, og.mu) and np.array_equal(g2.cat, og.cat)


def test_growing_from_all_points_is_the_adaptive_run(orc, disk):
    """n_init = N_total: nothing to add, h unscaled; the run is the
    adaptive run point for point."""
    wl, og = disk
    x, y, c, info = orc.run_adaptive(og, wl.x, wl.y, "hybrid", 200, nthreads=8)
    gx, gy, gc, ginfo = orc.run_growing(og, wl.x, wl.y, "hybrid", 200, wl.n, nthreads=8)
    assert ginfo["adds"] == []
    assert (ginfo["iters"], ginfo["switch_iter"], ginfo["stop_iter"], ginfo["reason"]) == \
        (info["iters"], info["switch_iter"], info["stop_iter"], info["reason"])
    assert np.array_equal(gx, x) and np.array_equal(gy, y) and np.array_equal(gc, c)


def test_growth_schedule_with_an_infinite_threshold(orc, disk):
    """t_add = inf: every iteration with a previous one to compare with adds
    min(floor(fac_add n), N - n) points; after an addition the next
    iteration has none, so additions fall on iterations 1, 3, 5, ... until
    all N points are in, and every iteration runs on the current count."""
    wl, og = disk
    _, _, _, info = orc.run_growing(og, wl.x, wl.y, "dm", 12, 400, t_add=INF, t_quality=0.0, t_amax=0.0,
                                    nthreads=8)
    assert info["adds"] == [(1, 240), (3, 384), (5, 614), (7, 362)]
    assert [h["n"] for h in info["history"]] == [400, 400, 640, 640, 1024, 1024, 1638, 1638] + [2000] * 4
    assert info["stop_iter"] == -1


def test_switch_and_termination_wait_for_the_last_points(orc, disk):
    """t_add = 0 (never adds) and thresholds that would end a plain run at
    its first comparison: while points are missing nothing switches or
    stops, and the count never changes."""
    wl, og = disk
    prm = orc.default_params(fac_end=0.0)
    _, _, _, plain = orc.run_adaptive(og, wl.x[:800], wl.y[:800], "hybrid", 6, t_quality=INF, t_amax=INF,
                                      t_switch=INF, params=prm, nthreads=8)
    assert plain["switch_iter"] == 1
    x, _, _, info = orc.run_growing(og, wl.x, wl.y, "hybrid", 6, 800, t_add=0.0, t_quality=INF, t_amax=INF,
                                    t_switch=INF, params=prm, nthreads=8)
    assert info["adds"] == [] and info["switch_iter"] == -1 and info["stop_iter"] == -1
    assert info["iters"] == 6 and len(x) == 800
    assert all(h["n"] == 800 and h["method"] == "dm" for h in info["history"])
