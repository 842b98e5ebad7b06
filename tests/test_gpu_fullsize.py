"""Parity at the headline size: the holes20 workload with 10^6 points on its
4096^2 grid, in the configuration the benchmark times (3.2 points per bin,
the density its autotuner picks on the current kernels; the fused kernel with
its replays), every point and every triangle compared
with the oracle.  The grid is the oracle's, uploaded."""
import os

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def T():
    from paper_2309_13824_amd import trime
    trime.lib()
    return trime


@pytest.fixture(scope="module")
def full(orc):
    wl = I.holes20(n=1000000, grid_n=4096, iters=1)
    return wl, orc.build_grid(wl)


@pytest.fixture(scope="module")
def oracle_step(orc, full):
    wl, og = full
    cat0 = orc.initial_categories(og, wl.x, wl.y)
    return orc.cvd_step(og, wl.x, wl.y, cat0, np.full(wl.n, -1.0), nthreads=THREADS)


@pytest.fixture(scope="module")
def oracle_mesh(orc, full):
    wl, og = full
    return orc.triangulate(og, wl.x, wl.y, THREADS)


def mesher(wl, prec, grid):
    from paper_2309_13824_amd.mesher import Mesher
    m = Mesher(wl, precision=prec, grid=grid, bin_density=3.2)
    m.load()
    return m


def h_of(og, x, y):
    fx = np.floor((x - og.x0) * (1.0 / og.dx)).astype(int)
    fy = np.floor((y - og.y0) * (1.0 / og.dy)).astype(int)
    return og.hcell[fy * (og.nx - 1) + fx].astype(np.float64)


def sorted_tris(tri, valid):
    tri = np.asarray(tri, np.int64)
    order = np.lexsort((tri[:, 2], tri[:, 1], tri[:, 0]))
    return tri[order], np.asarray(valid)[order]


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_full_size_cvd_step_matches_oracle(orc, T, full, oracle_step, prec):
    """One CVD iteration from the seeded points: every position within
    1e-12 h (FP64) or 1e-5 h (FP32) of the oracle's, every category equal."""
    wl, og = full
    xr, yr, cr, _, _, _ = oracle_step
    m = mesher(wl, prec, og)
    m.step_cvd(1)
    x, y, c = m.points()
    err = np.hypot(x - xr, y - yr) / h_of(og, xr, yr)
    i = int(np.argmax(err))
    print("holes20 10^6 %s: position error against the oracle max %.3g h (point %d, category %d, moved %.3g h), "
          "mean %.3g h" % ("fp64" if prec == FP64 else "fp32", err[i], i, cr[i],
                           np.hypot(xr[i] - wl.x[i], yr[i] - wl.y[i]) / h_of(og, xr, yr)[i], err.mean()), flush=True)
    assert err.max() <= (1e-12 if prec == FP64 else 1e-5), err.max()
    assert np.array_equal(c, cr)
    assert m.stats_raw().error == 0


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_full_size_triangulation_matches_oracle(orc, T, full, oracle_mesh, prec):
    """The 2e6 triangles of the seeded points and their validity flags equal
    the oracle's."""
    wl, og = full
    ref = oracle_mesh
    m = mesher(wl, prec, og)
    m.bin()
    m.extract()
    tri, valid = m.triangles()
    assert len(tri) == len(ref.tri)
    a, av = sorted_tris(tri, valid)
    b, bv = sorted_tris(ref.tri, ref.valid)
    assert np.array_equal(a, b)
    assert np.array_equal(av, bv)
    assert m.stats_raw().error == 0


@pytest.fixture(scope="module")
def oracle_dm_step(orc, full, oracle_mesh):
    wl, og = full
    cat0 = orc.initial_categories(og, wl.x, wl.y)
    return orc.dm_step(og, wl.x, wl.y, cat0, oracle_mesh)


def compare_step(label, m, og, wl, xr, yr, cr, prec):
    x, y, c = m.points()
    err = np.hypot(x - xr, y - yr) / h_of(og, xr, yr)
    print("%s %s: position error against the oracle max %.3g h, mean %.3g h" % (
        label, "fp64" if prec == FP64 else "fp32", err.max(), err.mean()), flush=True)
    assert err.max() <= (1e-12 if prec == FP64 else 1e-5), err.max()
    assert np.array_equal(c, cr)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_full_size_dm_step_matches_oracle(orc, T, full, oracle_dm_step, prec):
    """One DistMesh iteration from the seeded points (triangulation, Eq. 3
    scaling, forces, Euler step, treatment): every position, every category,
    fac_mu and the count of points that moved beyond fac_retria h equal the
    oracle's."""
    wl, og = full
    xr, yr, cr, moved, fm, _ = oracle_dm_step
    m = mesher(wl, prec, og)
    m.step_dm(1)
    compare_step("holes20 10^6 DistMesh", m, og, wl, xr, yr, cr, prec)
    st = m.stats()
    assert st["fac_mu"] == pytest.approx(fm, rel=1e-12 if prec == FP64 else 1e-6)
    assert st["moved"] == moved
    assert st["error"] == 0


@pytest.fixture(scope="module")
def ellipses(orc):
    """The ellipses recipe (the unit square minus 200 elliptical holes,
    hole-ramp sizing 1:10) at 2e6 points on a 1024^2 grid: the oracle builds
    its grid node by node against all 200 holes, which at the recipe's 8192^2
    would take hours."""
    wl = I.ellipses(n=2000000, grid_n=1024)
    return wl, orc.build_grid(wl)


@pytest.fixture(scope="module")
def ellipses_ref(orc, ellipses):
    wl, og = ellipses
    cat0 = orc.initial_categories(og, wl.x, wl.y)
    mesh = orc.triangulate(og, wl.x, wl.y, THREADS)
    dm = orc.dm_step(og, wl.x, wl.y, cat0, mesh)
    cvd = orc.cvd_step(og, wl.x, wl.y, cat0, np.full(wl.n, -1.0), nthreads=THREADS)
    return {"dm": dm, "cvd": cvd}


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("method", ["dm", "cvd"])
def test_ellipses_one_step_matches_oracle(orc, T, ellipses, ellipses_ref, method, prec):
    """The first iteration of each method of the ellipses schedule (70
    DistMesh then 30 CVD) at 2e6 points: positions within 1e-12 h (FP64) or
    1e-5 h (FP32) of the oracle's, categories equal (and for DistMesh fac_mu
    and the moved count)."""
    wl, og = ellipses
    ref = ellipses_ref[method]
    m = mesher(wl, prec, og)
    if method == "dm":
        m.step_dm(1)
    else:
        m.step_cvd(1)
    compare_step("ellipses 2e6 %s" % method, m, og, wl, ref[0], ref[1], ref[2], prec)
    st = m.stats()
    if method == "dm":
        assert st["fac_mu"] == pytest.approx(ref[4], rel=1e-12 if prec == FP64 else 1e-6)
        assert st["moved"] == ref[3]
    assert st["error"] == 0
