"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Both sides receive the same seeded positions and the same geometry-grid
arrays (the GPU-built grid, itself checked against the oracle's grid).
Connectivity must match bit for bit; positions after one step within
1e-12 h (FP64) and 1e-5 h (FP32), h the local target spacing.
"""
import math

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


@pytest.fixture(scope="module")
def T():
    from paper_2309_13824_amd import trime
    trime.lib()
    return trime


def mesher(wl, prec, **kw):
    from paper_2309_13824_amd.mesher import Mesher
    m = Mesher(wl, precision=prec, **kw)
    m.load()
    return m


def oracle_grid(orc, m):
    sdf, mu, cat, hcell, scal = m.grid_arrays()
    return orc.grid_from_arrays(m.wl.grid, sdf, mu, cat, hcell, scal[1])


def tri_set(tri, valid=None):
    out = {}
    for k, t in enumerate(tri):
        out[tuple(int(v) for v in t)] = None if valid is None else int(valid[k])
    return out


def h_of(og, x, y):
    fx = np.floor((x - og.x0) * (1.0 / og.dx)).astype(int)
    fy = np.floor((y - og.y0) * (1.0 / og.dy)).astype(int)
    return og.hcell[fy * (og.nx - 1) + fx].astype(np.float64)


# ------------------------------------------------------------------ grid --

@pytest.mark.parametrize("make", [lambda: I.disk(), lambda: I.holes20(n=20000, grid_n=512, iters=1),
                                  lambda: I.annulus(n=5000, grid_n=256)])
def test_grid_build_matches_oracle(orc, T, make):
    wl = make()
    m = mesher(wl, FP64)
    sdf, mu, cat, hcell, scal = m.grid_arrays()
    og = orc.build_grid(wl)
    rel = 4e-7 if wl.grid.dtype_bytes == 4 else 1e-15
    assert np.max(np.abs(sdf - og.sdf) / (np.abs(og.sdf) + 1e-300)) <= rel
    assert np.max(np.abs(mu - og.mu) / np.abs(og.mu)) <= rel
    assert np.array_equal(cat, og.cat)
    assert scal[0] == pytest.approx(og.H, rel=1e-13)
    assert scal[1] == pytest.approx(og.h_avg, rel=1e-12)
    # h_cell within one float32 ulp of the oracle's
    assert np.all(np.abs(hcell.view(np.int32) - og.hcell.view(np.int32)) <= 1)


# ----------------------------------------------------------------- cells --

@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("make", [lambda: I.disk(), lambda: I.random_box(500, seed=3),
                                  lambda: I.holes20(n=6000, grid_n=512, iters=1)])
def test_cells_match_oracle(orc, T, prec, make):
    wl = make()
    m = mesher(wl, prec)
    m.bin()
    got = m.cells()
    og = oracle_grid(orc, m)
    ref, _ = orc.cells(og, wl.x, wl.y)
    assert got == ref


def test_square_lattice_exact_ties(orc, T):
    """Exactly cocircular lattice: the cells come from the exact stage with
    the symbolic tie-break and must equal the oracle's bit for bit."""
    wl = I.square_lattice(8, 0.125)
    m = mesher(wl, FP32)
    m.bin()
    got = m.cells()
    og = oracle_grid(orc, m)
    ref, _ = orc.cells(og, wl.x, wl.y)
    assert got == ref
    st = m.stats()
    assert st["exact_calls"] > 0


# -------------------------------------------------------------- extraction --

@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("make", [lambda: I.disk(), lambda: I.holes20(n=8000, grid_n=512, iters=1),
                                  lambda: I.annulus(n=6000, grid_n=256)])
def test_triangles_and_adjacency_match_oracle(orc, T, prec, make):
    wl = make()
    m = mesher(wl, prec)
    m.bin()
    m.extract()
    tri, valid = m.triangles()
    adj = m.adjacency()
    og = oracle_grid(orc, m)
    ref = orc.triangulate(og, wl.x, wl.y)
    assert tri_set(tri, valid) == tri_set(ref.tri, ref.valid)
    rows = [tuple(int(v) for v in ref.col[ref.rowptr[i]:ref.rowptr[i + 1]]) for i in range(wl.n)]
    assert adj == rows
    st = m.stats()
    assert st["ntri"] == len(ref.tri) and st["nvalid"] == int(ref.valid.sum())
    q = orc.quality(wl.x, wl.y, ref.tri, ref.valid)
    assert st["half_mean_alpha"] == pytest.approx(q["half_mean_alpha"], rel=1e-12)
    assert st["min_q"] == pytest.approx(q["min_q"], rel=1e-12)


# --------------------------------------------------------------- one step --

def _tol(prec):
    return 1e-12 if prec == FP64 else 1e-5


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_dm_one_step_matches_oracle(orc, T, prec):
    wl = I.disk()
    m = mesher(wl, prec)
    m.step_dm(1)
    x, y, cat = m.points()
    og = oracle_grid(orc, m)
    mesh = orc.triangulate(og, wl.x, wl.y)
    cat0 = orc.initial_categories(og, wl.x, wl.y)
    xr, yr, cr, moved, fm, _ = orc.dm_step(og, wl.x, wl.y, cat0, mesh)
    h = h_of(og, xr, yr)
    err = np.hypot(x - xr, y - yr) / h
    assert err.max() <= _tol(prec), err.max()
    assert np.array_equal(cat, cr)
    st = m.stats()
    assert st["fac_mu"] == pytest.approx(fm, rel=1e-12 if prec == FP64 else 1e-6)
    assert st["moved"] == moved


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("make", [lambda: I.holes20(n=8000, grid_n=512, iters=1),
                                  lambda: I.annulus(n=6000, grid_n=256)])
def test_cvd_one_step_matches_oracle(orc, T, prec, make):
    wl = make()
    m = mesher(wl, prec)
    m.step_cvd(1)
    x, y, cat = m.points()
    og = oracle_grid(orc, m)
    cat0 = orc.initial_categories(og, wl.x, wl.y)
    xr, yr, cr, dr, lev, _ = orc.cvd_step(og, wl.x, wl.y, cat0, np.full(wl.n, -1.0), nthreads=8)
    h = h_of(og, xr, yr)
    err = np.hypot(x - xr, y - yr) / h
    assert err.max() <= _tol(prec), err.max()
    assert np.array_equal(cat, cr)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_cvd_three_steps_match_oracle(orc, T, prec):
    """Several iterations: the GPU state after each step is the input of the
    oracle's next step (one-step replay along the GPU trajectory)."""
    wl = I.holes20(n=5000, grid_n=512, iters=1)
    m = mesher(wl, prec)
    og = oracle_grid(orc, m)
    x, y = wl.x.copy(), wl.y.copy()
    cat = orc.initial_categories(og, x, y)
    dprev = np.full(wl.n, -1.0)
    for it in range(3):
        m.step_cvd(1)
        gx, gy, gc = m.points()
        xr, yr, cr, dr, lev, _ = orc.cvd_step(og, x, y, cat, dprev, nthreads=8)
        err = np.hypot(gx - xr, gy - yr) / h_of(og, xr, yr)
        assert err.max() <= _tol(prec), (it, err.max())
        assert np.array_equal(gc, cr)
        # continue the oracle from the GPU state (positions within tolerance)
        x, y, cat, dprev = gx, gy, gc, np.hypot(gx - x, gy - y)
