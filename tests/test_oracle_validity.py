"""Pins of the oracle's triangle validity (Procedure I's check; Sec. 4.1 Tests
1-3, with the reading count >= 2 valid, 0 invalid, 1 -> Test 3).

Every case is built by hand on a small grid whose node sdf is the affine
function x - 0.3 (bilinear interpolation reproduces it exactly), whose cell
categories are painted by the cell midpoint's x (inner below 0.1875,
boundary in [0.1875, 0.375), outer from 0.375), and whose h is 0.1 in every
cell, so geps = 0.01 min(h, h_avg) = 0.001.  The expected validity of each
triangle follows from the paper's rule and the construction, stated case by
case; nothing here re-evaluates the oracle's formulas.
"""
import math

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I

DX = 1.0 / 16.0
INNER, BOUNDARY, OUTER = 1, 2, 0


def hand_grid(orc, ny=65):
    """65 x ny nodes from (-2, -2), spacing 1/16."""
    nx = 65
    spec = I.GridSpec(nx, ny, -2.0, -2.0, DX, DX, 8)
    xs = -2.0 + np.arange(nx) * DX
    sdf = np.tile(xs - 0.3, ny)
    mid = -2.0 + (np.arange(nx - 1) + 0.5) * DX
    row = np.where(mid < 0.1875, INNER, np.where(mid < 0.375, BOUNDARY, OUTER)).astype(np.uint8)
    cat = np.tile(row, ny - 1)
    hcell = np.full((nx - 1) * (ny - 1), 0.1, np.float32)
    return orc.grid_from_arrays(spec, sdf, np.ones(nx * ny), cat, hcell, 0.1)


def valid(orc, g, pts, **prm):
    x = np.array([p[0] for p in pts], float)
    y = np.array([p[1] for p in pts], float)
    params = orc.default_params(**prm) if prm else None
    return orc.triangle_valid(g, x, y, 0, 1, 2, params)


def mids(pts):
    (ax, ay), (bx, by), (cx, cy) = pts
    return [((ax + bx) / 2, (ay + by) / 2), ((bx + cx) / 2, (by + cy) / 2), ((ax + cx) / 2, (ay + cy) / 2)]


def category(x, y, ymax=2.0):
    """Category of the cell holding (x, y) in the painted grid, None off it."""
    if not (-2.0 <= x < 2.0 and -2.0 <= y < ymax):
        return None
    i = math.floor((x + 2.0) / DX)
    m = -2.0 + (i + 0.5) * DX
    return INNER if m < 0.1875 else (BOUNDARY if m < 0.375 else OUTER)


def counted(x, y, ymax=2.0):
    """Test 2's count of one midpoint: an inner cell, or a boundary cell with
    sdf = x - 0.3 <= geps = 0.001."""
    c = category(x, y, ymax)
    return c == INNER or (c == BOUNDARY and x - 0.3 <= 0.001)


def test_construction_is_what_the_cases_assume(orc):
    g = hand_grid(orc)
    assert float(g.hcell[0]) == pytest.approx(0.1) and g.h_avg == 0.1
    # the painted categories sit where `category` says
    for x in (-1.0, 0.0, 0.18, 0.19, 0.3, 0.37, 0.38, 1.5):
        i = math.floor((x + 2.0) / DX)
        assert g.cat[32 * 64 + i] == category(x, 0.01)


def test_test1_centroid_decides(orc):
    g = hand_grid(orc)
    assert valid(orc, g, [(0.0, 0.0), (0.05, 0.0), (0.0, 0.05)]) == 1    # centroid in an inner cell
    assert valid(orc, g, [(0.5, 0.0), (0.55, 0.0), (0.5, 0.05)]) == 0    # centroid in an outer cell
    assert valid(orc, g, [(2.5, 0.0), (2.6, 0.0), (2.5, 0.1)]) == 0      # centroid off the grid
    # centroid x = 0.31 in a boundary cell: sdf = 0.01 > geps
    assert valid(orc, g, [(0.30, 0.0), (0.33, 0.0), (0.30, 0.03)]) == 0


@pytest.mark.parametrize("mode", [0, 1])
def test_test2_count_three_and_two_are_valid(orc, mode):
    g = hand_grid(orc)
    three = [(0.27, 0.0), (0.29, 0.02), (0.31, 0.0)]   # centroid x 0.29; midpoints x 0.28, 0.30, 0.29
    two = [(0.26, 0.0), (0.30, 0.03), (0.34, 0.0)]     # centroid x 0.30; midpoints x 0.28, 0.32, 0.30
    assert sum(counted(*m) for m in mids(three)) == 3
    assert sum(counted(*m) for m in mids(two)) == 2
    assert valid(orc, g, three, test2_mode=mode) == 1
    assert valid(orc, g, two, test2_mode=mode) == 1


@pytest.mark.parametrize("mode", [0, 1])
def test_test2_count_zero_is_invalid(orc, mode):
    """Large triangles whose centroid (x 0.29: boundary cell, sdf -0.01)
    passes Test 1 while no midpoint counts: all three off the grid, or two
    in outer cells and one off the grid."""
    g = hand_grid(orc)
    off = [(-5.13, -2.4), (5.71, -2.6), (0.29, 5.0)]   # midpoints (0.29,-2.5) (3,1.2) (-2.42,1.3)
    outer = [(-2.93, -2.0), (6.73, 0.0), (-2.93, 2.0)]  # midpoints (1.9,-1) (1.9,1) (-2.93,0)
    for pts in (off, outer):
        cx = sum(p[0] for p in pts) / 3
        assert category(cx, sum(p[1] for p in pts) / 3) == BOUNDARY and cx - 0.3 <= 0.001
        assert sum(counted(*m) for m in mids(pts)) == 0
        assert valid(orc, g, pts, test2_mode=mode) == 0


def isosceles(ratio):
    """a = (0, -w), b = (0, w), c = (0.7, 0): the circumcentre (x_cc, 0)
    solves x_cc^2 + w^2 = (0.7 - x_cc)^2, R = 0.7 - x_cc, and for x_cc < 0.3
    |sdf(cc)| / R = (0.3 - x_cc) / (0.7 - x_cc) = 1 - 0.4 / (0.7 - x_cc);
    w is chosen to give `ratio`.  Centroid (0.233, 0): boundary cell, sdf
    -0.067; midpoints (0, 0) inner (counts), (0.35, +-w/2) boundary with sdf
    0.05 > geps: count 1."""
    xcc = 0.7 - 0.4 / (1.0 - ratio)
    w = math.sqrt(0.49 - 1.4 * xcc)
    return [(0.0, -w), (0.0, w), (0.7, 0.0)]


@pytest.mark.parametrize("ratio,expect", [(0.1, 1), (0.3, 1), (0.39, 1), (0.41, 0), (0.6, 0)])
def test_test3_circumcentre_ratio(orc, ratio, expect):
    g = hand_grid(orc)
    pts = isosceles(ratio)
    assert sum(counted(*m) for m in mids(pts)) == 1
    assert valid(orc, g, pts) == expect
    # the alternative reading of Test 2 discards every count-1 triangle
    assert valid(orc, g, pts, test2_mode=1) == 0
    # a larger threshold T_tria keeps it
    assert valid(orc, g, pts, T_tria=0.7) == 1


def test_test3_ratio_with_positive_sdf(orc):
    """w = 0.1: x_cc = (0.49 - 0.01) / 1.4 = 0.3429 > 0.3, R = 0.3571,
    |sdf| / R = 0.0429 / 0.3571 = 0.12: valid."""
    g = hand_grid(orc)
    pts = [(0.0, -0.1), (0.0, 0.1), (0.7, 0.0)]
    assert sum(counted(*m) for m in mids(pts)) == 1
    assert valid(orc, g, pts) == 1
    assert valid(orc, g, pts, T_tria=0.1) == 0


def test_test3_circumcentre_off_grid_is_invalid(orc):
    """Three points on the circle of radius 3 about (0.3, 3): the
    circumcentre has sdf 0 (ratio 0) but lies above the grid (y < 2), so the
    triangle is invalid; on a grid reaching y = 6 it is valid."""
    def on_circle(phi):
        return (0.3 + 3.0 * math.sin(phi), 3.0 - 3.0 * math.cos(phi))
    pts = [on_circle(-0.12), on_circle(-0.08), on_circle(0.16)]
    cx, cy = sum(p[0] for p in pts) / 3, sum(p[1] for p in pts) / 3
    assert category(cx, cy) == BOUNDARY and cx - 0.3 <= 0.001
    assert sum(counted(*m) for m in mids(pts)) == 1
    assert valid(orc, hand_grid(orc), pts) == 0
    tall = hand_grid(orc, ny=129)  # y up to 6
    assert sum(counted(*m, ymax=6.0) for m in mids(pts)) == 1
    assert valid(orc, tall, pts) == 1
