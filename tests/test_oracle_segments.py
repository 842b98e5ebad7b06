"""Pins of the oracle's line-segment input (Sec. 3.2): the signed distance
to a closed clockwise loop of segments, checked against closed forms, an
independent inside test, dense sampling of the boundary and the tie rule."""
import math

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I


def box_sdf(x, y, x0, y0, x1, y1):
    """Textbook signed distance of an axis-aligned box."""
    ex, ey = max(x0 - x, x - x1), max(y0 - y, y - y1)
    if ex <= 0 and ey <= 0:
        return max(ex, ey)
    return math.hypot(max(ex, 0.0), max(ey, 0.0))


def winding_inside(verts, x, y):
    """Inside test by the total turning angle of the vertices seen from
    (x, y): +-2 pi inside a closed loop, 0 outside."""
    a = np.arctan2(verts[:, 1] - y, verts[:, 0] - x)
    d = np.diff(np.concatenate([a, a[:1]]))
    d = (d + np.pi) % (2 * np.pi) - np.pi
    return abs(d.sum()) > np.pi


def regular_cw(m, r, cx=0.0, cy=0.0, phase=0.1):
    th = phase - 2 * np.pi * np.arange(m) / m  # decreasing angles: clockwise
    return np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], 1)


def test_clockwise_square_is_the_box(orc):
    """Unit square as four clockwise segments: the box's signed distance
    inside, outside along the sides and outside the corners (where the
    nearest point is a vertex and the sign comes from the mean normal)."""
    sq = np.array([[0.0, 0.0], [0.0, 1.0], [1.0, 1.0], [1.0, 0.0]])
    rng = np.random.default_rng(7)
    pts = rng.uniform(-0.6, 1.6, (400, 2))
    pts = np.vstack([pts, [[0.5, 0.5], [-0.25, -0.25], [1.5, 1.25], [0.5, -0.75], [0.125, 0.5]]])
    for x, y in pts:
        d, _ = orc.segments_sdf(sq, x, y)
        assert d == pytest.approx(box_sdf(x, y, 0, 0, 1, 1), abs=1e-15), (x, y)


def test_sign_agrees_with_the_winding_number_and_distance_with_sampling(orc):
    """A regular 48-gon and the coast loop: the sign is the winding-number
    inside test, and |sdf| lies between the distance to a dense sample of
    the boundary minus its spacing and that distance (the sample is on the
    boundary, so it can only be farther)."""
    rng = np.random.default_rng(11)
    for verts in (regular_cw(48, 0.4, 0.5, 0.5), I.coast_loop(512)):
        nxt = np.roll(verts, -1, axis=0)
        u = np.linspace(0, 1, 401)
        samp = (verts[:, None, :] + u[None, :, None] * (nxt - verts)[:, None, :]).reshape(-1, 2)
        spacing = np.max(np.hypot(*(nxt - verts).T)) / 400
        for x, y in rng.uniform(0.0, 1.0, (200, 2)):
            d, _ = orc.segments_sdf(verts, x, y)
            ds = np.min(np.hypot(samp[:, 0] - x, samp[:, 1] - y))
            assert abs(d) <= ds + 1e-15 and abs(d) >= ds - spacing, (x, y, d, ds)
            if abs(d) > 1e-9:
                assert (d < 0) == winding_inside(verts, x, y), (x, y, d)


def test_reflex_and_convex_corners_use_the_vertex_normal(orc):
    """An L shape (clockwise).  Inside, below-left of its reflex corner (1, 1),
    both incident sides end at that vertex, so it is the nearest point and the
    value is minus the distance to it; beyond the convex corner (2, 0) the
    nearest point is that vertex and the value is plus the distance."""
    L = np.array([[0, 0], [0, 2], [1, 2], [1, 1], [2, 1], [2, 0]], np.float64)
    for t in (0.0625, 0.25, 0.375):  # dyadic: both sides' distances are exact, a true tie
        d, k = orc.segments_sdf(L, 1 - t, 1 - t / 2)
        assert d < 0 and abs(d) == pytest.approx(math.hypot(t, t / 2), rel=1e-15)
        assert k == 2  # segments 2 and 3 both end there: the lower index
    d, k = orc.segments_sdf(L, 2.3, -0.4)
    assert d == pytest.approx(0.5, rel=1e-15) and d > 0 and k == 4
    # in the notch outside the reflex corner: two sides at 0.2, tie to the lower
    d, k = orc.segments_sdf(L, 1.2, 1.2)
    assert d == pytest.approx(0.2, rel=1e-15) and d > 0 and k == 2


def test_equal_distances_go_to_the_lower_segment(orc):
    """The centre of the square is equally far from all four sides: the
    nearest segment reported is segment 0; a point on the diagonal near a
    corner is equally far from the two sides meeting there."""
    sq = np.array([[0.0, 0.0], [0.0, 1.0], [1.0, 1.0], [1.0, 0.0]])
    d, k = orc.segments_sdf(sq, 0.5, 0.5)
    assert d == -0.5 and k == 0
    d, k = orc.segments_sdf(sq, 0.75, 0.75)  # sides 1 (top) and 2 (right)
    assert d == -0.25 and k == 1


def test_segment_grid_is_the_pointwise_distance(orc):
    """The oracle grid of the coast workload: every node's value is the
    pointwise signed distance of the constructive geometry (loop minus disk),
    recomputed here from segments_sdf and the disk's closed form."""
    wl = I.coast(n=2000, segments=256, grid_n=64)
    og = orc.build_grid(wl)
    loop = wl.prims[0].poly
    g = wl.grid
    for j in range(0, g.ny, 7):
        for i in range(0, g.nx, 5):
            x, y = g.x0 + i * g.dx, g.y0 + j * g.dy
            s, _ = orc.segments_sdf(loop, x, y)
            t = math.hypot(x - 0.5, y - 0.5) - 0.05
            assert og.sdf[j * g.nx + i] == max(s, -t)


def test_needle_tip_needs_the_mean_normal(orc):
    """Beyond the tip of a thin clockwise needle the two sides' normals point
    almost opposite ways, and each alone calls one of these two mirrored
    points inside; their mean calls both outside, at the distance to the tip."""
    needle = np.array([[-0.01, 0.0], [0.0, 1.0], [0.01, 0.0]])
    for x in (0.005, -0.005):
        d, k = orc.segments_sdf(needle, x, 1.3)
        assert d > 0 and d == pytest.approx(math.hypot(x, 0.3), rel=1e-12), (x, d, k)
