"""Pins of the oracle's automatic sizing field (Sec. 3.3, Eq. 8; App. A):
boundary points of segment loops, medial-axis points from Voronoi poles,
their trimming, lfs and mu, against closed forms on a circle and a square,
small hand-made cases and the Lipschitz property of Eq. 8."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I


def loop_workload(verts, grid_n=128, K=0.1, fac_s=0.5):
    prims = [I.Prim(I.OP_INIT, I.PRIM_SEGMENTS, (), np.asarray(verts, np.float64))]
    grid = I.centred_grid(grid_n, 17, int(round(math.log2(grid_n))) + 4, 0.5, 8)
    return I.Workload("loop", prims, I.Sizing(I.SZ_AUTO, K, fac_s), grid, 1000, [], 0)


def circle(m, r=0.4, cx=0.5, cy=0.5):
    th = 0.1 - 2 * np.pi * np.arange(m) / m  # clockwise
    return np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], 1)


def test_boundary_points_split_long_segments_evenly(orc):
    """Every vertex, and floor(L / d_s) evenly spaced points inside each
    segment longer than d_s: all on the loop, spacing below d_s."""
    sq = np.array([[0.2, 0.2], [0.2, 0.8], [0.8, 0.8], [0.8, 0.2]])
    wl = loop_workload(sq, fac_s=0.5)
    au = orc.auto_sizing(wl, trim=False)
    per_side = math.floor(0.6 / au.d_s) + 1
    assert len(au.s) == 4 * per_side
    for k in range(4):
        a, b = sq[k], sq[(k + 1) % 4]
        pts = au.s[k * per_side:(k + 1) * per_side]
        assert np.array_equal(pts[0], a)
        t = np.linspace(0, 1, per_side + 1)[:-1]
        assert np.allclose(pts, a + t[:, None] * (b - a), rtol=0, atol=1e-15)
    step = np.hypot(*np.diff(np.vstack([au.s, au.s[:1]]), axis=0).T)
    assert step.max() < au.d_s


def test_circle_poles_meet_at_the_centre(orc):
    """Points exactly on a circle (no point inside a chord: d_s above the
    chord length): every Voronoi cell is a wedge whose one finite vertex is
    the centre, so every medial point is the centre, all are kept, lfs = R,
    and mu at the centre is K R + R."""
    R, K = 0.4, 0.1
    verts = circle(96, R)
    chord = 2 * R * math.sin(math.pi / 96)
    wl = loop_workload(verts, grid_n=128, K=K, fac_s=1.1 * chord / (17 * 2.0 ** -(7 + 4)))
    au = orc.auto_sizing(wl, trim=False)
    assert len(au.s) == 96 and au.d_s > chord
    assert len(au.medial) == 96
    assert np.allclose(au.medial, [0.5, 0.5], rtol=0, atol=1e-12)
    assert au.keep.all()
    assert np.allclose(au.lfs, R, rtol=1e-12)
    s_pts = np.ascontiguousarray(au.s.reshape(-1))
    lfs = np.ascontiguousarray(au.lfs)
    dp = C.POINTER(C.c_double)
    mu_c = orc.lib().orc_auto_mu(s_pts.ctypes.data_as(dp), lfs.ctypes.data_as(dp), len(au.s), K, 0.5, 0.5)
    assert mu_c == pytest.approx(K * R + R, rel=1e-12)


def dist_to_segment(p, a, b):
    ab = b - a
    t = np.clip(((p - a) @ ab) / (ab @ ab), 0, 1)
    return np.linalg.norm(p - (a + t[:, None] * ab), axis=1)


def test_square_medial_axis_is_its_diagonals(orc):
    """A square: with evenly split sides (no trimming) every kept medial
    point lies on a diagonal (its medial axis) and lfs of a boundary point
    is its distance to the diagonals within the spacing d_s; after trimming
    (uneven spacing) both hold within d_s and 2 d_s."""
    sq = np.array([[0.2, 0.2], [0.2, 0.8], [0.8, 0.8], [0.8, 0.2]])
    for trimmed, tol_axis, tol_lfs in ((False, 1e-12, 1.0), (True, 1.0, 2.0)):
        au = orc.auto_sizing(loop_workload(sq), trim=trimmed)
        m = au.medial[au.keep.astype(bool)]
        assert len(m) > 0
        off = np.minimum(np.abs((m[:, 0] - 0.5) - (m[:, 1] - 0.5)), np.abs((m[:, 0] - 0.5) + (m[:, 1] - 0.5)))
        assert off.max() <= (tol_axis if not trimmed else tol_axis * au.d_s)
        ref = np.minimum(dist_to_segment(au.s, np.array([0.2, 0.2]), np.array([0.8, 0.8])),
                         dist_to_segment(au.s, np.array([0.2, 0.8]), np.array([0.8, 0.2])))
        assert np.max(np.abs(au.lfs - ref)) < tol_lfs * au.d_s


def test_trimming_drops_isolated_points(orc):
    """Two clusters of four points within r_nei and two isolated points:
    with n_thres = 3 the cluster points (3 neighbours each) stay, the
    isolated ones go; with n_thres = 4 nothing stays."""
    pts = np.array([[0, 0], [0.01, 0], [0, 0.01], [0.01, 0.01],
                    [1, 1], [1.01, 1], [1, 1.01], [1.01, 1.01],
                    [0.5, 0.5], [0.3, 0.8]], np.float64)
    m = np.ascontiguousarray(pts.reshape(-1))
    keep = np.zeros(10, np.uint8)
    dp = C.POINTER(C.c_double)
    kept = orc.lib().orc_trim_medial(m.ctypes.data_as(dp), 10, 0.05, 3, keep.ctypes.data_as(C.POINTER(C.c_uint8)))
    assert kept == 8 and keep.tolist() == [1] * 8 + [0, 0]
    kept = orc.lib().orc_trim_medial(m.ctypes.data_as(dp), 10, 0.05, 4, keep.ctypes.data_as(C.POINTER(C.c_uint8)))
    assert kept == 0


def test_mu_is_k_lipschitz_and_below_lfs_on_the_boundary(orc):
    """Eq. 8 on the coast loop: |mu(x) - mu(y)| <= K |x - y| for random
    pairs, and mu(s) <= lfs(s) at every boundary point."""
    loop = I.coast_loop(300)
    K = 0.2
    au = orc.auto_sizing(loop_workload(loop, K=K))
    s_pts = np.ascontiguousarray(au.s.reshape(-1))
    lfs = np.ascontiguousarray(au.lfs)
    dp = C.POINTER(C.c_double)
    f = lambda x, y: orc.lib().orc_auto_mu(s_pts.ctypes.data_as(dp), lfs.ctypes.data_as(dp), len(au.s), K, x, y)  # noqa
    rng = np.random.default_rng(3)
    for (x0, y0), (x1, y1) in rng.uniform(0.1, 0.9, (200, 2, 2)):
        assert abs(f(x0, y0) - f(x1, y1)) <= K * math.hypot(x1 - x0, y1 - y0) * (1 + 1e-12) + 1e-15
    for k in range(0, len(au.s), 7):
        assert f(*au.s[k]) <= au.lfs[k]


def test_grid_mu_is_the_field_at_the_nodes(orc):
    """The grid built with automatic sizing carries mu(node) at every node
    (spot checks against the pointwise field)."""
    wl = loop_workload(circle(64, 0.35), grid_n=64, K=0.15)
    og = orc.build_grid(wl)
    au = orc.auto_sizing(wl)
    s_pts = np.ascontiguousarray(au.s.reshape(-1))
    lfs = np.ascontiguousarray(au.lfs)
    dp = C.POINTER(C.c_double)
    g = wl.grid
    for j in range(0, g.ny, 9):
        for i in range(0, g.nx, 7):
            x, y = g.x0 + i * g.dx, g.y0 + j * g.dy
            want = orc.lib().orc_auto_mu(s_pts.ctypes.data_as(dp), lfs.ctypes.data_as(dp), len(au.s), 0.15, x, y)
            assert og.mu[j * g.nx + i] == want


def trim(orc, prims_wl, pts, d_s, geps):
    from oracle.oracle import _geometry, _p
    prims, _, poly, keep = _geometry(prims_wl)
    p = np.ascontiguousarray(np.asarray(pts, np.float64).reshape(-1))
    n = orc.lib().orc_trim_boundary(prims, len(prims_wl.prims), _p(poly, C.c_double), d_s, geps,
                                    p.ctypes.data_as(C.POINTER(C.c_double)), len(p) // 2)
    return p[:2 * n].reshape(-1, 2)


def test_trimming_by_hand():
    """Four points 0.3 d_s apart on the bottom side of a large square (the
    rest far away): sweep 1 merges 0 with 1 (to 0.15) and 2 with 3 (to 0.75),
    sweep 2 merges them (to 0.45), sweep 3 changes nothing."""
    from oracle import oracle as orc
    sq = np.array([[0.0, 0.0], [0.0, 8.0], [8.0, 8.0], [8.0, 0.0]])
    wl = loop_workload(sq)
    d_s = 0.125
    pts = [[4 + 0.3 * d_s * k, 0.0] for k in range(4)]
    out = trim(orc, wl, pts, d_s, 1e-9)
    assert out.shape == (1, 2)
    assert out[0, 0] == pytest.approx(4 + 0.45 * d_s, rel=1e-15) and out[0, 1] == 0.0


def test_trimmed_points_keep_a_valid_spacing_of_d_s(orc):
    """After trimming, no two remaining points closer than d_s have their
    midpoint on the boundary, and every point stays within geps of it."""
    for verts in (np.array([[0.2, 0.2], [0.2, 0.8], [0.8, 0.8], [0.8, 0.2]]), I.coast_loop(400)):
        wl = loop_workload(verts, fac_s=0.5)
        au = orc.auto_sizing(wl)
        raw = orc.auto_sizing(wl, trim=False)
        assert len(au.s) < len(raw.s)
        geps = 0.01 * min(wl.grid.dx, wl.grid.dy)
        dist = lambda x, y: abs(orc.segments_sdf(verts, x, y)[0])  # noqa: E731
        s = au.s
        for i in range(len(s)):
            assert dist(*s[i]) <= geps
            d = np.hypot(s[:, 0] - s[i, 0], s[:, 1] - s[i, 1])
            for j in np.nonzero((d < au.d_s) & (np.arange(len(s)) != i))[0]:
                assert dist(*(0.5 * (s[i] + s[j]))) > geps, (i, j)


def test_boundary_points_of_a_constructive_geometry(orc):
    """A box minus a disk inside it and minus a disk across its edge: the
    inner disk keeps every sample, the crossing disk only the samples inside
    the box (about the share of its circle there), the box loses its samples
    inside the crossing disk, and every kept point has |sdf| <= geps."""
    prims = [I.Prim(I.OP_INIT, I.PRIM_BOX, (0.2, 0.2, 0.8, 0.8)),
             I.Prim(I.OP_DIFF, I.PRIM_DISK, (0.4, 0.5, 0.1)),
             I.Prim(I.OP_DIFF, I.PRIM_DISK, (0.8, 0.5, 0.1))]
    grid = I.centred_grid(128, 17, 11, 0.5, 8)
    wl = I.Workload("csg", prims, I.Sizing(I.SZ_AUTO, 0.1, 0.5), grid, 1000, [], 0)
    au = orc.auto_sizing(wl, trim=False)
    s = au.s
    geps = 0.01 * grid.dx
    for x, y in s:
        assert abs(orc.sdf_eval(wl, x, y)) <= geps
    r_in = np.hypot(s[:, 0] - 0.4, s[:, 1] - 0.5)
    r_x = np.hypot(s[:, 0] - 0.8, s[:, 1] - 0.5)
    m_disk = math.floor(2 * math.pi * 0.1 / au.d_s) + 1
    assert np.count_nonzero(np.abs(r_in - 0.1) < 1e-12) == m_disk
    on_x = np.abs(r_x - 0.1) < 1e-12
    assert abs(np.count_nonzero(on_x) - m_disk / 2) <= 2
    assert np.all(s[on_x, 0] <= 0.8 + 1e-12)
    on_box_right = (np.abs(s[:, 0] - 0.8) < 1e-12) & ~on_x
    assert np.all(np.abs(s[on_box_right, 1] - 0.5) >= 0.1 - 1e-12)
