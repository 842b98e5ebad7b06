"""Pins of the oracle's quality statistics (Eq. 10-11), sizing fields and h
field (Sec. 3.3, 3.7), the DistMesh scaling factor with mu at the edge
midpoints (Eq. 3), and the AND rule when octagons bind (Sec. 4.1).

Expected values come from closed forms of hand-made configurations,
invariants of the definitions, or a brute-force Delaunay triangulation in
rational arithmetic; none re-runs the oracle's own code path.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I
from tests import exact_ref as X


# ------------------------------------------------------- Eq. 10-11 stats --

def right_alpha(a, b):
    """alpha = R / (2 r) of a right triangle with legs a, b: R = c / 2,
    r = (a + b - c) / 2."""
    c = math.hypot(a, b)
    return (c / 2) / (a + b - c)


def test_quality_statistics_closed_forms(orc):
    """An equilateral triangle (alpha = beta = 1), a right isosceles one
    (alpha = sqrt2 / (2 (2 - sqrt2)), beta = sqrt2), a right triangle with
    legs 4 and 1 (beta = sqrt17 / 1 > 3: the open last bin) and one invalid
    triangle that must be left out."""
    x = np.array([0.0, 1.0, 0.5, 2.0, 3.0, 2.0, 4.0, 8.0, 4.0, 10.0, 10.1, 10.0])
    y = np.array([0.0, 0.0, math.sqrt(3) / 2, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 5.0])
    tri = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11]], np.int32)
    valid = np.array([1, 1, 1, 0], np.uint8)
    q = orc.quality(x, y, tri, valid)
    a2 = math.sqrt(2) / (2 * (2 - math.sqrt(2)))
    assert a2 == pytest.approx(right_alpha(1, 1), rel=1e-15)
    a3 = right_alpha(4, 1)
    b3 = math.sqrt(17)
    assert q["ntri"] == 3
    # Eq. 11 with p = 1/2: M = (mean of x^(1/2))^2
    assert q["half_mean_alpha"] == pytest.approx(((1 + math.sqrt(a2) + math.sqrt(a3)) / 3) ** 2, rel=1e-14)
    assert q["half_mean_beta"] == pytest.approx(((1 + 2 ** 0.25 + math.sqrt(b3)) / 3) ** 2, rel=1e-14)
    assert q["max_alpha"] == pytest.approx(a3, rel=1e-14)
    assert q["min_q"] == pytest.approx(1 / a3, rel=1e-14)
    assert q["mean_q"] == pytest.approx((1 + 1 / a2 + 1 / a3) / 3, rel=1e-14)
    # beta histogram: 40 bins of width 0.05 on [1, 3), the last one open;
    # beta 1 -> bin 0, sqrt2 = 1.414 -> bin 8, sqrt17 -> bin 39
    h = q["hist_beta"]
    ref = np.zeros(40)
    ref[[0, 8, 39]] = 1 / 3
    assert np.allclose(h, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("edge", [1e-3, 1e-9, 1e-13])
def test_quality_histogram_last_bin_holds_any_large_beta(orc, edge):
    """A valid triangle with one edge far shorter than the others: beta =
    longest / shortest edge is ~1e3, ~1e9 or ~1e13, beyond the range of an
    int once scaled to a bin index, and still counts in the open last bin."""
    x = np.array([0.0, edge, 0.5])
    y = np.array([0.0, 0.0, 1.0])
    tri = np.array([[0, 1, 2]], np.int32)
    q = orc.quality(x, y, tri, np.array([1], np.uint8))
    beta = math.hypot(0.5, 1.0) / edge
    assert q["half_mean_beta"] == pytest.approx(beta, rel=1e-9)
    ref = np.zeros(40)
    ref[39] = 1.0
    assert np.array_equal(q["hist_beta"], ref)


def test_quality_half_mean_between_mean_and_geometric_mean(orc):
    """M_1/2 of Eq. 11 lies between the geometric and the arithmetic mean
    (power-mean inequality), equal to both only for equal values."""
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 1, (60, 2))
    tri = np.array([[3 * k, 3 * k + 1, 3 * k + 2] for k in range(20)], np.int32)
    t = tri.copy()
    ax, ay = pts[t[:, 0]].T
    bx, by = pts[t[:, 1]].T
    cx, cy = pts[t[:, 2]].T
    cw = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
    t[cw < 0] = t[cw < 0][:, [0, 2, 1]]
    q = orc.quality(pts[:, 0], pts[:, 1], t)
    al = np.array([orc.triangle_quality(pts[a], pts[b], pts[c])[0] for a, b, c in t])
    assert math.exp(np.log(al).mean()) < q["half_mean_alpha"] < al.mean()
    assert q["max_alpha"] == pytest.approx(al.max(), rel=1e-15)


# ------------------------------------------------------------ sizing nodes --

def box_workload(sizing, n=1000, nodes=33, lo=0.0, step=1.0 / 32):
    """A box covering the whole node grid (nodes x nodes from lo, spacing
    step), FP64 nodes."""
    grid = I.GridSpec(nodes, nodes, lo, lo, step, step, 8)
    hi = lo + (nodes - 1) * step
    prims = [I.Prim(I.OP_INIT, I.PRIM_BOX, (lo - 1.0, lo - 1.0, hi + 1.0, hi + 1.0))]
    return I.Workload("box", prims, sizing, grid, n, [], 0)


def node_value(g, field, x, y):
    i = int(round((x - g.x0) / g.dx))
    j = int(round((y - g.y0) / g.dy))
    assert g.x0 + i * g.dx == x and g.y0 + j * g.dy == y
    return field[j * g.nx + i]


def test_gauss_density_nodes(orc):
    """rho = a0 + a1 sum_k exp(-|x - c_k|^2 / s2), mu = rho^-1/2 (the
    headline workload's density): a centre on a node gives rho = a0 + a1
    there; at distance d with s2 = d^2 / ln 2 the term is exactly 1/2; far
    away rho -> a0; two centres on one node add (a sum, not a max)."""
    d = 0.125
    s2 = d * d / math.log(2.0)
    one = I.Sizing(I.SZ_GAUSS_RHO, a0=1.0, a1=4.0, s2=s2, cent=np.array([[0.5, 0.5]]))
    g = orc.build_grid(box_workload(one))
    assert node_value(g, g.mu, 0.5, 0.5) == pytest.approx(1 / math.sqrt(5.0), rel=1e-15)
    assert node_value(g, g.mu, 0.5 + d, 0.5) == pytest.approx(1 / math.sqrt(3.0), rel=1e-14)
    assert node_value(g, g.mu, 0.5, 0.5 - d) == pytest.approx(1 / math.sqrt(3.0), rel=1e-14)
    assert node_value(g, g.mu, 0.0, 0.0) == pytest.approx(1.0, rel=1e-8)
    two = I.Sizing(I.SZ_GAUSS_RHO, a0=1.0, a1=4.0, s2=s2, cent=np.array([[0.5, 0.5], [0.5, 0.5]]))
    g2 = orc.build_grid(box_workload(two))
    assert node_value(g2, g2.mu, 0.5, 0.5) == pytest.approx(1 / 3.0, rel=1e-15)


def test_abs_sdf_nodes(orc):
    """mu = a0 + a1 |sdf|: on the unit disk |sdf| = ||x| - 1|."""
    sz = I.Sizing(I.SZ_ABS_SDF, a0=1.0, a1=2.0)
    wl = I.Workload("d", [I.Prim(I.OP_INIT, I.PRIM_DISK, (0.0, 0.0, 1.0))], sz,
                    I.GridSpec(65, 65, -1.25, -1.25, 2.5 / 64, 2.5 / 64, 8), 1000, [], 0)
    g = orc.build_grid(wl)
    xs = -1.25 + np.arange(65) * (2.5 / 64)
    X_, Y_ = np.meshgrid(xs, xs)
    ref = 1.0 + 2.0 * np.abs(np.hypot(X_, Y_) - 1.0)
    assert np.allclose(g.mu.reshape(65, 65), ref, rtol=1e-15, atol=0)
    assert node_value(g, g.mu, 0.0, 0.0) == 3.0


def test_hole_ramp_nodes(orc):
    """mu = 1 + (a0 - 1) min(d_H / a1, 1), d_H the distance to the nearest
    listed hole (here two disks): 1 on a hole's boundary, a0 from a1 away,
    halfway up at a1 / 2; the outer box is not a hole."""
    prims = [I.Prim(I.OP_INIT, I.PRIM_BOX, (-1.0, -1.0, 2.0, 2.0)),
             I.Prim(I.OP_DIFF, I.PRIM_DISK, (0.25, 0.5, 0.125)),
             I.Prim(I.OP_DIFF, I.PRIM_DISK, (0.75, 0.5, 0.0625))]
    sz = I.Sizing(I.SZ_HOLE_RAMP, a0=10.0, a1=0.25, holes=[1, 2])
    wl = I.Workload("h", prims, sz, I.GridSpec(33, 33, 0.0, 0.0, 1 / 32, 1 / 32, 8), 1000, [], 0)
    g = orc.build_grid(wl)
    assert node_value(g, g.mu, 0.375, 0.5) == pytest.approx(1.0, abs=1e-15)     # on hole 1
    assert node_value(g, g.mu, 0.8125, 0.5) == pytest.approx(1.0, abs=1e-15)    # on hole 2
    assert node_value(g, g.mu, 0.25, 0.5) == pytest.approx(1 + 9 * 0.5, rel=1e-15)  # hole 1's centre: d_H = r
    assert node_value(g, g.mu, 0.5, 0.5) == pytest.approx(1 + 9 * (0.125 / 0.25), rel=1e-15)  # 0.125 from hole 1
    assert node_value(g, g.mu, 0.625, 0.5) == pytest.approx(1 + 9 * (0.0625 / 0.25), rel=1e-15)  # nearer hole 2
    assert node_value(g, g.mu, 0.0, 0.0) == pytest.approx(10.0, rel=1e-15)      # > a1 from both


# ---------------------------------------------------------------- h field --

def selected(g):
    s = g.sdf.reshape(g.ny, g.nx)
    sm = (((s[:-1, :-1] + s[:-1, 1:]) + (s[1:, :-1] + s[1:, 1:])) * 0.25).reshape(-1)
    return (g.cat == 1) | ((g.cat == 2) & (sm <= 0.5 * min(g.dx, g.dy)))


@pytest.mark.parametrize("make", [lambda: I.holes20(n=20000, grid_n=256, iters=1),
                                  lambda: I.annulus(n=5000, grid_n=256)])
def test_h_field_counts_n_points(orc, make):
    """Sec. 3.7: a cell of area dx dy is meant to hold dx dy / h^2 points, and
    the h field is scaled so that the selected cells hold N in total.  h_avg
    is the mean h of the selected cells."""
    wl = make()
    g = orc.build_grid(wl)
    sel = selected(g)
    h = g.hcell.astype(np.float64)
    assert np.sum(g.dx * g.dy / h[sel] ** 2) == pytest.approx(wl.n, rel=1e-6)
    assert g.h_avg == pytest.approx(h[sel].mean(), rel=1e-12)
    # h follows the cell's mean mu: the ratio h / mu_cell is one constant
    m = g.mu.reshape(g.ny, g.nx)
    mc = (((m[:-1, :-1] + m[:-1, 1:]) + (m[1:, :-1] + m[1:, 1:])) * 0.25).reshape(-1)
    r = h / mc
    assert np.allclose(r, g.H, rtol=1e-7, atol=0)


def test_h_field_invariant_under_mu_scale(orc):
    """Scaling mu by c scales H by 1/c and leaves every h_cell as it was
    (h depends on the relative sizing only); more points shrink h by
    sqrt(N1 / N2)."""
    base = I.annulus(n=5000, grid_n=128)
    g1 = orc.build_grid(base)
    sc = I.annulus(n=5000, grid_n=128)
    sc.sizing = I.Sizing(sc.sizing.kind, a0=sc.sizing.a0 * 4.0, a1=sc.sizing.a1 * 4.0)
    g2 = orc.build_grid(sc)
    assert g2.H == pytest.approx(g1.H / 4.0, rel=1e-14)
    assert np.allclose(g2.hcell, g1.hcell, rtol=2 ** -23, atol=0)
    more = I.annulus(n=20000, grid_n=128)
    g3 = orc.build_grid(more)
    assert g3.H == pytest.approx(g1.H / 2.0, rel=1e-14)


# ------------------------------------------------------------ fac_mu, Eq. 3 --

def test_fac_mu_takes_mu_at_edge_midpoints(orc):
    """A chain p0 - p1 - p2 inside the half plane x <= 0.3 with
    mu = 1 + 10 |sdf| = 1 + 10 (0.3 - x) (linear there, so bilinear is
    exact).  Eq. 3 with mu at the midpoints: mu(m01) = 5, mu(m12) = 3.5,
    fac = sqrt((l01^2 + l12^2) / (5^2 + 3.5^2)); each end is pushed
    dt k max(1.2 fac mu(m) - l, 0) along its edge (Eq. 2, 5)."""
    sz = I.Sizing(I.SZ_ABS_SDF, a0=1.0, a1=10.0)
    wl = I.Workload("hp", [I.Prim(I.OP_INIT, I.PRIM_BOX, (-5.0, -5.0, 0.3, 5.0))], sz,
                    I.centred_grid(128, 1, 6, 0.0, 8), 100, [], 0)
    g = orc.build_grid(wl)
    x = np.array([-0.2, 0.0, 0.1])
    y = np.array([0.0, 0.01, -0.02])
    rowptr = np.array([0, 1, 3, 4], np.int64)
    col = np.array([1, 0, 2, 1], np.int32)
    mesh = orc.Mesh(np.zeros((0, 3), np.int32), np.zeros(0, np.uint8), rowptr, col, {})
    cat = np.ones(3, np.uint8)
    xn, yn, cn, moved, fm, _ = orc.dm_step(g, x, y, cat, mesh)
    l01 = math.hypot(0.2, 0.01)
    l12 = math.hypot(0.1, 0.03)
    fac = math.sqrt((l01 ** 2 + l12 ** 2) / (5.0 ** 2 + 3.5 ** 2))
    assert fm == pytest.approx(fac, rel=1e-13)
    f01 = max(1.2 * fac * 5.0 - l01, 0.0)
    f12 = max(1.2 * fac * 3.5 - l12, 0.0)
    assert f01 > 0 and f12 > 0
    assert xn[0] - x[0] == pytest.approx(0.2 * f01 * (x[0] - x[1]) / l01, rel=1e-11)
    assert yn[0] - y[0] == pytest.approx(0.2 * f01 * (y[0] - y[1]) / l01, rel=1e-11)
    assert xn[2] - x[2] == pytest.approx(0.2 * f12 * (x[2] - x[1]) / l12, rel=1e-11)
    assert yn[2] - y[2] == pytest.approx(0.2 * f12 * (y[2] - y[1]) / l12, rel=1e-11)
    f1x = f01 * (x[1] - x[0]) / l01 + f12 * (x[1] - x[2]) / l12
    assert xn[1] - x[1] == pytest.approx(0.2 * f1x, rel=1e-11)
    assert list(cn) == [1, 1, 1]


# -------------------------------------------------- AND rule, binding octagons --

def octagon_contains(c, v, h):
    """c strictly inside the octagon of apothem S = fl32(5 h) (D =
    fl32(fl32(sqrt2) S)) centred on v, in exact arithmetic."""
    S = np.float32(5.0) * np.float32(h)
    D = np.float32(1.41421356) * S
    ux, uy = c[0] - Fr(v[0]), c[1] - Fr(v[1])
    return abs(ux) < Fr(float(S)) and abs(uy) < Fr(float(S)) and abs(ux) + abs(uy) < Fr(float(D))


@pytest.mark.parametrize("seed", [31, 32])
def test_and_rule_with_binding_octagons(orc, seed):
    """Per-cell h small enough that octagons bind: the triangles are exactly
    the Delaunay triangles (brute force, rational incircle with symbolic
    perturbation) whose circumcentre lies strictly inside the octagons of
    all three vertices (each with the h of its own cell) and the box."""
    wl = I.random_box(22, seed=seed)
    g = orc.build_grid(wl)
    rng = np.random.default_rng(seed)
    g.hcell = rng.uniform(0.008, 0.04, g.hcell.shape).astype(np.float32)
    m = orc.triangulate(g, wl.x, wl.y)
    pts = list(zip(wl.x, wl.y))
    box = (g.x0, g.y0, g.x0 + (g.nx - 1) * g.dx, g.y0 + (g.ny - 1) * g.dy)

    def h_of(i):
        ci = math.floor((pts[i][0] - g.x0) * (1.0 / g.dx))
        cj = math.floor((pts[i][1] - g.y0) * (1.0 / g.dy))
        return g.hcell[cj * (g.nx - 1) + ci]

    dt = X.delaunay_brute(pts)
    keep, owner_only = set(), 0
    for t in dt:
        c = X.circumcentre(pts, t)
        inside = [octagon_contains(c, pts[i], h_of(i)) for i in t]
        if all(inside) and X.circumcentre_inside(pts, t, box):
            keep.add(t)
        elif inside[0]:
            owner_only += 1  # inside the owner's octagon, outside another's
    assert len(keep) < len(dt)  # the octagons bind
    assert owner_only > 0       # and the other vertices' octagons matter
    assert set(tuple(sorted(map(int, t))) for t in m.tri) == keep
