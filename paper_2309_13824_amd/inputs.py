"""Seeded synthetic workloads for the mesher hot path.

This module only describes inputs: the geometry (a CSG list of analytic
primitives), the sizing/density field, the node grid that carries them and
the initial point positions.  It holds none of the meshing arithmetic; both
the GPU library and the CPU oracle receive the same description and the same
initial point array.

Workloads (the paper meshes its own shapes at N = 1e4..1e7, Sec. 7; these
stand in for them with holes and strong density variation):

* ``disk``      unit disk, uniform sizing, 2,000 points, 256^2 grid (FP64),
                50 DistMesh iterations.
* ``annulus``   annulus 0.3 <= |x| <= 1 minus 3 disks, mu = 1 + 2|sdf|,
                1e5 points, 1024^2 grid, 30 CVD then 70 DistMesh iterations.
* ``holes20``   unit square minus 20 disks, rho = 1 + 4 sum_k exp(-|x-c_k|^2/0.01)
                over 5 centres, 1e6 points, 4096^2 grid, 100 CVD iterations.
* ``ellipses``  unit square minus 200 ellipses, mu = 1 + 9 min(d_H/0.1, 1),
                1e7 points, 8192^2 grid, 70 DistMesh then 30 CVD iterations.
* ``stars``     512 star polygons on 512^2 grids each, log-uniform point counts.

Grids are vertex-centred; spacings and origins are dyadic rationals so that
node coordinates are exact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# CSG operations and primitive kinds (shared numbering of the input format)
OP_INIT, OP_UNION, OP_DIFF, OP_INTERSECT = 0, 1, 2, 3
PRIM_DISK, PRIM_BOX, PRIM_ELLIPSE, PRIM_POLYGON, PRIM_SEGMENTS = 0, 1, 2, 3, 4
SZ_UNIFORM, SZ_ABS_SDF, SZ_GAUSS_RHO, SZ_HOLE_RAMP, SZ_AUTO = 0, 1, 2, 3, 4


@dataclass
class Prim:
    op: int
    kind: int
    p: tuple = ()
    poly: np.ndarray | None = None  # (nv, 2) for polygons


@dataclass
class Sizing:
    kind: int = SZ_UNIFORM
    a0: float = 0.0
    a1: float = 0.0
    s2: float = 1.0
    cent: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    holes: list = field(default_factory=list)
    # automatic sizing (Eq. 8): K = a0, d_s = a1 min(dx, dy), and the medial
    # point trimming's n_thres and fac_nei
    n_thres: int = 3
    fac_nei: float = 2.0
    fac_geps: float = 0.01  # boundary tolerance of the boundary-point trimming


@dataclass
class GridSpec:
    nx: int
    ny: int
    x0: float
    y0: float
    dx: float
    dy: float
    dtype_bytes: int  # 8: float64 nodes, 4: float32 nodes


@dataclass
class Workload:
    name: str
    prims: list
    sizing: Sizing
    grid: GridSpec
    n: int
    schedule: list  # [("dm"|"cvd", iterations), ...]
    seed: int
    x: np.ndarray | None = None
    y: np.ndarray | None = None

    def poly_array(self):
        """Concatenated polygon vertices and (voff, nv) per primitive."""
        verts, offs = [], []
        off = 0
        for p in self.prims:
            if p.kind in (PRIM_POLYGON, PRIM_SEGMENTS):
                offs.append((off, len(p.poly)))
                verts.append(np.asarray(p.poly, dtype=np.float64))
                off += len(p.poly)
            else:
                offs.append((0, 0))
        arr = np.concatenate(verts) if verts else np.zeros((0, 2))
        return np.ascontiguousarray(arr, dtype=np.float64), offs


def centred_grid(n: int, span_num: int, span_log2: int, centre: float, dtype_bytes: int) -> GridSpec:
    """n x n nodes with spacing span_num * 2^-span_log2, centred (dyadic)."""
    d = span_num * 2.0 ** (-span_log2)
    x0 = centre - (n - 1) * d / 2.0
    return GridSpec(n, n, x0, x0, d, d, dtype_bytes)


# ---------------------------------------------------------------- sampling --
# Inside tests and densities below are the workload definitions evaluated for
# drawing initial points only.

def _in_polygon(poly: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Even-odd (crossing number) inside test of a closed polygon."""
    ins = np.zeros(x.shape, dtype=bool)
    nv = len(poly)
    for a in range(nv):
        ax, ay = poly[a]
        bx, by = poly[(a + 1) % nv]
        cross = (ay > y) != (by > y)
        with np.errstate(divide="ignore", invalid="ignore"):
            xi = ax + (y - ay) * (bx - ax) / (by - ay)
        ins ^= cross & (x < xi)
    return ins


class _Buckets:
    """Points bucketed on a uniform grid so that a primitive is evaluated only
    at the points inside its bounding box (many small holes)."""

    def __init__(self, x, y, nb=256):
        self.x0, self.y0 = float(x.min()), float(y.min())
        self.w = max(float(x.max()) - self.x0, float(y.max()) - self.y0, 1e-12) / nb * (1 + 1e-9)
        self.nb = nb
        ix = np.minimum(((x - self.x0) / self.w).astype(np.int64), nb - 1)
        iy = np.minimum(((y - self.y0) / self.w).astype(np.int64), nb - 1)
        cell = iy * nb + ix
        self.order = np.argsort(cell, kind="stable")
        self.start = np.searchsorted(cell[self.order], np.arange(nb * nb + 1))

    def points_in(self, bx0, by0, bx1, by1):
        nb = self.nb
        i0 = max(int((bx0 - self.x0) / self.w), 0)
        i1 = min(int((bx1 - self.x0) / self.w), nb - 1)
        j0 = max(int((by0 - self.y0) / self.w), 0)
        j1 = min(int((by1 - self.y0) / self.w), nb - 1)
        if i1 < i0 or j1 < j0:
            return np.zeros(0, np.int64)
        parts = [self.order[self.start[j * nb + i0]:self.start[j * nb + i1 + 1]] for j in range(j0, j1 + 1)]
        return np.concatenate(parts)


def _prim_bbox(p, pad=0.0):
    if p.kind == PRIM_DISK:
        r = p.p[2] + pad
        return p.p[0] - r, p.p[1] - r, p.p[0] + r, p.p[1] + r
    if p.kind == PRIM_ELLIPSE:
        r = max(p.p[2], p.p[3]) + pad
        return p.p[0] - r, p.p[1] - r, p.p[0] + r, p.p[1] + r
    if p.kind == PRIM_BOX:
        return p.p[0] - pad, p.p[1] - pad, p.p[2] + pad, p.p[3] + pad
    poly = np.asarray(p.poly)
    return poly[:, 0].min() - pad, poly[:, 1].min() - pad, poly[:, 0].max() + pad, poly[:, 1].max() + pad


def _prim_inside(p, x, y):
    if p.kind == PRIM_DISK:
        return (x - p.p[0]) ** 2 + (y - p.p[1]) ** 2 < p.p[2] ** 2
    if p.kind == PRIM_BOX:
        return (x > p.p[0]) & (x < p.p[2]) & (y > p.p[1]) & (y < p.p[3])
    if p.kind == PRIM_ELLIPSE:
        c, s_ = math.cos(p.p[4]), math.sin(p.p[4])
        u = c * (x - p.p[0]) + s_ * (y - p.p[1])
        v = -s_ * (x - p.p[0]) + c * (y - p.p[1])
        return (u / p.p[2]) ** 2 + (v / p.p[3]) ** 2 < 1.0
    return _in_polygon(np.asarray(p.poly, np.float64), x, y)


def _inside(wl: Workload, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    if len(wl.prims) > 16 and all(p.op == OP_DIFF for p in wl.prims[1:]) and len(x) > 0:
        # a base shape minus many holes: each hole is tested near itself only
        ins = _prim_inside(wl.prims[0], x, y)
        bk = _Buckets(x, y)
        for p in wl.prims[1:]:
            idx = bk.points_in(*_prim_bbox(p))
            if len(idx):
                ins[idx] &= ~_prim_inside(p, x[idx], y[idx])
        return ins
    ins = None
    for p in wl.prims:
        if p.kind == PRIM_DISK:
            t = (x - p.p[0]) ** 2 + (y - p.p[1]) ** 2 < p.p[2] ** 2
        elif p.kind == PRIM_BOX:
            t = (x > p.p[0]) & (x < p.p[2]) & (y > p.p[1]) & (y < p.p[3])
        elif p.kind == PRIM_ELLIPSE:
            c, s = math.cos(p.p[4]), math.sin(p.p[4])
            u = c * (x - p.p[0]) + s * (y - p.p[1])
            v = -s * (x - p.p[0]) + c * (y - p.p[1])
            t = (u / p.p[2]) ** 2 + (v / p.p[3]) ** 2 < 1.0
        else:
            t = _in_polygon(np.asarray(p.poly, np.float64), x, y)
        if p.op == OP_INIT:
            ins = t
        elif p.op == OP_UNION:
            ins = ins | t
        elif p.op == OP_DIFF:
            ins = ins & ~t
        else:
            ins = ins & t
    return ins


def _weight(wl: Workload, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Sampling weight proportional to the target point density."""
    sz = wl.sizing
    if sz.kind in (SZ_UNIFORM, SZ_AUTO):
        # automatic sizing is computed by the method itself: uniform start
        return np.ones_like(x)
    if sz.kind == SZ_GAUSS_RHO:
        acc = np.zeros_like(x)
        for cx, cy in sz.cent:
            acc += np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / sz.s2)
        return sz.a0 + sz.a1 * acc
    if sz.kind == SZ_ABS_SDF:
        # distance to the nearest boundary of the disks making the shape
        d = np.full_like(x, np.inf)
        for p in wl.prims:
            if p.kind == PRIM_DISK:
                d = np.minimum(d, np.abs(np.hypot(x - p.p[0], y - p.p[1]) - p.p[2]))
        mu = sz.a0 + sz.a1 * d
        return 1.0 / mu ** 2
    if sz.kind == SZ_HOLE_RAMP:
        # holes farther than a1 leave mu at a0: each hole is visited near itself
        d = np.full_like(x, np.inf)
        bk = _Buckets(x, y) if len(x) else None
        for k in sz.holes:
            p = wl.prims[k]
            r = max(p.p[2], p.p[3]) if p.kind == PRIM_ELLIPSE else p.p[2]
            idx = bk.points_in(*_prim_bbox(p, sz.a1)) if bk is not None else np.zeros(0, np.int64)
            if len(idx):
                d[idx] = np.minimum(d[idx], np.maximum(np.hypot(x[idx] - p.p[0], y[idx] - p.p[1]) - r, 0.0))
        mu = 1.0 + (sz.a0 - 1.0) * np.minimum(d / sz.a1, 1.0)
        return 1.0 / mu ** 2
    raise ValueError(sz.kind)


def sample_points(wl: Workload, rng: np.random.Generator, bbox) -> tuple[np.ndarray, np.ndarray]:
    """Rejection sampling proportional to the density, strictly inside."""
    x0, y0, x1, y1 = bbox
    xs, ys = [], []
    need = wl.n
    wmax = None
    while need > 0:
        m = max(4 * need, 1024)
        x = rng.uniform(x0, x1, m)
        y = rng.uniform(y0, y1, m)
        keep = _inside(wl, x, y)
        x, y = x[keep], y[keep]
        w = _weight(wl, x, y)
        if wmax is None:
            wmax = float(w.max()) * 1.05 if len(w) else 1.0
        u = rng.uniform(0.0, wmax, len(x))
        keep = u < w
        x, y = x[keep][:need], y[keep][:need]
        xs.append(x)
        ys.append(y)
        need -= len(x)
    return np.concatenate(xs), np.concatenate(ys)


def _place_disjoint(rng, count, rmin, rmax, lo, hi, gap, ok=lambda cx, cy, r: True, max_tries=200000):
    out = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place holes")
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(lo + r + gap, hi - r - gap)
        cy = rng.uniform(lo + r + gap, hi - r - gap)
        if not ok(cx, cy, r):
            continue
        if all((cx - a) ** 2 + (cy - b) ** 2 > (r + c + gap) ** 2 for a, b, c in out):
            out.append((cx, cy, r))
    return out


# --------------------------------------------------------------- workloads --

def disk(n: int = 2000, seed: int = 1001, iters: int = 50) -> Workload:
    wl = Workload("disk", [Prim(OP_INIT, PRIM_DISK, (0.0, 0.0, 1.0))], Sizing(SZ_UNIFORM),
                  centred_grid(256, 5, 9, 0.0, 8), n, [("dm", iters)], seed)
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2])
    r = np.sqrt(rng.uniform(0, 1, n))
    t = 2 * np.pi * rng.uniform(0, 1, n)
    wl.x, wl.y = r * np.cos(t), r * np.sin(t)
    return wl


def annulus(n: int = 100000, seed: int = 1002, grid_n: int = 1024) -> Workload:
    ss = np.random.SeedSequence(seed).spawn(3)
    g_rng = np.random.default_rng(ss[0])
    gap = 0.02
    holes = []
    while len(holes) < 3:
        r = g_rng.uniform(0.05, 0.12)
        rc = g_rng.uniform(0.3 + r + gap, 1.0 - r - gap)
        th = g_rng.uniform(0, 2 * np.pi)
        cx, cy = rc * np.cos(th), rc * np.sin(th)
        if all((cx - a) ** 2 + (cy - b) ** 2 > (r + c + gap) ** 2 for a, b, c in holes):
            holes.append((cx, cy, r))
    prims = [Prim(OP_INIT, PRIM_DISK, (0.0, 0.0, 1.0)), Prim(OP_DIFF, PRIM_DISK, (0.0, 0.0, 0.3))]
    prims += [Prim(OP_DIFF, PRIM_DISK, h) for h in holes]
    span_log2 = 11 if grid_n == 1024 else int(round(math.log2(grid_n))) + 1
    wl = Workload("annulus", prims, Sizing(SZ_ABS_SDF, 1.0, 2.0),
                  centred_grid(grid_n, 5, span_log2, 0.0, 4), n, [("cvd", 30), ("dm", 70)], seed)
    wl.x, wl.y = sample_points(wl, np.random.default_rng(ss[2]), (-1, -1, 1, 1))
    return wl


def coast_loop(m: int = 4096, seed: int = 1006) -> np.ndarray:
    """A closed clockwise loop of m segments around (0.5, 0.5): radius
    r(theta) = 0.3 (1 + sum_k a_k cos(k theta + phi_k)), k = 2..48, with
    a_k = 0.22 k^-1.2 u_k, u_k ~ U[-1, 1] and phi_k ~ U[0, 2 pi), clipped to
    [0.12, 0.46]: a coastline-like shape with narrow bays and sharp turns,
    standing in for the paper's line-segment inputs (Sec. 3.2).  Vertices at
    decreasing angles 2 pi (m - j) / m (clockwise)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[0])
    k = np.arange(2, 49)
    amp = 0.22 * k ** -1.2 * rng.uniform(-1, 1, len(k))
    ph = rng.uniform(0, 2 * np.pi, len(k))
    th = 2 * np.pi * (m - np.arange(m)) / m
    r = 0.3 * (1.0 + (amp[None, :] * np.cos(k[None, :] * th[:, None] + ph[None, :])).sum(1))
    r = np.clip(r, 0.12, 0.46)
    return np.ascontiguousarray(np.stack([0.5 + r * np.cos(th), 0.5 + r * np.sin(th)], 1), np.float64)


def coast(n: int = 100000, segments: int = 4096, seed: int = 1006, grid_n: int = 1024, iters: int = 50) -> Workload:
    """Line-segment input (Sec. 3.2): the coast_loop shape minus a disk of
    radius 0.05 at (0.5, 0.5), uniform sizing, on a grid over [0, 1]^2 (with
    a margin); CVD iterations."""
    ss = np.random.SeedSequence(seed).spawn(3)
    loop = coast_loop(segments, seed)
    prims = [Prim(OP_INIT, PRIM_SEGMENTS, (), loop), Prim(OP_DIFF, PRIM_DISK, (0.5, 0.5, 0.05))]
    log2n = int(round(math.log2(grid_n)))
    grid = centred_grid(grid_n, 17, log2n + 4, 0.5, 8)
    wl = Workload("coast", prims, Sizing(SZ_UNIFORM), grid, n, [("cvd", iters)], seed)
    wl.x, wl.y = sample_points(wl, np.random.default_rng(ss[2]), (0, 0, 1, 1))
    return wl


def holes20(n: int = 1000000, seed: int = 1003, grid_n: int = 4096, iters: int = 100) -> Workload:
    ss = np.random.SeedSequence(seed).spawn(3)
    holes = _place_disjoint(np.random.default_rng(ss[0]), 20, 0.02, 0.08, 0.0, 1.0, 0.02)
    cent = np.random.default_rng(ss[1]).uniform(0, 1, (5, 2))
    prims = [Prim(OP_INIT, PRIM_BOX, (0.0, 0.0, 1.0, 1.0))]
    prims += [Prim(OP_DIFF, PRIM_DISK, h) for h in holes]
    log2n = int(round(math.log2(grid_n)))
    # spacing 17 * 2^-(log2n + 4): the span covers [0, 1] with a ~3% margin
    grid = centred_grid(grid_n, 17, log2n + 4, 0.5, 4)
    wl = Workload("holes20", prims, Sizing(SZ_GAUSS_RHO, 1.0, 4.0, 0.01, cent), grid, n,
                  [("cvd", iters)], seed)
    wl.x, wl.y = sample_points(wl, np.random.default_rng(ss[2]), (0, 0, 1, 1))
    return wl


def ellipses(n: int = 10000000, seed: int = 1004, grid_n: int = 8192, n_holes: int = 200) -> Workload:
    ss = np.random.SeedSequence(seed).spawn(3)
    rng = np.random.default_rng(ss[0])
    out = []
    tries = 0
    while len(out) < n_holes:
        tries += 1
        if tries > 1000000:
            raise RuntimeError("could not place ellipses")
        a, b = rng.uniform(0.005, 0.03, 2)
        phi = rng.uniform(0, np.pi)
        r = max(a, b)
        cx, cy = rng.uniform(r + 0.005, 1 - r - 0.005, 2)
        if all((cx - e[0]) ** 2 + (cy - e[1]) ** 2 > (r + max(e[2], e[3]) + 0.005) ** 2 for e in out):
            out.append((cx, cy, a, b, phi, 0.0))
    prims = [Prim(OP_INIT, PRIM_BOX, (0.0, 0.0, 1.0, 1.0))]
    prims += [Prim(OP_DIFF, PRIM_ELLIPSE, e) for e in out]
    log2n = int(round(math.log2(grid_n)))
    grid = centred_grid(grid_n, 17, log2n + 4, 0.5, 4)
    wl = Workload("ellipses", prims, Sizing(SZ_HOLE_RAMP, 10.0, 0.1, holes=list(range(1, n_holes + 1))),
                  grid, n, [("dm", 70), ("cvd", 30)], seed)
    wl.x, wl.y = sample_points(wl, np.random.default_rng(ss[2]), (0, 0, 1, 1))
    return wl


def stars(count: int = 512, seed: int = 1005, grid_n: int = 512, iters: int = 60,
          n_range=(3.0, 5.0)) -> list:
    """A batch of star-shaped polygons, each on its own grid: n_v ~ U{8..64}
    vertices at angles 2 pi (j + u_j) / n_v, u_j ~ U[-0.3, 0.3], radii
    U[0.5, 1]; point counts round(10^U[3, 5]) (log-uniform); uniform sizing;
    DistMesh iterations."""
    ss = np.random.SeedSequence(seed).spawn(3)
    g_rng = np.random.default_rng(ss[0])
    n_rng = np.random.default_rng(ss[1])
    p_seeds = ss[2].spawn(count)
    out = []
    for s_ in range(count):
        nv = int(g_rng.integers(8, 65))
        u = g_rng.uniform(-0.3, 0.3, nv)
        th = 2.0 * np.pi * (np.arange(nv) + u) / nv
        r = g_rng.uniform(0.5, 1.0, nv)
        poly = np.stack([r * np.cos(th), r * np.sin(th)], 1)
        n = int(round(10.0 ** n_rng.uniform(*n_range)))
        wl = Workload("star%d" % s_, [Prim(OP_INIT, PRIM_POLYGON, (), poly)], Sizing(SZ_UNIFORM),
                      centred_grid(grid_n, 5, int(round(math.log2(grid_n))) + 1, 0.0, 4), n, [("dm", iters)],
                      seed)
        rng = np.random.default_rng(p_seeds[s_])
        wl.x, wl.y = sample_points(wl, rng, (-1.0, -1.0, 1.0, 1.0))
        out.append(wl)
    return out


def square_lattice(k: int = 6, spacing: float = 0.125) -> Workload:
    """k x k square lattice (exactly cocircular quadruples) in a uniform box."""
    prims = [Prim(OP_INIT, PRIM_BOX, (-0.5, -0.5, 0.5 + k * spacing, 0.5 + k * spacing))]
    wl = Workload("square_lattice", prims, Sizing(SZ_UNIFORM), centred_grid(64, 1, 4, k * spacing / 2, 8),
                  k * k, [("dm", 1)], 0)
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    wl.x = (ii.ravel() * spacing).astype(np.float64)
    wl.y = (jj.ravel() * spacing).astype(np.float64)
    return wl


def random_box(n: int = 30, seed: int = 7, grid_n: int = 64, lo: float = 0.0, hi: float = 1.0) -> Workload:
    """n uniform points in a box that lies well inside the grid."""
    span = (hi - lo) * 1.5
    d = 2.0 ** math.ceil(math.log2(span / (grid_n - 1)))
    grid = GridSpec(grid_n, grid_n, 0.5 * (lo + hi) - d * (grid_n - 1) / 2, 0.5 * (lo + hi) - d * (grid_n - 1) / 2,
                    d, d, 8)
    wl = Workload("random_box", [Prim(OP_INIT, PRIM_BOX, (lo, lo, hi, hi))], Sizing(SZ_UNIFORM), grid, n,
                  [("dm", 1)], seed)
    rng = np.random.default_rng(seed)
    wl.x = rng.uniform(lo, hi, n)
    wl.y = rng.uniform(lo, hi, n)
    return wl


def degenerate(kind: str) -> Workload:
    """Small point sets in the unit box that the exact predicates must
    settle: "collinear" (six points on one horizontal line, no triangle),
    "coincident" (four copies of one point: one takes the whole box, the
    others have empty cells), "near" (three points 1e-13 apart plus two far
    ones: triangles with beta near 1e12), "disk_ties" (disk points on the
    boundary circle, on grid nodes and on an exact lattice block)."""
    if kind == "collinear":
        wl = random_box(6, seed=3)
        wl.x[:] = [0.1, 0.3, 0.5, 0.7, 0.9, 0.2]
        wl.y[:] = 0.5
    elif kind == "coincident":
        wl = random_box(4, seed=3)
        wl.x[:] = 0.37
        wl.y[:] = 0.61
    elif kind == "near":
        wl = random_box(5, seed=3)
        wl.x[:] = [0.5, 0.5 + 1e-13, 0.5, 0.2, 0.8]
        wl.y[:] = [0.5, 0.5, 0.5 + 1e-13, 0.3, 0.7]
    elif kind == "disk_ties":
        # 600 disk points, four of them exactly on the circle, two on grid
        # nodes, and an exact 4 x 4 lattice block (cocircular quadruples)
        wl = disk(n=600)
        g = wl.grid
        wl.x[:4] = [1.0, 0.0, -1.0, 0.0]
        wl.y[:4] = [0.0, 1.0, 0.0, -1.0]
        wl.x[4], wl.y[4] = g.x0 + 100 * g.dx, g.y0 + 120 * g.dy
        wl.x[5], wl.y[5] = g.x0 + 101 * g.dx, g.y0 + 120 * g.dy
        wl.x[6:22] = 0.3 + 0.01 * np.repeat(np.arange(4), 4)
        wl.y[6:22] = 0.2 + 0.01 * np.tile(np.arange(4), 4)
    else:
        raise ValueError("unknown degenerate case %r" % kind)
    wl.name = "degenerate_" + kind
    return wl


WORKLOADS = {"disk": disk, "annulus": annulus, "holes20": holes20, "ellipses": ellipses}
