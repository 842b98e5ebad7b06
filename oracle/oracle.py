"""ctypes binding of the CPU oracle (test infrastructure only).

The oracle defines what the GPU hot path must compute: FP64 arithmetic,
exact combinatorial predicates with symbolic tie-breaking, the paper's steps
in the paper's order.  Only the test-suite, the smoke check and the CPU
baseline of the benchmark may import this module; the product library never
does.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
SOURCES = ["orc_exact.c", "orc_grid.c", "orc_mesh.c", "orc_sizing.c", "orc_step.c"]

CAT_OUTER, CAT_INNER, CAT_BOUNDARY = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile liborc.so with gcc (-O2, no FP contraction, OpenMP)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    hdrs = [os.path.join(HERE, h) for h in ("orc.h", "orc_internal.h")]
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(s) <= t for s in srcs + hdrs):
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class Prim(C.Structure):
    _fields_ = [("op", C.c_int32), ("kind", C.c_int32), ("p", C.c_double * 6),
                ("voff", C.c_int32), ("nv", C.c_int32)]


class Sizing(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a0", C.c_double), ("a1", C.c_double), ("s2", C.c_double),
                ("ncent", C.c_int32), ("cent", C.POINTER(C.c_double)), ("nholes", C.c_int32),
                ("holes", C.POINTER(C.c_int32)), ("lfs", C.POINTER(C.c_double))]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("y0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("inv_dx", C.c_double),
                ("inv_dy", C.c_double), ("sdf", C.POINTER(C.c_double)),
                ("mu", C.POINTER(C.c_double)), ("cat", C.POINTER(C.c_uint8)),
                ("hcell", C.POINTER(C.c_float)), ("h_avg", C.c_double)]


class Params(C.Structure):
    _fields_ = [("fac_F", C.c_double), ("fac_voro", C.c_double), ("fac_pt", C.c_double),
                ("fac_retria", C.c_double), ("fac_end", C.c_double), ("fac_geps", C.c_double),
                ("T_tria", C.c_double), ("alpha_hat", C.c_double), ("T_newton", C.c_int32),
                ("k_spring", C.c_double), ("dt", C.c_double), ("cvd_max_level", C.c_int32),
                ("trace_max_steps", C.c_int32), ("trace_bisect", C.c_int32),
                ("test2_mode", C.c_int32)]


COUNTER_NAMES = ["candidates", "clip_tests", "cuts", "exact_calls", "sos_calls", "quad_points",
                 "level_cap_hits", "newton_fail", "trace_fail", "empty_cells"]


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in COUNTER_NAMES]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n in COUNTER_NAMES}


class Stats(C.Structure):
    _fields_ = [("ntri", C.c_int64), ("min_q", C.c_double), ("mean_q", C.c_double),
                ("half_mean_alpha", C.c_double), ("half_mean_beta", C.c_double),
                ("max_alpha", C.c_double), ("hist_beta", C.c_double * 40)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp, fp, u8p, i32p, i64p = (C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_uint8),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int64))
        L.orc_default_params.argtypes = [C.POINTER(Params)]
        L.orc_grid_build.argtypes = [C.POINTER(Prim), C.c_int32, dp, C.POINTER(Sizing), C.c_int32,
                                     C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_int32, C.c_int64, dp, dp, u8p, fp, dp, dp]
        L.orc_sdf_eval.argtypes = [C.POINTER(Prim), C.c_int32, dp, C.c_double, C.c_double]
        L.orc_sdf_eval.restype = C.c_double
        L.orc_segments_sdf.argtypes = [dp, C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_int32)]
        L.orc_segments_sdf.restype = C.c_double
        L.orc_boundary_points.argtypes = [C.POINTER(Prim), C.c_int32, dp, C.c_double, C.c_double, dp, C.c_int64]
        L.orc_boundary_points.restype = C.c_int64
        L.orc_trim_boundary.argtypes = [C.POINTER(Prim), C.c_int32, dp, C.c_double, C.c_double, dp, C.c_int64]
        L.orc_trim_boundary.restype = C.c_int64
        L.orc_medial_points.argtypes = [dp, C.c_int64, dp, dp, C.c_int64]
        L.orc_medial_points.restype = C.c_int64
        L.orc_trim_medial.argtypes = [dp, C.c_int64, C.c_double, C.c_int32, C.POINTER(C.c_uint8)]
        L.orc_trim_medial.restype = C.c_int64
        L.orc_lfs.argtypes = [dp, C.c_int64, dp, C.c_int64, C.POINTER(C.c_uint8), dp]
        L.orc_auto_mu.argtypes = [dp, dp, C.c_int64, C.c_double, C.c_double, C.c_double]
        L.orc_auto_mu.restype = C.c_double
        L.orc_grid_init.argtypes = [C.POINTER(Grid), C.c_int32, C.c_int32, C.c_double, C.c_double,
                                    C.c_double, C.c_double, dp, dp, u8p, fp, C.c_double]
        L.orc_cells_all.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, i32p, i32p,
                                    C.c_int, C.c_int, C.POINTER(Counters)]
        L.orc_cells_all_pairs.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, i32p,
                                          i32p, C.c_int]
        L.orc_cell.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, C.c_int64, i32p,
                               dp, dp, C.c_int, C.POINTER(Counters)]
        L.orc_triangulate.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, i32p, u8p,
                                      C.c_int64, i64p, i64p, i32p, C.c_int64, i64p, C.c_int,
                                      C.POINTER(Counters)]
        L.orc_triangle_valid.argtypes = [C.POINTER(Grid), C.POINTER(Params), dp, dp, C.c_int32,
                                         C.c_int32, C.c_int32]
        L.orc_fac_mu.argtypes = [C.POINTER(Grid), C.c_int64, dp, dp, i64p, i32p, dp, dp]
        L.orc_fac_mu.restype = C.c_double
        L.orc_dm_step.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, u8p, i64p, i32p,
                                  dp, dp, dp, dp, u8p, dp, C.POINTER(Counters)]
        L.orc_dm_step.restype = C.c_int64
        L.orc_cvd_step.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, u8p, dp, dp, dp,
                                   u8p, dp, i32p, C.c_int, C.POINTER(Counters)]
        L.orc_cvd_centroid.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, C.c_int64,
                                       C.c_double, dp, dp, dp, C.POINTER(Counters)]
        L.orc_treat.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_double, C.c_double, C.c_uint8,
                                C.c_double, C.c_double, dp, dp, u8p, C.POINTER(Counters)]
        L.orc_point_category.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_double, C.c_double]
        L.orc_point_category.restype = C.c_uint8
        L.orc_point_categories.argtypes = [C.POINTER(Grid), C.POINTER(Params), C.c_int64, dp, dp, u8p]
        L.orc_quality.argtypes = [dp, dp, i32p, u8p, C.c_int64, C.POINTER(Stats)]
        L.orc_triangle_quality.argtypes = [C.c_double] * 6 + [dp, dp]
        L.orc_predicate.argtypes = [C.POINTER(Grid), C.POINTER(Params), dp, dp, C.c_int64, C.c_int32,
                                    C.c_int32, C.c_int32, C.POINTER(C.c_int)]
        L.orc_incircle_sign.argtypes = [C.c_double] * 8
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def default_params(**kw) -> Params:
    p = Params()
    lib().orc_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@dataclass
class OracleGrid:
    """Grid arrays (float64 copies of the node values) and the C view."""
    nx: int
    ny: int
    x0: float
    y0: float
    dx: float
    dy: float
    sdf: np.ndarray
    mu: np.ndarray
    cat: np.ndarray
    hcell: np.ndarray
    h_avg: float
    H: float = 0.0

    def c(self) -> Grid:
        g = Grid()
        self._keep = [np.ascontiguousarray(self.sdf, np.float64), np.ascontiguousarray(self.mu, np.float64),
                      np.ascontiguousarray(self.cat, np.uint8), np.ascontiguousarray(self.hcell, np.float32)]
        s, m, ca, h = self._keep
        lib().orc_grid_init(C.byref(g), self.nx, self.ny, self.x0, self.y0, self.dx, self.dy,
                            _p(s, C.c_double), _p(m, C.c_double), _p(ca, C.c_uint8), _p(h, C.c_float),
                            self.h_avg)
        return g


def _geometry(wl):
    poly, offs = wl.poly_array()
    prims = (Prim * max(len(wl.prims), 1))()
    for k, pr in enumerate(wl.prims):
        prims[k].op = pr.op
        prims[k].kind = pr.kind
        for t, v in enumerate(pr.p):
            prims[k].p[t] = float(v)
        prims[k].voff, prims[k].nv = offs[k]
    sz = Sizing()
    s = wl.sizing
    sz.kind, sz.a0, sz.a1, sz.s2 = s.kind, s.a0, s.a1, s.s2
    cent = np.ascontiguousarray(np.asarray(s.cent, np.float64).reshape(-1))
    holes = np.ascontiguousarray(np.asarray(s.holes, np.int32))
    sz.ncent = len(cent) // 2
    sz.cent = _p(cent, C.c_double)
    sz.nholes = len(holes)
    sz.holes = _p(holes, C.c_int32)
    keep = (poly, cent, holes)
    return prims, sz, poly, keep


@dataclass
class AutoSizing:
    """The automatic sizing field's ingredients (Sec. 3.3, Eq. 8)."""
    s: np.ndarray       # (ns, 2) boundary points
    medial: np.ndarray  # (nm, 2) medial-axis approximating points
    keep: np.ndarray    # (nm,) kept by the trimming
    lfs: np.ndarray     # (ns,) local feature size of each boundary point
    d_s: float
    r_nei: float


def auto_sizing(wl, trim=True) -> AutoSizing:
    """Boundary points of the workload's geometry (App. A; every primitive's
    boundary sampled, the points on the whole boundary kept) at
    d_s = fac_s min(dx, dy) (fac_s = sizing.a1), trimmed (trim=True) with
    geps = fac_geps min(dx, dy), medial-axis points from
    their Voronoi cells clipped to the grid's box grown by its size on every
    side, trimming with r_nei = fac_nei n_thres d_s, and lfs (orc.h states
    each step)."""
    g = wl.grid
    sz = wl.sizing
    prims, _, poly, keep_ = _geometry(wl)
    d_s = sz.a1 * min(g.dx, g.dy)
    geps = sz.fac_geps * min(g.dx, g.dy)
    n = lib().orc_boundary_points(prims, len(wl.prims), _p(poly, C.c_double), d_s, geps, None, 0)
    s = np.empty((n, 2), np.float64)
    lib().orc_boundary_points(prims, len(wl.prims), _p(poly, C.c_double), d_s, geps, _p(s, C.c_double), n)
    if trim:
        n = lib().orc_trim_boundary(prims, len(wl.prims), _p(poly, C.c_double), d_s, geps, _p(s, C.c_double), n)
        s = np.ascontiguousarray(s[:n])
    W, H = (g.nx - 1) * g.dx, (g.ny - 1) * g.dy
    box = np.array([g.x0 - W, g.y0 - H, g.x0 + 2 * W, g.y0 + 2 * H], np.float64)
    m = np.empty((2 * n, 2), np.float64)
    nm = lib().orc_medial_points(_p(s, C.c_double), n, _p(box, C.c_double), _p(m, C.c_double), 2 * n)
    m = np.ascontiguousarray(m[:nm])
    r_nei = sz.fac_nei * sz.n_thres * d_s
    keep = np.zeros(nm, np.uint8)
    lib().orc_trim_medial(_p(m, C.c_double), nm, r_nei, sz.n_thres, _p(keep, C.c_uint8))
    lfs = np.empty(n, np.float64)
    lib().orc_lfs(_p(s, C.c_double), n, _p(m, C.c_double), nm, _p(keep, C.c_uint8), _p(lfs, C.c_double))
    return AutoSizing(s, m, keep, lfs, d_s, r_nei)


def build_grid(wl) -> OracleGrid:
    g = wl.grid
    prims, sz, poly, keep = _geometry(wl)
    if wl.sizing.kind == 4:  # automatic: mu from the boundary points and lfs
        au = auto_sizing(wl)
        s_pts = np.ascontiguousarray(au.s.reshape(-1))
        lfs = np.ascontiguousarray(au.lfs)
        keep = keep + (s_pts, lfs)
        sz.ncent = len(au.s)
        sz.cent = _p(s_pts, C.c_double)
        sz.lfs = _p(lfs, C.c_double)
        sz.a0 = wl.sizing.a0
    nn = g.nx * g.ny
    sdf = np.empty(nn, np.float64)
    mu = np.empty(nn, np.float64)
    cat = np.empty((g.nx - 1) * (g.ny - 1), np.uint8)
    hcell = np.empty((g.nx - 1) * (g.ny - 1), np.float32)
    h_avg = C.c_double()
    H = C.c_double()
    rc = lib().orc_grid_build(prims, len(wl.prims), _p(poly, C.c_double), C.byref(sz), g.nx, g.ny, g.x0,
                              g.y0, g.dx, g.dy, g.dtype_bytes, wl.n, _p(sdf, C.c_double),
                              _p(mu, C.c_double), _p(cat, C.c_uint8), _p(hcell, C.c_float),
                              C.byref(h_avg), C.byref(H))
    if rc != 0:
        raise RuntimeError("oracle grid build failed")
    return OracleGrid(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, sdf, mu, cat, hcell, h_avg.value, H.value)


def grid_from_arrays(spec, sdf, mu, cat, hcell, h_avg) -> OracleGrid:
    """Oracle view of grid arrays produced elsewhere (the shared input)."""
    return OracleGrid(spec.nx, spec.ny, spec.x0, spec.y0, spec.dx, spec.dy,
                      np.asarray(sdf, np.float64).reshape(-1), np.asarray(mu, np.float64).reshape(-1),
                      np.asarray(cat, np.uint8).reshape(-1), np.asarray(hcell, np.float32).reshape(-1),
                      float(h_avg))


def sdf_eval(wl, x, y) -> float:
    prims, sz, poly, keep = _geometry(wl)
    return lib().orc_sdf_eval(prims, len(wl.prims), _p(poly, C.c_double), float(x), float(y))


def segments_sdf(verts, x, y):
    """Signed distance of (x, y) to the closed clockwise loop through verts
    ((m, 2) array), and the index of the nearest segment (Sec. 3.2; the rule
    is stated with orc_segments_sdf in orc.h)."""
    v = np.ascontiguousarray(np.asarray(verts, np.float64).reshape(-1))
    k = C.c_int32(-1)
    d = lib().orc_segments_sdf(_p(v, C.c_double), len(v) // 2, float(x), float(y), C.byref(k))
    return d, k.value


def cells(grid: OracleGrid, x, y, cap=64, all_pairs=False, nthreads=1, params=None):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    n = len(x)
    cons = np.zeros((n, cap), np.int32)
    ncons = np.zeros(n, np.int32)
    g = grid.c()
    prm = params or default_params()
    cnt = Counters()
    if all_pairs:
        rc = lib().orc_cells_all_pairs(C.byref(g), C.byref(prm), n, _p(x, C.c_double), _p(y, C.c_double),
                                       _p(cons, C.c_int32), _p(ncons, C.c_int32), cap)
    else:
        rc = lib().orc_cells_all(C.byref(g), C.byref(prm), n, _p(x, C.c_double), _p(y, C.c_double),
                                 _p(cons, C.c_int32), _p(ncons, C.c_int32), cap, nthreads, C.byref(cnt))
    if rc != 0:
        raise RuntimeError("oracle cells failed")
    return [tuple(cons[i, :ncons[i]]) for i in range(n)], cnt.as_dict()


def cell(grid: OracleGrid, x, y, i, params=None):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    cons = np.zeros(256, np.int32)
    vx = np.zeros(256)
    vy = np.zeros(256)
    g = grid.c()
    prm = params or default_params()
    m = lib().orc_cell(C.byref(g), C.byref(prm), len(x), _p(x, C.c_double), _p(y, C.c_double), i,
                       _p(cons, C.c_int32), _p(vx, C.c_double), _p(vy, C.c_double), 256, None)
    if m < 0:
        raise RuntimeError("oracle cell failed")
    return cons[:m].copy(), vx[:m].copy(), vy[:m].copy()


@dataclass
class Mesh:
    tri: np.ndarray     # (T, 3) owned triangles, CCW, owner first
    valid: np.ndarray   # (T,) uint8
    rowptr: np.ndarray  # (n+1,) int64
    col: np.ndarray     # adjacency of valid triangles, rows sorted
    counters: dict

    def valid_tri(self):
        return self.tri[self.valid.astype(bool)]


def triangulate(grid: OracleGrid, x, y, nthreads=1, params=None) -> Mesh:
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    n = len(x)
    g = grid.c()
    prm = params or default_params()
    tcap = 4 * n + 64
    acap = 12 * n + 64
    for _ in range(2):
        tri = np.zeros((tcap, 3), np.int32)
        valid = np.zeros(tcap, np.uint8)
        rowptr = np.zeros(n + 1, np.int64)
        col = np.zeros(acap, np.int32)
        nt = C.c_int64()
        na = C.c_int64()
        cnt = Counters()
        rc = lib().orc_triangulate(C.byref(g), C.byref(prm), n, _p(x, C.c_double), _p(y, C.c_double),
                                   _p(tri, C.c_int32), _p(valid, C.c_uint8), tcap, C.byref(nt),
                                   _p(rowptr, C.c_int64), _p(col, C.c_int32), acap, C.byref(na), nthreads,
                                   C.byref(cnt))
        if rc == 0:
            return Mesh(tri[:nt.value].copy(), valid[:nt.value].copy(), rowptr, col[:na.value].copy(),
                        cnt.as_dict())
        if rc == -1:
            tcap = max(tcap, nt.value)
            acap = max(acap, na.value)
            continue
        raise RuntimeError("oracle triangulate failed (%d)" % rc)
    raise RuntimeError("oracle triangulate: capacity")


def triangle_valid(grid: OracleGrid, x, y, a, b, c, params=None) -> int:
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    g = grid.c()
    prm = params or default_params()
    return lib().orc_triangle_valid(C.byref(g), C.byref(prm), _p(x, C.c_double), _p(y, C.c_double), a, b, c)


def point_categories(grid: OracleGrid, x, y, params=None) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    g = grid.c()
    prm = params or default_params()
    out = np.empty(len(x), np.uint8)
    lib().orc_point_categories(C.byref(g), C.byref(prm), len(x), _p(x, C.c_double), _p(y, C.c_double),
                               _p(out, C.c_uint8))
    return out


def fac_mu(grid: OracleGrid, x, y, mesh: Mesh):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    g = grid.c()
    sl = C.c_double()
    sm = C.c_double()
    f = lib().orc_fac_mu(C.byref(g), len(x), _p(x, C.c_double), _p(y, C.c_double),
                         _p(mesh.rowptr, C.c_int64), _p(mesh.col, C.c_int32), C.byref(sl), C.byref(sm))
    return f, sl.value, sm.value


def dm_step(grid: OracleGrid, x, y, cat, mesh: Mesh, xl=None, yl=None, params=None):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    cat = np.ascontiguousarray(cat, np.uint8)
    n = len(x)
    xn = np.empty(n)
    yn = np.empty(n)
    cn = np.empty(n, np.uint8)
    xl = np.ascontiguousarray(x if xl is None else xl, np.float64)
    yl = np.ascontiguousarray(y if yl is None else yl, np.float64)
    g = grid.c()
    prm = params or default_params()
    fm = C.c_double()
    cnt = Counters()
    moved = lib().orc_dm_step(C.byref(g), C.byref(prm), n, _p(x, C.c_double), _p(y, C.c_double),
                              _p(cat, C.c_uint8), _p(mesh.rowptr, C.c_int64), _p(mesh.col, C.c_int32),
                              _p(xl, C.c_double), _p(yl, C.c_double), _p(xn, C.c_double), _p(yn, C.c_double),
                              _p(cn, C.c_uint8), C.byref(fm), C.byref(cnt))
    return xn, yn, cn, int(moved), fm.value, cnt.as_dict()


def cvd_step(grid: OracleGrid, x, y, cat, dprev, nthreads=1, params=None):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    cat = np.ascontiguousarray(cat, np.uint8)
    dprev = np.ascontiguousarray(dprev, np.float64)
    n = len(x)
    xn = np.empty(n)
    yn = np.empty(n)
    cn = np.empty(n, np.uint8)
    dn = np.empty(n)
    lev = np.empty(n, np.int32)
    g = grid.c()
    prm = params or default_params()
    cnt = Counters()
    lib().orc_cvd_step(C.byref(g), C.byref(prm), n, _p(x, C.c_double), _p(y, C.c_double), _p(cat, C.c_uint8),
                       _p(dprev, C.c_double), _p(xn, C.c_double), _p(yn, C.c_double), _p(cn, C.c_uint8),
                       _p(dn, C.c_double), _p(lev, C.c_int32), nthreads, C.byref(cnt))
    return xn, yn, cn, dn, lev, cnt.as_dict()


def cvd_centroid(grid: OracleGrid, x, y, i, dprev=-1.0, params=None):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    g = grid.c()
    prm = params or default_params()
    cx = C.c_double()
    cy = C.c_double()
    a = C.c_double()
    L = lib().orc_cvd_centroid(C.byref(g), C.byref(prm), len(x), _p(x, C.c_double), _p(y, C.c_double), i,
                               dprev, C.byref(cx), C.byref(cy), C.byref(a), None)
    return cx.value, cy.value, a.value, L


def treat(grid: OracleGrid, xo, yo, cat_old, xn, yn, params=None):
    g = grid.c()
    prm = params or default_params()
    xf = C.c_double()
    yf = C.c_double()
    cf = C.c_uint8()
    lib().orc_treat(C.byref(g), C.byref(prm), xo, yo, cat_old, xn, yn, C.byref(xf), C.byref(yf), C.byref(cf),
                    None)
    return xf.value, yf.value, cf.value


def quality(x, y, tri, valid=None) -> dict:
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    st = Stats()
    vp = _p(np.ascontiguousarray(valid, np.uint8), C.c_uint8) if valid is not None else None
    lib().orc_quality(_p(x, C.c_double), _p(y, C.c_double), _p(tri, C.c_int32), vp, len(tri), C.byref(st))
    return {"ntri": st.ntri, "min_q": st.min_q, "mean_q": st.mean_q, "half_mean_alpha": st.half_mean_alpha,
            "half_mean_beta": st.half_mean_beta, "max_alpha": st.max_alpha,
            "hist_beta": np.array(st.hist_beta[:])}


def triangle_quality(a, b, c):
    al = C.c_double()
    be = C.c_double()
    lib().orc_triangle_quality(a[0], a[1], b[0], b[1], c[0], c[1], C.byref(al), C.byref(be))
    return al.value, be.value


def predicate(grid: OracleGrid, x, y, i, c1, c2, c3, params=None):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    g = grid.c()
    prm = params or default_params()
    ue = C.c_int(0)
    s = lib().orc_predicate(C.byref(g), C.byref(prm), _p(x, C.c_double), _p(y, C.c_double), i, c1, c2, c3,
                            C.byref(ue))
    return s, ue.value


def incircle_sign(a, b, c, d) -> int:
    return lib().orc_incircle_sign(a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1])


def initial_categories(grid: OracleGrid, x, y, params=None) -> np.ndarray:
    """Initial point categories (Sec. 3.5): inner cell -> inner; boundary cell
    -> boundary when |sdf| <= geps, else inner."""
    return point_categories(grid, x, y, params)


def run(grid: OracleGrid, x, y, schedule, params=None, nthreads=1, retriangulate="flag"):
    """Full run of a fixed schedule [("dm"|"cvd", iters), ...] (Alg. 1, Alg. 2).

    DistMesh triangulates on the first iteration of a segment and then only
    when the previous iteration moved a point more than fac_retria*h since the
    last triangulation (retriangulate="flag"), or every iteration ("always").
    Returns final positions, categories, the last mesh and per-iteration info.
    """
    prm = params or default_params()
    x = np.array(x, np.float64)
    y = np.array(y, np.float64)
    cat = initial_categories(grid, x, y, prm)
    dprev = np.full(len(x), -1.0)
    info = []
    mesh = None
    for method, iters in schedule:
        retri = True
        xl, yl = x.copy(), y.copy()
        for _ in range(iters):
            if method == "dm":
                if retri or retriangulate == "always" or mesh is None:
                    mesh = triangulate(grid, x, y, nthreads, prm)
                    xl, yl = x.copy(), y.copy()
                    tri_now = True
                else:
                    tri_now = False
                xn, yn, cn, moved, fm, _ = dm_step(grid, x, y, cat, mesh, xl, yl, prm)
                retri = moved > 0
                dn = np.hypot(xn - x, yn - y)
                info.append({"method": "dm", "triangulated": tri_now, "moved": moved, "fac_mu": fm})
            else:
                mesh = triangulate(grid, x, y, nthreads, prm)
                xn, yn, cn, dn, lev, _ = cvd_step(grid, x, y, cat, dprev, nthreads, prm)
                info.append({"method": "cvd", "triangulated": True, "max_level": int(lev.max()) if len(lev) else 0})
            x, y, cat, dprev = xn, yn, cn, dn
    final = triangulate(grid, x, y, nthreads, prm)
    return x, y, cat, final, info


STOP_QUALITY, STOP_MOVEMENT = 1, 2


def cell_h(grid: OracleGrid, x, y) -> np.ndarray:
    """h of the grid cell holding each point (Sec. 3.7): the cell index is
    floor((x - x0) / dx) with the division taken as a product by 1/dx,
    clamped to the grid."""
    fx = np.floor((np.asarray(x) - grid.x0) * (1.0 / grid.dx)).astype(np.int64)
    fy = np.floor((np.asarray(y) - grid.y0) * (1.0 / grid.dy)).astype(np.int64)
    fx = np.clip(fx, 0, grid.nx - 2)
    fy = np.clip(fy, 0, grid.ny - 2)
    return grid.hcell[fy * (grid.nx - 1) + fx].astype(np.float64)


def run_adaptive(grid: OracleGrid, x, y, mode, max_iter, t_quality=0.001, t_amax=0.005, t_switch=0.0015,
                 params=None, nthreads=1):
    """Adaptive run: termination tests and the DistMesh -> CVD switch.

    mode is "dm", "cvd" or "hybrid" (DistMesh first, then CVD).  Every
    iteration measures the mesh it works on: the triangles of its
    triangulation (DistMesh reuses the last one until a point has moved more
    than fac_retria*h, Alg. 1) at the positions the iteration starts from,
    giving M_1/2(alpha), M_1/2(beta) (Eq. 10-11) and max alpha over the valid
    triangles.  After the iteration's update, with r the relative change of
    each of the three against the previous iteration:

    - hybrid, DistMesh phase: switch to CVD for the next iteration when
      r(M_1/2 alpha) < t_switch (Sec. 4.2, hybrid meshing; Table 8);
    - otherwise stop when r(M_1/2 alpha) < t_quality, r(M_1/2 beta) <
      t_quality and r(max alpha) < t_amax (Sec. 6, the quality criteria),
      else when no inner point (category of the start position) moved by
      fac_end*h or more, h of the cell it started in (Sec. 6 and Sec. 3.7,
      T_end_mvmt).

    The first iteration has no previous statistics, so only the movement test
    can end it.  Returns the final positions and categories and a dict with
    the iterations run, the iteration that switched and the one that stopped
    (-1 when none), the stop reason (STOP_QUALITY / STOP_MOVEMENT, 0) and the
    per-iteration history.
    """
    prm = params or default_params()
    x = np.array(x, np.float64)
    y = np.array(y, np.float64)
    cat = initial_categories(grid, x, y, prm)
    dprev = np.full(len(x), -1.0)
    hybrid = mode == "hybrid"
    method = "cvd" if mode == "cvd" else "dm"
    mesh, retri, xl, yl = None, True, None, None
    prev, switch_iter, stop_iter, reason, hist = None, -1, -1, 0, []
    for it in range(max_iter):
        ran = method
        if method == "dm":
            if retri or mesh is None:
                mesh = triangulate(grid, x, y, nthreads, prm)
                xl, yl = x.copy(), y.copy()
            q = quality(x, y, mesh.tri, mesh.valid)
            xn, yn, cn, moved, _, _ = dm_step(grid, x, y, cat, mesh, xl, yl, prm)
            retri = moved > 0
            dn = np.sqrt((xn - x) * (xn - x) + (yn - y) * (yn - y))
        else:
            mesh = triangulate(grid, x, y, nthreads, prm)
            q = quality(x, y, mesh.tri, mesh.valid)
            xn, yn, cn, dn, _, _ = cvd_step(grid, x, y, cat, dprev, nthreads, prm)
        cur = (q["half_mean_alpha"], q["half_mean_beta"], q["max_alpha"])
        step = np.sqrt((xn - x) * (xn - x) + (yn - y) * (yn - y))
        moving = bool(np.any((cat == CAT_INNER) & (step >= prm.fac_end * cell_h(grid, x, y))))
        rel = None
        if prev is not None and q["ntri"] > 0 and min(prev) > 0:
            rel = tuple(abs(c - p) / p for c, p in zip(cur, prev))
        stop = False
        if hybrid and method == "dm":
            if rel is not None and rel[0] < t_switch:
                method = "cvd"
                switch_iter = it
        elif rel is not None and rel[0] < t_quality and rel[1] < t_quality and rel[2] < t_amax:
            stop, reason = True, STOP_QUALITY
        elif not moving:
            stop, reason = True, STOP_MOVEMENT
        hist.append({"method": ran, "quality": cur, "rel": rel, "moving": moving})
        prev = cur if q["ntri"] > 0 else None
        x, y, cat, dprev = xn, yn, cn, dn
        if stop:
            stop_iter = it
            break
    return x, y, cat, {"iters": len(hist), "switch_iter": switch_iter, "stop_iter": stop_iter,
                       "reason": reason, "history": hist}


def scaled_grid(grid: OracleGrid, h_scale: float) -> OracleGrid:
    """The grid with every h scaled for the current point count (Sec. 3.7:
    when points are added, the geometric quantities are scaled by
    sqrt(N_old / N_current)): h_cell = fl32(h_cell * h_scale), h_avg too."""
    hc = (grid.hcell.astype(np.float64) * h_scale).astype(np.float32)
    return OracleGrid(grid.nx, grid.ny, grid.x0, grid.y0, grid.dx, grid.dy, grid.sdf, grid.mu, grid.cat, hc,
                      grid.h_avg * h_scale, grid.H)


def added_points(grid: OracleGrid, x, y, mesh: Mesh, n_add: int, params=None):
    """Point addition (Sec. 3.6): the n_add valid triangles with the largest
    ratio of circumradius to the local desired edge length h (the h of the
    grid cell holding the triangle's centroid) give one new point each, at
    their centroids.  Ties in the ratio go to the smaller (owner id, second
    id) of the triangle (the owner is its smallest id, first in CCW order).
    The new points are returned in the order of (owner id, second id) of
    their triangles: they get the ids n, n + 1, ...  The circumradius is
    sqrt(|ab|^2 |bc|^2 |ca|^2) / (2 |(b - a) x (c - a)|) and the centroid
    ((x_a + x_b) + x_c) / 3, in FP64."""
    tri = mesh.tri[mesh.valid.astype(bool)].astype(np.int64)
    xa, ya, xb, yb, xc, yc = x[tri[:, 0]], y[tri[:, 0]], x[tri[:, 1]], y[tri[:, 1]], x[tri[:, 2]], y[tri[:, 2]]
    d1x, d1y, d2x, d2y = xb - xa, yb - ya, xc - xa, yc - ya
    cross = d1x * d2y - d1y * d2x
    la2 = d1x * d1x + d1y * d1y
    lb2 = (xc - xb) * (xc - xb) + (yc - yb) * (yc - yb)
    lc2 = d2x * d2x + d2y * d2y
    R = np.sqrt(la2 * lb2 * lc2) / (2.0 * np.abs(cross))
    gx = ((xa + xb) + xc) / 3.0
    gy = ((ya + yb) + yc) / 3.0
    ratio = R / cell_h(grid, gx, gy)
    order = np.lexsort((tri[:, 1], tri[:, 0], -ratio))
    sel = order[:n_add]
    sel = sel[np.lexsort((tri[sel, 1], tri[sel, 0]))]
    return gx[sel], gy[sel]


def run_growing(grid: OracleGrid, x_all, y_all, mode, max_iter, n_init, t_add=0.002, fac_add=0.6,
                t_quality=0.001, t_amax=0.005, t_switch=0.0015, params=None, nthreads=1):
    """Adaptive run with point addition (Sec. 3.6): it starts from the first
    n_init points; while fewer than N_total = len(x_all) points are in the
    mesh, an iteration whose relative changes of M_1/2(alpha) and
    M_1/2(beta) are both below t_add adds min(floor(fac_add N_current),
    N_total - N_current) points (added_points), and the switch and
    termination tests (run_adaptive) wait until all points are in.  The
    geometric quantities follow the current count: h scaled by
    sqrt(N_total / N_current) (the grid is built for N_total).  After an
    addition the next iteration has no previous statistics, DistMesh
    re-triangulates, and the new points start with d_prev = -1 and the
    category of their position.  Returns the final points and categories
    and a dict with the iterations at which points were added (and the
    counts), the switch and stop iterations, the reason and the history."""
    prm = params or default_params()
    n_total = len(x_all)
    n = int(n_init)
    x = np.array(x_all[:n], np.float64)
    y = np.array(y_all[:n], np.float64)
    gcur = scaled_grid(grid, math.sqrt(n_total / n))
    cat = initial_categories(gcur, x, y, prm)
    dprev = np.full(n, -1.0)
    hybrid = mode == "hybrid"
    method = "cvd" if mode == "cvd" else "dm"
    mesh, retri, xl, yl = None, True, None, None
    prev, switch_iter, stop_iter, reason, hist, adds = None, -1, -1, 0, [], []
    for it in range(max_iter):
        ran = method
        if method == "dm":
            if retri or mesh is None:
                mesh = triangulate(gcur, x, y, nthreads, prm)
                xl, yl = x.copy(), y.copy()
            q = quality(x, y, mesh.tri, mesh.valid)
            xn, yn, cn, moved, _, _ = dm_step(gcur, x, y, cat, mesh, xl, yl, prm)
            retri = moved > 0
            dn = np.sqrt((xn - x) * (xn - x) + (yn - y) * (yn - y))
        else:
            mesh = triangulate(gcur, x, y, nthreads, prm)
            q = quality(x, y, mesh.tri, mesh.valid)
            xn, yn, cn, dn, _, _ = cvd_step(gcur, x, y, cat, dprev, nthreads, prm)
        cur = (q["half_mean_alpha"], q["half_mean_beta"], q["max_alpha"])
        step = np.sqrt((xn - x) * (xn - x) + (yn - y) * (yn - y))
        moving = bool(np.any((cat == CAT_INNER) & (step >= prm.fac_end * cell_h(gcur, x, y))))
        rel = None
        if prev is not None and q["ntri"] > 0 and min(prev) > 0:
            rel = tuple(abs(c - p) / p for c, p in zip(cur, prev))
        stop, add = False, 0
        if n < n_total:
            if rel is not None and rel[0] < t_add and rel[1] < t_add:
                add = min(int(math.floor(fac_add * n)), n_total - n)
        elif hybrid and method == "dm":
            if rel is not None and rel[0] < t_switch:
                method = "cvd"
                switch_iter = it
        elif rel is not None and rel[0] < t_quality and rel[1] < t_quality and rel[2] < t_amax:
            stop, reason = True, STOP_QUALITY
        elif not moving:
            stop, reason = True, STOP_MOVEMENT
        hist.append({"method": ran, "n": n, "quality": cur, "rel": rel, "moving": moving})
        prev = cur if q["ntri"] > 0 else None
        x, y, cat, dprev = xn, yn, cn, dn
        if add > 0:
            # the mesh of this iteration at the updated positions picks the triangles
            gx, gy = added_points(gcur, x, y, mesh, add, prm)
            n += add
            gcur = scaled_grid(grid, math.sqrt(n_total / n))
            x = np.concatenate([x, gx])
            y = np.concatenate([y, gy])
            cat = np.concatenate([cat, initial_categories(gcur, gx, gy, prm)])
            dprev = np.concatenate([dprev, np.full(add, -1.0)])
            adds.append((it, add))
            prev, retri = None, True
        if stop:
            stop_iter = it
            break
    return x, y, cat, {"iters": len(hist), "adds": adds, "switch_iter": switch_iter, "stop_iter": stop_iter,
                       "reason": reason, "history": hist}
