"""Python binding of the trime C ABI (include/trime.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libtrime.so.  PyTorch provides device memory and the stream.  The
module refuses to run without the built library and a HIP device.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TRIME_LIB selects another build of the same library (tuning variants)
LIB_PATH = os.environ.get("TRIME_LIB", os.path.join(HERE, "libtrime.so"))

FP64, FP32 = 0, 1
CAT_OUTER, CAT_INNER, CAT_BOUNDARY = 0, 1, 2
METHOD_DM, METHOD_CVD, METHOD_DM_ALWAYS = 0, 1, 2
TRI_PER_POINT = 16
STATUS = {0: "TRIME_OK", 1: "TRIME_EINVAL", 2: "TRIME_EUNSUPPORTED", 3: "TRIME_ECAPACITY",
          4: "TRIME_EHIP", 5: "TRIME_EDEGENERATE"}


class TrimeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


# ---------------------------------------------------------------- structs --
class Prim(C.Structure):
    _fields_ = [("op", C.c_int32), ("kind", C.c_int32), ("p", C.c_double * 6), ("voff", C.c_int32),
                ("nv", C.c_int32)]


class Geometry(C.Structure):
    _fields_ = [("nprims", C.c_int32), ("prims", C.POINTER(Prim)), ("npoly", C.c_int32),
                ("poly", C.POINTER(C.c_double))]


class Sizing(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a0", C.c_double), ("a1", C.c_double), ("s2", C.c_double),
                ("ncent", C.c_int32), ("cent", C.POINTER(C.c_double)), ("nholes", C.c_int32),
                ("holes", C.POINTER(C.c_int32)), ("n_thres", C.c_int32), ("fac_nei", C.c_double),
                ("fac_geps", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("y0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("dtype_bytes", C.c_int32)]


class GridScalars(C.Structure):
    _fields_ = [("H", C.c_double), ("h_avg", C.c_double), ("area_sel", C.c_double), ("n_sel", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("fac_F", C.c_double), ("fac_voro", C.c_double), ("fac_pt", C.c_double),
                ("fac_retria", C.c_double), ("fac_end", C.c_double), ("fac_geps", C.c_double),
                ("T_tria", C.c_double), ("alpha_hat", C.c_double), ("T_newton", C.c_int32),
                ("k_spring", C.c_double), ("dt", C.c_double), ("cvd_max_level", C.c_int32),
                ("trace_max_steps", C.c_int32), ("trace_bisect", C.c_int32), ("test2_mode", C.c_int32)]


class AdaptCtl(C.Structure):
    _fields_ = [("method", C.c_int32), ("stopped", C.c_int32), ("iters", C.c_int32), ("switch_iter", C.c_int32),
                ("stop_iter", C.c_int32), ("reason", C.c_int32), ("moving", C.c_int32), ("have_prev", C.c_int32),
                ("growing", C.c_int32), ("add_request", C.c_int32), ("gate", C.c_int32 * 8), ("prev", C.c_double * 3), ("last", C.c_double * 3),
                ("rel", C.c_double * 3)]


class Stats(C.Structure):
    _fields_ = [("fp64_replays", C.c_int64), ("exact_points", C.c_int64), ("exact_calls", C.c_int64),
                ("sos_calls", C.c_int64), ("overflow_points", C.c_int64), ("newton_fail", C.c_int64),
                ("trace_fail", C.c_int64), ("level_cap_hits", C.c_int64), ("empty_cells", C.c_int64),
                ("ntri", C.c_int64), ("nvalid", C.c_int64), ("moved", C.c_int64),
                ("triangulations", C.c_int64), ("iterations", C.c_int64), ("retri_flag", C.c_int32),
                ("error", C.c_int32), ("sum_l2", C.c_double), ("sum_mu2", C.c_double),
                ("fac_mu", C.c_double), ("sum_sqrt_alpha", C.c_double), ("sum_sqrt_beta", C.c_double),
                ("sum_q", C.c_double), ("max_alpha", C.c_double), ("nq", C.c_int64),
                ("hist_beta", C.c_int64 * 40), ("work_candidates", C.c_int64), ("work_margins", C.c_int64),
                ("work_cuts", C.c_int64), ("work_leaves", C.c_int64), ("adapt", AdaptCtl),
                ("half_mean_alpha", C.c_double), ("half_mean_beta", C.c_double), ("mean_q", C.c_double),
                ("min_q", C.c_double), ("quality_acc", C.c_uint64 * 6)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("hist_beta", "adapt", "quality_acc")}
        a = self.adapt
        d["adapt"] = {"method": a.method, "stopped": a.stopped, "iters": a.iters, "switch_iter": a.switch_iter,
                      "stop_iter": a.stop_iter, "reason": a.reason, "growing": a.growing,
                      "last": tuple(a.last[:]),
                      "rel": tuple(a.rel[:])}
        d["hist_beta"] = np.array(self.hist_beta[:], np.int64)
        return d


class PosBuf(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("dprev", C.c_void_p), ("cat", C.c_void_p)]


class OrdBuf(C.Structure):
    _fields_ = [("id", C.c_void_p), ("span", C.c_void_p), ("xl", C.c_void_p), ("yl", C.c_void_p)]


class State(C.Structure):
    _fields_ = [("n", C.c_int64), ("precision", C.c_int32), ("max_deg", C.c_int32),
                ("bin_density", C.c_double), ("grid", Grid), ("sdf", C.c_void_p), ("mu", C.c_void_p),
                ("cat_grid", C.c_void_p), ("hcell", C.c_void_p), ("scal", C.c_void_p),
                ("params", Params), ("pos", PosBuf * 2), ("ord", OrdBuf * 2), ("cur_pos", C.c_int32),
                ("cur_ord", C.c_int32), ("adj", C.c_void_p), ("deg", C.c_void_p), ("tri", C.c_void_p),
                ("tri_valid", C.c_void_p), ("tri_n", C.c_void_p), ("perm", C.c_void_p),
                ("key", C.c_void_p), ("rank", C.c_void_p), ("order", C.c_void_p), ("bin_start", C.c_void_p),
                ("bin_fill", C.c_void_p), ("scan_tmp", C.c_void_p), ("queue", C.c_void_p),
                ("counters", C.c_void_p), ("partials", C.c_void_p), ("stats", C.c_void_p),
                ("nbx", C.c_int32), ("nby", C.c_int32), ("lbits", C.c_int32), ("bx0", C.c_double),
                ("by0", C.c_double), ("bw", C.c_double), ("area_sel", C.c_double), ("nkeys", C.c_int64),
                ("ev_cells", C.c_void_p * 2), ("n_cap", C.c_int64), ("h_scale", C.c_double),
                ("nkeys_cap", C.c_int64), ("n_grid", C.c_int64), ("warm_n", C.c_void_p * 2),
                ("warm_nb", C.c_void_p * 2), ("old_slot", C.c_void_p), ("new_slot", C.c_void_p),
                ("xcd_run", C.c_int32)]


ADAPT_DM, ADAPT_CVD, ADAPT_HYBRID = 0, 1, 2
STOP_NONE, STOP_QUALITY, STOP_MOVEMENT = 0, 1, 2


class Adaptive(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_iter", C.c_int32), ("t_quality", C.c_double), ("t_amax", C.c_double),
                ("t_switch", C.c_double)]


class Growing(C.Structure):
    _fields_ = [("base", Adaptive), ("n_total", C.c_int64), ("t_add", C.c_double), ("fac_add", C.c_double)]


class Schedule(C.Structure):
    _fields_ = [("nseg", C.c_int32), ("method", C.POINTER(C.c_int32)), ("iters", C.POINTER(C.c_int32))]


class Cells(C.Structure):
    _fields_ = [("cap", C.c_int32), ("cons", C.c_void_p), ("ncons", C.c_void_p)]


EXPORTED = ["trime_last_error", "trime_version", "trime_default_params", "trime_sdf_grid_build",
            "trime_state_workspace_bytes", "trime_state_bind", "trime_state_load", "trime_export_points",
            "trime_export_triangles", "trime_export_adjacency", "trime_bin_points", "trime_voronoi_cells",
            "trime_delaunay_extract", "trime_step_dm", "trime_step_cvd", "trime_step_hybrid",
            "trime_quality", "trime_stats_read", "trime_stats_check", "trime_autotune_workspace_bytes",
            "trime_autotune", "trime_batch_graph_create", "trime_graph_launch", "trime_graph_destroy",
            "trime_step_adaptive", "trime_batch_create", "trime_batch_run", "trime_batch_destroy",
            "trime_batch_make_persistent",
            "trime_add_points", "trime_run_growing", "trime_auto_sizing", "trime_sdf_grid_build_noalloc"]

_lib = None


def lib(require_gpu: bool = True):
    """The loaded libtrime.so.  Raises when it is not built (or, by default,
    when no HIP device is visible): there is no CPU fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtrime.so is not built (run __graft_entry__.build())")
        # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
        # libtrime.so binds to, so the process holds a single HIP runtime.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.POINTER(State)
        L.trime_last_error.restype = C.c_char_p
        L.trime_version.restype = C.c_char_p
        L.trime_default_params.argtypes = [C.POINTER(Params)]
        L.trime_sdf_grid_build.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing), C.POINTER(Grid), C.c_int64,
                                           vp, vp, vp, vp, vp, vp]
        L.trime_sdf_grid_build_noalloc.argtypes = L.trime_sdf_grid_build.argtypes
        L.trime_state_workspace_bytes.argtypes = [st, C.POINTER(C.c_size_t)]
        L.trime_state_bind.argtypes = [st, vp, C.c_size_t, vp]
        L.trime_state_load.argtypes = [st, vp, vp, vp]
        L.trime_export_points.argtypes = [st, vp, vp, vp, vp]
        L.trime_export_triangles.argtypes = [st, vp, vp, C.c_int64, vp, vp]
        L.trime_export_adjacency.argtypes = [st, vp, vp, vp]
        L.trime_bin_points.argtypes = [st, vp]
        L.trime_voronoi_cells.argtypes = [st, C.POINTER(Cells), vp]
        L.trime_delaunay_extract.argtypes = [st, vp]
        L.trime_step_dm.argtypes = [st, C.c_int32, C.c_int32, C.c_int32, vp]
        L.trime_step_cvd.argtypes = [st, C.c_int32, vp]
        L.trime_step_hybrid.argtypes = [st, C.POINTER(Schedule), vp]
        L.trime_quality.argtypes = [st, vp]
        L.trime_stats_read.argtypes = [st, C.POINTER(Stats), vp]
        L.trime_stats_check.argtypes = [C.POINTER(Stats)]
        dp = C.POINTER(C.c_double)
        L.trime_autotune_workspace_bytes.argtypes = [st, dp, C.c_int32, C.POINTER(C.c_size_t)]
        L.trime_autotune.argtypes = [st, vp, C.c_size_t, vp, vp, dp, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                     C.c_int32, dp, C.POINTER(C.c_int32), C.POINTER(C.c_float), vp]
        L.trime_batch_graph_create.argtypes = [C.POINTER(st), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                               C.POINTER(vp), vp]
        L.trime_graph_launch.argtypes = [vp, vp]
        L.trime_graph_destroy.argtypes = [vp]
        L.trime_step_adaptive.argtypes = [st, C.POINTER(Adaptive), vp]
        L.trime_batch_create.argtypes = [C.POINTER(st), C.c_int32, C.c_int32, C.POINTER(vp)]
        L.trime_batch_run.argtypes = [vp, C.c_int32, vp]
        L.trime_batch_destroy.argtypes = [vp]
        L.trime_batch_make_persistent.argtypes = [vp, C.c_int32, C.c_int32]
        L.trime_add_points.argtypes = [st, C.c_int64, vp]
        L.trime_run_growing.argtypes = [st, C.POINTER(Growing), vp]
        i64p = C.POINTER(C.c_int64)
        L.trime_auto_sizing.argtypes = [C.POINTER(Geometry), C.POINTER(Sizing), C.POINTER(Grid), vp, C.c_int64, i64p,
                                        vp, vp, C.c_int64, i64p, vp, vp]
        for f in EXPORTED:
            if f not in ("trime_last_error", "trime_version", "trime_default_params"):
                getattr(L, f).restype = C.c_int
        _lib = L
    if require_gpu:
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("trime needs a HIP device; none is visible")
    return _lib


def _check(code):
    if code != 0:
        raise TrimeError(code, lib(False).trime_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def default_params(**kw) -> Params:
    p = Params()
    lib(False).trime_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ------------------------------------------------------------- entry points --
def sdf_grid_build(geometry, sizing, grid, n_total, sdf, mu, cat, hcell, scal, stream=None):
    _check(lib().trime_sdf_grid_build(C.byref(geometry), C.byref(sizing), C.byref(grid), int(n_total),
                                      _ptr(sdf), _ptr(mu), _ptr(cat), _ptr(hcell), _ptr(scal), _stream(stream)))


def sdf_grid_build_noalloc(geometry, sizing, grid, n_total, sdf, mu, cat, hcell, scal, stream=None):
    """trime_sdf_grid_build without any allocation (a static scratch array
    per GPU; calls overlapping on one GPU race)."""
    _check(lib().trime_sdf_grid_build_noalloc(C.byref(geometry), C.byref(sizing), C.byref(grid), int(n_total),
                                              _ptr(sdf), _ptr(mu), _ptr(cat), _ptr(hcell), _ptr(scal),
                                              _stream(stream)))


def state_workspace_bytes(state) -> int:
    b = C.c_size_t()
    _check(lib().trime_state_workspace_bytes(C.byref(state), C.byref(b)))
    return b.value


def state_bind(state, ws, stream=None):
    _check(lib().trime_state_bind(C.byref(state), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def state_load(state, x, y, stream=None):
    _check(lib().trime_state_load(C.byref(state), _ptr(x), _ptr(y), _stream(stream)))


def bin_points(state, stream=None):
    _check(lib().trime_bin_points(C.byref(state), _stream(stream)))


def voronoi_cells(state, cells, stream=None):
    _check(lib().trime_voronoi_cells(C.byref(state), C.byref(cells), _stream(stream)))


def delaunay_extract(state, stream=None):
    _check(lib().trime_delaunay_extract(C.byref(state), _stream(stream)))


def step_dm(state, n_iter, fresh=True, always=False, stream=None):
    _check(lib().trime_step_dm(C.byref(state), int(n_iter), int(bool(fresh)), int(bool(always)), _stream(stream)))


def step_cvd(state, n_iter, stream=None):
    _check(lib().trime_step_cvd(C.byref(state), int(n_iter), _stream(stream)))


def step_hybrid(state, schedule, stream=None):
    meth = (C.c_int32 * len(schedule))(*[METHOD_DM if m == "dm" else METHOD_CVD for m, _ in schedule])
    its = (C.c_int32 * len(schedule))(*[int(k) for _, k in schedule])
    sch = Schedule(len(schedule), meth, its)
    _check(lib().trime_step_hybrid(C.byref(state), C.byref(sch), _stream(stream)))


def step_adaptive(state, mode, max_iter, t_quality=0.001, t_amax=0.005, t_switch=0.0015, stream=None):
    """mode: "dm", "cvd" or "hybrid"; the outcome is in the stats (adapt)."""
    m = {"dm": ADAPT_DM, "cvd": ADAPT_CVD, "hybrid": ADAPT_HYBRID}[mode]
    cfg = Adaptive(m, int(max_iter), float(t_quality), float(t_amax), float(t_switch))
    _check(lib().trime_step_adaptive(C.byref(state), C.byref(cfg), _stream(stream)))


def add_points(state, n_add, stream=None):
    """Appends the centroids of the n_add valid triangles with the largest
    circumradius / h (synchronises); the state's h scale becomes
    sqrt(n_grid / n) for the new n (the new points' categories and spans use
    it)."""
    _check(lib().trime_add_points(C.byref(state), int(n_add), _stream(stream)))


def run_growing(state, mode, max_iter, n_total, t_add=0.002, fac_add=0.6, t_quality=0.001, t_amax=0.005,
                t_switch=0.0015, stream=None):
    """Adaptive run with point addition up to n_total points (h read times
    sqrt(n_grid / n) as the count grows); the outcome is in the stats."""
    m = {"dm": ADAPT_DM, "cvd": ADAPT_CVD, "hybrid": ADAPT_HYBRID}[mode]
    cfg = Growing(Adaptive(m, int(max_iter), float(t_quality), float(t_amax), float(t_switch)), int(n_total),
                  float(t_add), float(fac_add))
    _check(lib().trime_run_growing(C.byref(state), C.byref(cfg), _stream(stream)))


def auto_sizing(geo, sz, grid, pts, medial, keep, lfs, stream=None):
    """Boundary points, medial points with keep flags and lfs of the
    automatic sizing field into device tensors; returns (ns, nm)."""
    ns, nm = C.c_int64(0), C.c_int64(0)
    _check(lib().trime_auto_sizing(C.byref(geo), C.byref(sz), C.byref(grid), _ptr(pts), pts.numel() // 2,
                                   C.byref(ns), _ptr(medial), _ptr(keep), medial.numel() // 2, C.byref(nm), _ptr(lfs),
                                   _stream(stream)))
    return ns.value, nm.value


def quality(state, stream=None):
    _check(lib().trime_quality(C.byref(state), _stream(stream)))


def export_points(state, x, y, cat, stream=None):
    _check(lib().trime_export_points(C.byref(state), _ptr(x), _ptr(y), _ptr(cat), _stream(stream)))


def export_triangles(state, tri, valid, count, stream=None):
    _check(lib().trime_export_triangles(C.byref(state), _ptr(tri), _ptr(valid), tri.shape[0], _ptr(count),
                                        _stream(stream)))


def export_adjacency(state, deg, col, stream=None):
    _check(lib().trime_export_adjacency(C.byref(state), _ptr(deg), _ptr(col), _stream(stream)))


def autotune_workspace_bytes(state, densities) -> int:
    d = (C.c_double * len(densities))(*densities)
    n = C.c_size_t(0)
    _check(lib().trime_autotune_workspace_bytes(C.byref(state), d, len(densities), C.byref(n)))
    return n.value


def autotune(state, ws, x, y, densities, n_iter, xcd_runs=None, stream=None):
    """Returns (best density, best XCD run, ms per iteration of each
    (density, run) candidate, density-major)."""
    d = (C.c_double * len(densities))(*densities)
    runs = list(xcd_runs) if xcd_runs else []
    r = (C.c_int32 * max(len(runs), 1))(*(runs or [0]))
    ms = (C.c_float * (len(densities) * max(len(runs), 1)))()
    best = C.c_double(0)
    best_r = C.c_int32(0)
    _check(lib().trime_autotune(C.byref(state), _ptr(ws), ws.numel() * ws.element_size(), _ptr(x), _ptr(y), d,
                                len(densities), r if runs else None, len(runs), int(n_iter), C.byref(best),
                                C.byref(best_r), ms, _stream(stream)))
    return best.value, best_r.value, list(ms)


def batch_graph_create(states, method, n_iter, nstreams, stream):
    """One graph of n_iter iterations of every state (method METHOD_DM or
    METHOD_CVD), captured on `stream` (not the null stream)."""
    arr = (C.POINTER(State) * len(states))(*[C.pointer(s) for s in states])
    g = C.c_void_p()
    _check(lib().trime_batch_graph_create(arr, len(states), int(method), int(n_iter), int(nstreams), C.byref(g),
                                          _stream(stream)))
    return g


def batch_create(states, method):
    """A batch running every kernel of an iteration once for all states
    (method METHOD_DM, METHOD_CVD or METHOD_DM_ALWAYS: DistMesh re-triangulating
    every iteration); synchronises (uploads its tables)."""
    arr = (C.POINTER(State) * len(states))(*[C.pointer(s) for s in states])
    b = C.c_void_p()
    _check(lib().trime_batch_create(arr, len(states), int(method), C.byref(b)))
    return b


def batch_run(b, n_iter, stream=None):
    _check(lib().trime_batch_run(b, int(n_iter), _stream(stream)))


def batch_make_persistent(b, tiles_cells=1, tiles_other=4):
    """Switches the batch to one persistent launch per batch_run (work items
    of tiles_cells fast-cell tiles or tiles_other blocks of the other bulk
    kernels).  Raises TrimeError unless the library was built with
    TRIME_PERSIST_ENABLE (switched off by default)."""
    _check(lib().trime_batch_make_persistent(b, int(tiles_cells), int(tiles_other)))


def batch_destroy(b):
    _check(lib().trime_batch_destroy(b))


def graph_launch(g, stream=None):
    _check(lib().trime_graph_launch(g, _stream(stream)))


def graph_destroy(g):
    _check(lib().trime_graph_destroy(g))


def stats_read(state, stream=None) -> Stats:
    s = Stats()
    _check(lib().trime_stats_read(C.byref(state), C.byref(s), _stream(stream)))
    return s


def stats_check(stats) -> int:
    return lib(False).trime_stats_check(C.byref(stats))
