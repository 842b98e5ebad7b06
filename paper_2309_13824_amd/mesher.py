"""A meshing run on one GPU: owns the device tensors of one workload and
calls the C ABI (paper_2309_13824_amd.trime) for every step."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import trime as T


def _geometry(wl):
    poly, offs = wl.poly_array()
    prims = (T.Prim * len(wl.prims))()
    for k, pr in enumerate(wl.prims):
        prims[k].op = pr.op
        prims[k].kind = pr.kind
        for t, v in enumerate(pr.p):
            prims[k].p[t] = float(v)
        prims[k].voff, prims[k].nv = offs[k]
    poly = np.ascontiguousarray(poly.reshape(-1), np.float64)
    geo = T.Geometry(len(wl.prims), prims, len(poly) // 2, poly.ctypes.data_as(C.POINTER(C.c_double)))
    s = wl.sizing
    cent = np.ascontiguousarray(np.asarray(s.cent, np.float64).reshape(-1))
    holes = np.ascontiguousarray(np.asarray(s.holes, np.int32))
    sz = T.Sizing(s.kind, s.a0, s.a1, s.s2, len(cent) // 2, cent.ctypes.data_as(C.POINTER(C.c_double)),
                  len(holes), holes.ctypes.data_as(C.POINTER(C.c_int32)), s.n_thres, s.fac_nei, s.fac_geps)
    return geo, sz, (prims, poly, cent, holes)


class Mesher:
    """Grid + state of one workload on the current HIP device."""

    def __init__(self, wl, precision=T.FP64, max_deg=16, params=None, bin_density=0.0, device="cuda",
                 grid=None, n_init=None):
        """grid: None builds the geometry grid on the GPU (trime_sdf_grid_build);
        otherwise an object with sdf, mu, cat, hcell (node / cell arrays), H and
        h_avg whose arrays are uploaded as the grid (a grid built elsewhere).
        n_init: the state starts with the first n_init of the workload's
        points and has room for all of them (point addition, run_growing);
        the grid is built for all, h scaled by sqrt(N / n_init)."""
        import torch
        T.lib()
        self.torch = torch
        self.wl = wl
        self.dev = torch.device(device)
        g = wl.grid
        self.grid = T.Grid(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, g.dtype_bytes)
        gd = torch.float32 if g.dtype_bytes == 4 else torch.float64
        nn, nc = g.nx * g.ny, (g.nx - 1) * (g.ny - 1)
        if grid is None:
            self.sdf = torch.empty(nn, dtype=gd, device=self.dev)
            self.mu = torch.empty(nn, dtype=gd, device=self.dev)
            self.cat = torch.empty(nc, dtype=torch.uint8, device=self.dev)
            self.hcell = torch.empty(nc, dtype=torch.float32, device=self.dev)
            self.scal = torch.zeros(4, dtype=torch.float64, device=self.dev)
            geo, sz, keep = _geometry(wl)
            T.sdf_grid_build(geo, sz, self.grid, wl.n, self.sdf, self.mu, self.cat, self.hcell, self.scal)
            torch.cuda.synchronize()
            del keep
        else:
            up = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), device=self.dev).to(dt)  # noqa: E731
            self.sdf = up(grid.sdf, gd)
            self.mu = up(grid.mu, gd)
            self.cat = up(grid.cat, torch.uint8)
            self.hcell = up(grid.hcell, torch.float32)
            area = float(np.count_nonzero(grid.cat)) * g.dx * g.dy  # bin sizing only
            self.scal = torch.tensor([grid.H, grid.h_avg, area, 0.0], dtype=torch.float64, device=self.dev)
        st = T.State()
        n0 = wl.n if n_init is None else int(n_init)
        st.n = n0
        st.n_cap = wl.n
        st.n_grid = wl.n  # the grid is built for all of the workload's points
        st.precision = precision
        st.max_deg = max_deg
        st.bin_density = bin_density
        st.grid = self.grid
        st.sdf, st.mu = self.sdf.data_ptr(), self.mu.data_ptr()
        st.cat_grid, st.hcell, st.scal = self.cat.data_ptr(), self.hcell.data_ptr(), self.scal.data_ptr()
        st.params = params if params is not None else T.default_params()
        self.state = st
        nbytes = T.state_workspace_bytes(st)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        T.state_bind(st, self.ws)
        self.n = n0

    # ---------------------------------------------------------------- input
    def load(self, x=None, y=None):
        torch = self.torch
        x = self.wl.x[:self.n] if x is None else x
        y = self.wl.y[:self.n] if y is None else y
        self.x_in = torch.as_tensor(np.ascontiguousarray(x, np.float64), device=self.dev)
        self.y_in = torch.as_tensor(np.ascontiguousarray(y, np.float64), device=self.dev)
        T.state_load(self.state, self.x_in, self.y_in)

    # ---------------------------------------------------------------- steps
    def bin(self):
        T.bin_points(self.state)

    def extract(self):
        T.delaunay_extract(self.state)

    def cells(self, cap=64):
        torch = self.torch
        cons = torch.full((self.n * cap,), -99, dtype=torch.int32, device=self.dev)
        ncons = torch.zeros(self.n, dtype=torch.int32, device=self.dev)
        out = T.Cells(cap, cons.data_ptr(), ncons.data_ptr())
        T.voronoi_cells(self.state, out)
        cons = cons.view(self.n, cap).cpu().numpy()
        ncons = ncons.cpu().numpy()
        return [tuple(int(v) for v in cons[i, :ncons[i]]) if ncons[i] >= 0 else None for i in range(self.n)]

    def autotune(self, densities=(2.0, 3.3, 5.0, 8.0), n_iter=3, x=None, y=None, xcd_runs=None):
        """Picks the bin density (points per bin) and, given xcd_runs, the
        XCD run of the fused cell kernel with the fastest CVD iterations on
        this workload; the state is left loaded with (x, y).  Returns the
        density and the ms of every candidate (keyed by density, or by
        (density, run) when xcd_runs is given).  The results do not depend
        on the choice."""
        torch = self.torch
        need = T.autotune_workspace_bytes(self.state, densities)
        if need > self.ws.numel():
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.dev)
        x = self.wl.x if x is None else x
        y = self.wl.y if y is None else y
        self.x_in = torch.as_tensor(np.ascontiguousarray(x, np.float64), device=self.dev)
        self.y_in = torch.as_tensor(np.ascontiguousarray(y, np.float64), device=self.dev)
        best, run, ms = T.autotune(self.state, self.ws, self.x_in, self.y_in, densities, n_iter, xcd_runs)
        if not xcd_runs:
            return best, dict(zip(densities, ms))
        keys = [(d, r) for d in densities for r in xcd_runs]
        return best, dict(zip(keys, ms))

    def step_dm(self, n_iter, fresh=True, always=False):
        T.step_dm(self.state, n_iter, fresh, always)

    def step_cvd(self, n_iter):
        T.step_cvd(self.state, n_iter)

    def step_hybrid(self, schedule):
        T.step_hybrid(self.state, schedule)

    def step_adaptive(self, mode, max_iter, t_quality=0.001, t_amax=0.005, t_switch=0.0015):
        """Adaptive run (termination tests, hybrid switch); returns the
        control block: iterations run, switch and stop iterations, reason."""
        T.step_adaptive(self.state, mode, max_iter, t_quality, t_amax, t_switch)
        return self.stats_raw().as_dict()["adapt"]

    def run_growing(self, mode, max_iter, t_add=0.002, fac_add=0.6, t_quality=0.001, t_amax=0.005,
                    t_switch=0.0015):
        """Adaptive run with point addition up to all of the workload's
        points (Sec. 3.6); returns the control block like step_adaptive."""
        T.run_growing(self.state, mode, max_iter, self.wl.n, t_add, fac_add, t_quality, t_amax, t_switch)
        self.n = int(self.state.n)
        return self.stats_raw().as_dict()["adapt"]

    def add_points(self, n_add):
        T.add_points(self.state, n_add)
        self.n = int(self.state.n)

    def quality(self):
        T.quality(self.state)

    # --------------------------------------------------------------- output
    def grid_arrays(self):
        return (self.sdf.double().cpu().numpy(), self.mu.double().cpu().numpy(), self.cat.cpu().numpy(),
                self.hcell.cpu().numpy(), self.scal.cpu().numpy())

    def points(self):
        torch = self.torch
        x = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        y = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        c = torch.empty(self.n, dtype=torch.uint8, device=self.dev)
        T.export_points(self.state, x, y, c)
        return x.cpu().numpy(), y.cpu().numpy(), c.cpu().numpy()

    def triangles(self):
        torch = self.torch
        cap = self.n * T.TRI_PER_POINT
        tri = torch.empty((cap, 3), dtype=torch.int32, device=self.dev)
        valid = torch.empty(cap, dtype=torch.uint8, device=self.dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=self.dev)
        T.export_triangles(self.state, tri, valid, cnt)
        m = int(cnt.item())
        return tri[:m].cpu().numpy(), valid[:m].cpu().numpy()

    def adjacency(self):
        torch = self.torch
        md = self.state.max_deg
        deg = torch.empty(self.n, dtype=torch.int32, device=self.dev)
        col = torch.empty(self.n * md, dtype=torch.int32, device=self.dev)
        T.export_adjacency(self.state, deg, col)
        deg = deg.cpu().numpy()
        col = col.view(self.n, md).cpu().numpy()
        return [tuple(int(v) for v in col[i, :deg[i]]) for i in range(self.n)]

    def stats(self) -> dict:
        return T.stats_read(self.state).as_dict()

    def stats_raw(self):
        return T.stats_read(self.state)

    REASONS = {1: "predicate", 2: "vertex", 3: "polygon", 4: "and_test", 5: "cvd_level", 6: "treatment",
               7: "box", 8: "heavy", 9: "vertex_error"}

    def replay_reasons(self) -> dict:
        """Points sent from the fast kernels to a replay, by reason (since load)."""
        off = self.state.counters - self.ws.data_ptr()
        c = self.ws[off:off + 128].view(self.torch.int32).cpu().numpy()
        return {name: int(c[8 + k]) for k, name in self.REASONS.items()}


class Batch:
    """Many shapes meshed together; the Meshers stay usable one by one.

    kind "kernels" (trime_batch_create): every kernel of an iteration is
    launched once for all shapes; kind "persistent" (the same batch after
    trime_batch_make_persistent, items of `tiles` = (fast-cell tiles, other
    blocks)): one launch per run; kind "graph" (trime_batch_graph_create):
    the shapes' own launches in one graph over nstreams streams."""

    def __init__(self, meshers, method="dm", n_iter=2, nstreams=8, kind="graph", tiles=(1, 4)):
        import torch
        self.torch = torch
        self.meshers = list(meshers)
        self.n_iter = n_iter
        self.kind = kind
        self.stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        meth = {"dm": T.METHOD_DM, "cvd": T.METHOD_CVD, "dm_always": T.METHOD_DM_ALWAYS}[method]
        self.graph = self.batch = None
        if kind in ("kernels", "persistent"):
            self.batch = T.batch_create([m.state for m in self.meshers], meth)
            if kind == "persistent":
                T.batch_make_persistent(self.batch, tiles[0], tiles[1])
        else:
            self.graph = T.batch_graph_create([m.state for m in self.meshers], meth, n_iter, nstreams, self.stream)
        torch.cuda.synchronize()

    def run(self, iters):
        """iters iterations of every shape (a multiple of n_iter)."""
        if iters % self.n_iter:
            raise ValueError("iters must be a multiple of %d" % self.n_iter)
        if self.batch is not None:
            T.batch_run(self.batch, iters, self.stream)
            return
        for _ in range(iters // self.n_iter):
            T.graph_launch(self.graph, self.stream)

    def close(self):
        if self.graph is not None:
            self.torch.cuda.synchronize()
            T.graph_destroy(self.graph)
            self.graph = None
        if self.batch is not None:
            self.torch.cuda.synchronize()
            T.batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
