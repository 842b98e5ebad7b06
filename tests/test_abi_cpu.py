"""The C ABI without a GPU: the library loads, exports every function the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trime.h")
LIB = os.path.join(ROOT, "paper_2309_13824_amd", "libtrime.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trime_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def T():
    if not os.path.exists(LIB):
        from paper_2309_13824_amd import build
        build.build()
    from paper_2309_13824_amd import trime
    return trime


def test_header_declares_the_entry_points():
    names = declared()
    for f in ("trime_sdf_grid_build", "trime_bin_points", "trime_voronoi_cells", "trime_delaunay_extract",
              "trime_step_dm", "trime_step_cvd", "trime_step_hybrid"):
        assert f in names


def test_library_exports_every_declared_symbol(T):
    L = T.lib(require_gpu=False)
    for f in declared():
        assert hasattr(L, f), f
    assert set(declared()) == set(T.EXPORTED)


def test_version_and_defaults(T):
    L = T.lib(require_gpu=False)
    assert L.trime_version().startswith(b"trime")
    p = T.default_params()
    assert (p.fac_F, p.fac_voro, p.fac_pt, p.fac_retria, p.fac_end, p.fac_geps, p.T_tria, p.alpha_hat,
            p.T_newton) == (1.2, 5.0, 0.4, 0.1, 0.001, 0.01, 0.4, 1.0, 10)


def test_null_and_bad_arguments_rejected_on_host(T):
    L = T.lib(require_gpu=False)
    # grid build with null geometry
    g = T.Grid(16, 16, 0.0, 0.0, 0.1, 0.1, 8)
    rc = L.trime_sdf_grid_build(None, None, C.byref(g), 100, None, None, None, None, None, None)
    assert rc == 1 and b"null" in L.trime_last_error()
    # bad grid dtype
    g2 = T.Grid(16, 16, 0.0, 0.0, 0.1, 0.1, 3)
    st = T.State()
    st.n = 10
    st.grid = g2
    b = C.c_size_t()
    assert L.trime_state_workspace_bytes(C.byref(st), C.byref(b)) == 1
    # missing grid arrays
    st.grid = g
    assert L.trime_state_workspace_bytes(C.byref(st), C.byref(b)) == 1
    # unbound state
    st.sdf = st.mu = st.cat_grid = st.hcell = st.scal = 256
    assert L.trime_step_cvd(C.byref(st), 1, None) == 1
    assert L.trime_bin_points(C.byref(st), None) == 1
    # negative, zero and too large n (at most 2^30 points)
    for n in (-5, 0, (1 << 30) + 1):
        st.n = n
        assert L.trime_state_workspace_bytes(C.byref(st), C.byref(b)) == 1
        assert b"bad n" in L.trime_last_error()
    # bad precision
    st.n = 10
    st.precision = 7
    assert L.trime_state_workspace_bytes(C.byref(st), C.byref(b)) == 1


def test_schedule_validation(T):
    L = T.lib(require_gpu=False)
    st = T.State()
    assert L.trime_step_hybrid(C.byref(st), None, None) == 1


def test_adaptive_configuration_rejected_on_host(T):
    """Unbound state, null configuration, unknown mode, negative budget and
    negative or NaN thresholds return TRIME_EINVAL before anything is
    launched (the state below only looks bound: none of its pointers is ever
    dereferenced on these paths)."""
    L = T.lib(require_gpu=False)
    st = T.State()
    good = T.Adaptive(T.ADAPT_HYBRID, 10, 0.001, 0.005, 0.0015)
    assert L.trime_step_adaptive(C.byref(st), C.byref(good), None) == 1
    st.n = 10
    st.grid = T.Grid(16, 16, 0.0, 0.0, 0.1, 0.1, 8)
    st.sdf = st.mu = st.cat_grid = st.hcell = st.scal = 256
    st.stats = 512
    st.pos[0].x = 768
    assert L.trime_step_adaptive(C.byref(st), None, None) == 1
    for bad in (T.Adaptive(7, 10, 0.001, 0.005, 0.0015), T.Adaptive(T.ADAPT_DM, -1, 0.001, 0.005, 0.0015),
                T.Adaptive(T.ADAPT_CVD, 10, -0.001, 0.005, 0.0015),
                T.Adaptive(T.ADAPT_CVD, 10, 0.001, float("nan"), 0.0015),
                T.Adaptive(T.ADAPT_HYBRID, 10, 0.001, 0.005, -1.0)):
        assert L.trime_step_adaptive(C.byref(st), C.byref(bad), None) == 1
        assert b"trime_step_adaptive" in L.trime_last_error()


def test_growing_configuration_rejected_on_host(T):
    """Point addition and growing runs: a capacity below n, n_add outside
    [0, n_cap - n], a negative n_grid, n_total outside [n, n_cap], a negative
    t_add and fac_add <= 0 return TRIME_EINVAL on the host (the state only
    looks bound, as above)."""
    L = T.lib(require_gpu=False)
    st = T.State()
    st.n = 10
    st.grid = T.Grid(16, 16, 0.0, 0.0, 0.1, 0.1, 8)
    st.sdf = st.mu = st.cat_grid = st.hcell = st.scal = 256
    st.stats = 512
    st.pos[0].x = 768
    st.n_cap = 5
    assert L.trime_add_points(C.byref(st), 1, None) == 1
    assert b"n_cap" in L.trime_last_error()
    st.n_cap = 20
    for n_add in (-1, 11):
        assert L.trime_add_points(C.byref(st), n_add, None) == 1
        assert b"trime_add_points" in L.trime_last_error()
    st.n_grid = -5
    assert L.trime_add_points(C.byref(st), 1, None) == 1
    assert b"n_grid" in L.trime_last_error()
    st.n_grid = 20
    base = T.Adaptive(T.ADAPT_HYBRID, 10, 0.001, 0.005, 0.0015)
    assert L.trime_run_growing(C.byref(st), None, None) == 1
    for n_total, t_add, fac in ((9, 0.002, 0.6), (21, 0.002, 0.6), (20, -0.1, 0.6), (20, 0.002, 0.0),
                                (20, float("nan"), 0.6)):
        assert L.trime_run_growing(C.byref(st), C.byref(T.Growing(base, n_total, t_add, fac)), None) == 1
        assert b"trime_run_growing" in L.trime_last_error()
    bad_mode = T.Adaptive(9, 10, 0.001, 0.005, 0.0015)
    assert L.trime_run_growing(C.byref(st), C.byref(T.Growing(bad_mode, 20, 0.002, 0.6)), None) == 1


def test_auto_sizing_arguments_rejected_on_host(T):
    """trime_auto_sizing: null outputs, a sizing kind other than AUTO, a
    nonpositive fac_s, a negative K and a bad polygon range return
    TRIME_EINVAL before any device work; too small outputs return
    TRIME_ECAPACITY with the boundary-point count."""
    L = T.lib(require_gpu=False)
    verts = np.array([[0.2, 0.2], [0.2, 0.8], [0.8, 0.8], [0.8, 0.2]], np.float64).reshape(-1)
    prims = (T.Prim * 1)()
    prims[0].op, prims[0].kind, prims[0].voff, prims[0].nv = 0, 4, 0, 4
    geo = T.Geometry(1, prims, 4, verts.ctypes.data_as(C.POINTER(C.c_double)))
    grid = T.Grid(64, 64, 0.0, 0.0, 1.0 / 63, 1.0 / 63, 8)
    ns, nm = C.c_int64(0), C.c_int64(0)
    good = T.Sizing(4, 0.1, 0.5, 0.0, 0, None, 0, None, 0, 0.0, 0.0)
    fake = C.c_void_p(256)

    def call(sz, g=geo, s_cap=10 ** 6, m_cap=10 ** 6, out=fake):
        return L.trime_auto_sizing(C.byref(g), C.byref(sz), C.byref(grid), out, s_cap, C.byref(ns), out, out, m_cap,
                                   C.byref(nm), out, None)

    assert call(good, out=None) == 1
    for bad in (T.Sizing(0, 0.1, 0.5, 0.0, 0, None, 0, None, 0, 0.0, 0.0),
                T.Sizing(4, 0.1, 0.0, 0.0, 0, None, 0, None, 0, 0.0, 0.0),
                T.Sizing(4, -0.1, 0.5, 0.0, 0, None, 0, None, 0, 0.0, 0.0),
                T.Sizing(4, 0.1, 0.5, 0.0, 0, None, 0, None, -1, 0.0, 0.0)):
        assert call(bad) == 1
        assert b"trime_auto_sizing" in L.trime_last_error()
    prims[0].nv = 9  # beyond npoly
    assert call(good) == 1 and b"polygon" in L.trime_last_error()
    prims[0].nv = 4
    assert call(good, s_cap=3) == 3  # TRIME_ECAPACITY before any device work
    assert ns.value > 3 and nm.value == -1


def test_batch_arguments_rejected_on_host(T):
    L = T.lib(require_gpu=False)
    out = C.c_void_p()
    assert L.trime_batch_create(None, 1, 0, C.byref(out)) == 1
    st = T.State()
    arr = (C.POINTER(T.State) * 1)(C.pointer(st))
    assert L.trime_batch_create(arr, 1, 0, C.byref(out)) == 1  # unbound state
    assert L.trime_batch_create(arr, 1, 5, C.byref(out)) == 1  # bad method
    assert L.trime_batch_run(None, 2, None) == 1
    assert L.trime_batch_destroy(None) == 0


def test_placement_and_persistent_batch_rejected_on_host(T):
    """An XCD run outside [0, 256] is refused by every entry point that
    checks the state; trime_autotune refuses such a candidate; the
    persistent batch refuses to switch on (it is built out of the device
    library), leaving the batch as it was."""
    L = T.lib(require_gpu=False)
    st = T.State()
    st.n = 10
    st.grid = T.Grid(16, 16, 0.0, 0.0, 0.1, 0.1, 8)
    st.sdf = st.mu = st.cat_grid = st.hcell = st.scal = 256
    st.stats = 512
    st.pos[0].x = 768
    st.n_cap = 20
    for bad in (-1, 257):
        st.xcd_run = bad
        assert L.trime_add_points(C.byref(st), 1, None) == 1
        assert b"xcd_run" in L.trime_last_error()
    st.xcd_run = 0
    d = (C.c_double * 1)(2.0)
    runs = (C.c_int32 * 2)(8, 300)
    best, best_r = C.c_double(0), C.c_int32(0)
    assert L.trime_autotune(C.byref(st), C.c_void_p(256), 1 << 20, C.c_void_p(256), C.c_void_p(256), d, 1, runs, 2,
                            2, C.byref(best), C.byref(best_r), None, None) == 1
    assert b"trime_autotune" in L.trime_last_error()
    assert L.trime_batch_make_persistent(None, 1, 4) == 1
    assert b"switched off" in L.trime_last_error()


def test_stats_check_codes(T):
    L = T.lib(require_gpu=False)
    s = T.Stats()
    assert L.trime_stats_check(C.byref(s)) == 0
    s.error = 1
    assert L.trime_stats_check(C.byref(s)) == 3
    s.error = 0
    s.empty_cells = 2
    assert L.trime_stats_check(C.byref(s)) == 5


def test_struct_sizes_match_header(T):
    """The ctypes mirrors have the sizes the C compiler gives the structs."""
    import subprocess
    import tempfile
    src = r'''
#include <stdio.h>
#include "trime.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(trime_prim), sizeof(trime_sizing), sizeof(trime_grid),
         sizeof(trime_params), sizeof(trime_stats), sizeof(trime_state), sizeof(trime_grid_scalars),
         sizeof(trime_adaptive), sizeof(trime_growing));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(v) for v in out]
    assert sizes == [C.sizeof(T.Prim), C.sizeof(T.Sizing), C.sizeof(T.Grid), C.sizeof(T.Params),
                     C.sizeof(T.Stats), C.sizeof(T.State), C.sizeof(T.GridScalars), C.sizeof(T.Adaptive),
                     C.sizeof(T.Growing)]
