"""The library's kernels and host code run on the CPU (tests/cpu_emu: a
stand-in HIP runtime whose block threads are fibers) under
AddressSanitizer and UndefinedBehaviorSanitizer: whole CVD iterations with
every pass and the hand-off between them (fast kernel -> FP64 replay and
deferred-centroid queues -> exact stage), each iteration fed by the previous
one's output, every buffer of the state in an allocation of its own and the
queue counts checked against their capacities after every launch.  The
positions are compared with the oracle's iterations.  The persistent batch
kernel runs there too, its blocks taking turns where a block sleeps in a wait
or fences between two work items (the schedule's tables, item decoding and
waits, and every kernel's one-wavefront form), against the same shapes run
alone."""
import os
import struct
import subprocess

import numpy as np
import pytest

from paper_2309_13824_amd import inputs as I
from tests.cpu_emu import build as EB

FP64, FP32 = 0, 1


@pytest.fixture(scope="module")
def exe():
    return EB.build()


def write_case(path, wl, og, prec, density, iters, method=1):
    g = wl.grid
    dt = np.float32 if g.dtype_bytes == 4 else np.float64
    area = float(np.count_nonzero(og.cat)) * g.dx * g.dy  # bin sizing only, as the Mesher passes it
    with open(path, "wb") as f:
        f.write(struct.pack("<qiiddddiidii", wl.n, g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, g.dtype_bytes, prec,
                            density, iters, method))
        f.write(np.ascontiguousarray(og.sdf, dt).tobytes())
        f.write(np.ascontiguousarray(og.mu, dt).tobytes())
        f.write(np.ascontiguousarray(og.cat, np.uint8).tobytes())
        f.write(np.ascontiguousarray(og.hcell, np.float32).tobytes())
        f.write(np.array([og.H, og.h_avg, area, 0.0], np.float64).tobytes())
        f.write(np.ascontiguousarray(wl.x, np.float64).tobytes())
        f.write(np.ascontiguousarray(wl.y, np.float64).tobytes())


def run(exe, tmp_path, wl, og, prec, density, iters, timeout=1800):
    from paper_2309_13824_amd import trime as T
    cin, cout = str(tmp_path / "case.bin"), str(tmp_path / "out.bin")
    write_case(cin, wl, og, prec, density, iters)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, cin, cout], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=timeout, env=env)
    assert r.returncode == 0, r.stdout[-6000:]
    print(r.stdout.strip().splitlines()[-1], flush=True)
    n = wl.n
    raw = open(cout, "rb").read()
    its, off = [], 0
    for _ in range(iters):
        x = np.frombuffer(raw, np.float64, n, off)
        y = np.frombuffer(raw, np.float64, n, off + 8 * n)
        c = np.frombuffer(raw, np.uint8, n, off + 16 * n)
        its.append((x, y, c))
        off += 17 * n
    st = T.Stats.from_buffer_copy(raw[off:off + C_sizeof(T.Stats)])
    maxq = np.frombuffer(raw, np.int64, 3, off + C_sizeof(T.Stats))
    return its, st, maxq


def C_sizeof(t):
    import ctypes
    return ctypes.sizeof(t)


def h_of(og, x, y):
    fx = np.floor((x - og.x0) * (1.0 / og.dx)).astype(int)
    fy = np.floor((y - og.y0) * (1.0 / og.dy)).astype(int)
    return og.hcell[fy * (og.nx - 1) + fx].astype(np.float64)


def oracle_iterations(orc, og, wl, iters):
    x, y = wl.x.copy(), wl.y.copy()
    cat = orc.initial_categories(og, x, y)
    dprev = np.full(wl.n, -1.0)
    out = []
    for _ in range(iters):
        x, y, cat, dprev, _, _ = orc.cvd_step(og, x, y, cat, dprev, nthreads=8)
        out.append((x, y, cat))
    return out


def check(its, ref, og, prec):
    tol = 1e-11 if prec == FP64 else 1e-5
    for k, ((x, y, c), (xr, yr, cr)) in enumerate(zip(its, ref)):
        err = np.hypot(x - xr, y - yr) / h_of(og, xr, yr)
        assert err.max() <= tol * (k + 1), (k, err.max())
        assert np.array_equal(c, cr), k


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_emulated_cvd_iterations(orc, exe, tmp_path, prec):
    """Two CVD iterations of a small holes20 case at a grid whose box is
    within reach of the boundary points' octagons (they take the exact
    stage): no sanitizer report, queues within capacity, positions as the
    oracle's."""
    wl = I.holes20(n=1500, grid_n=128, iters=1)
    og = orc.build_grid(wl)
    its, st, maxq = run(exe, tmp_path, wl, og, prec, 3.3, 2)
    assert st.error == 0
    assert maxq[1] > 0  # points reached the exact stage (the box within reach)
    check(its, oracle_iterations(orc, og, wl, 2), og, prec)


def run_method(exe, tmp_path, wl, og, prec, method, iters=1):
    cin, cout = str(tmp_path / "case.bin"), str(tmp_path / "out.bin")
    write_case(cin, wl, og, prec, 3.3, iters, method=method)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, cin, cout], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-6000:]
    return open(cout, "rb").read()


def parse_cells_and_mesh(raw, n):
    """Method 4's output: cells by id, the triangles with validity, the
    adjacency rows by id, then the stats."""
    from paper_2309_13824_amd import trime as T
    cap, off = 64, 0
    ncons = np.frombuffer(raw, np.int32, n, off); off += 4 * n
    cons = np.frombuffer(raw, np.int32, n * cap, off).reshape(n, cap); off += 4 * n * cap
    cnt = int(np.frombuffer(raw, np.int64, 1, off)[0]); off += 8
    tri = np.frombuffer(raw, np.int32, 3 * cnt, off).reshape(cnt, 3); off += 12 * cnt
    valid = np.frombuffer(raw, np.uint8, cnt, off); off += cnt
    md = int(np.frombuffer(raw, np.int32, 1, off)[0]); off += 4
    deg = np.frombuffer(raw, np.int32, n, off); off += 4 * n
    col = np.frombuffer(raw, np.int32, n * md, off).reshape(n, md); off += 4 * n * md
    st = T.Stats.from_buffer_copy(raw[off:off + C_sizeof(T.Stats)])
    cells = [tuple(int(v) for v in cons[i, :ncons[i]]) if ncons[i] >= 0 else None for i in range(n)]
    tris = {(tuple(int(v) for v in t), int(f)) for t, f in zip(tri, valid)}
    rows = [tuple(int(v) for v in col[i, :deg[i]]) for i in range(n)]
    return cells, tris, rows, st


TINY = [1, 2, 3, 5, "collinear", "coincident", "near", "disk_ties"]


def tiny_workload(case):
    return I.random_box(case, seed=5 + case) if isinstance(case, int) else I.degenerate(case)


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("case", TINY)
def test_emulated_tiny_inputs(orc, exe, tmp_path, case, prec):
    """One to five points in a box, the degenerate sets (collinear,
    coincident, 1e-13 apart), and 600 disk points with some on the boundary
    circle, on grid nodes and on a lattice block (exact-stage ties).  The cells, the triangles with validity and the
    adjacency after one binning and extraction, two CVD iterations and one
    DistMesh step, each against the oracle, with no sanitizer report and the
    queues within capacity."""
    wl = tiny_workload(case)
    n = wl.n
    og = orc.build_grid(wl)
    cells, tris, rows, st = parse_cells_and_mesh(run_method(exe, tmp_path, wl, og, prec, 4), n)
    assert st.error == 0
    ref_cells, _ = orc.cells(og, wl.x, wl.y)
    assert cells == ref_cells
    ref = orc.triangulate(og, wl.x, wl.y)
    assert tris == {(tuple(int(v) for v in t), int(f)) for t, f in zip(ref.tri, ref.valid)}
    assert rows == [tuple(int(v) for v in ref.col[ref.rowptr[i]:ref.rowptr[i + 1]]) for i in range(n)]
    q = orc.quality(wl.x, wl.y, ref.tri, ref.valid)
    assert np.array_equal(st.as_dict()["hist_beta"], np.round(q["hist_beta"] * q["ntri"]).astype(np.int64))
    its, st, _ = run(exe, tmp_path, wl, og, prec, 3.3, 2)
    assert st.error == 0
    check(its, oracle_iterations(orc, og, wl, 2), og, prec)
    raw = run_method(exe, tmp_path, wl, og, prec, 0)
    x, y, c = (np.frombuffer(raw, np.float64, n, 0), np.frombuffer(raw, np.float64, n, 8 * n),
               np.frombuffer(raw, np.uint8, n, 16 * n))
    cat0 = orc.initial_categories(og, wl.x, wl.y)
    xr, yr, cr, _, _, _ = orc.dm_step(og, wl.x, wl.y, cat0, ref)
    err = np.hypot(x - xr, y - yr) / h_of(og, xr, yr)
    assert err.max() <= (1e-12 if prec == FP64 else 1e-5), err.max()
    assert np.array_equal(c, cr)


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("method", [1, 0, 4])
def test_emulated_points_off_the_grid(orc, exe, tmp_path, method, prec):
    """Two points outside the grid's box (one just below it, one far away)
    among 600 disk points: a CVD step, a DistMesh step, and the cells and
    extraction run with no sanitizer report and the queues within capacity;
    the two points keep their positions and the stats carry the error."""
    wl = I.disk(n=600)
    wl.x[2], wl.y[2] = 0.0, -1.25
    wl.x[3], wl.y[3] = 5.0, 7.0
    og = orc.build_grid(wl)
    raw = run_method(exe, tmp_path, wl, og, prec, method)
    n = wl.n
    if method == 4:
        st = parse_cells_and_mesh(raw, n)[3]
    else:
        x, y = np.frombuffer(raw, np.float64, n, 0), np.frombuffer(raw, np.float64, n, 8 * n)
        assert (x[2], y[2], x[3], y[3]) == (0.0, -1.25, 5.0, 7.0)
        assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
        st = T_stats(raw[17 * n:])
    assert st.error != 0


def T_stats(raw):
    from paper_2309_13824_amd import trime as T
    return T.Stats.from_buffer_copy(raw[:C_sizeof(T.Stats)])


@pytest.mark.slow
@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("density", [3.3, 1.5, 7.0])
def test_emulated_bin_size_case(orc, exe, tmp_path, prec, density):
    """The case of the bin-size independence test at full size: holes20 with
    20,000 points on a 512^2 grid, three CVD iterations, at three bin
    densities (points per bin)."""
    wl = I.holes20(n=20000, grid_n=512, iters=1)
    og = orc.build_grid(wl)
    its, st, maxq = run(exe, tmp_path, wl, og, prec, density, 3)
    print("queues: replay %d, exact %d, deferred %d" % tuple(maxq), flush=True)
    assert st.error == 0
    assert maxq[1] > 0
    check(its, oracle_iterations(orc, og, wl, 3), og, prec)


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("method", ["dm", "cvd"])
def test_emulated_persistent_batch(orc, exe, tmp_path, method, prec):
    """A persistent batch of two shapes (1,500 holes20 points and the first
    500 of them, on a 128^2 grid whose box the boundary points' octagons
    reach), four blocks taking turns: four iterations, after every two the
    positions, categories and statistics of each shape bit-identical to the
    shape run alone, no sanitizer report, queues within capacity, and the
    blocks did wait on each other."""
    wl = I.holes20(n=1500, grid_n=128, iters=1)
    og = orc.build_grid(wl)
    cin, cout = str(tmp_path / "case.bin"), str(tmp_path / "out.bin")
    write_case(cin, wl, og, prec, 3.3, 4, method=2 if method == "dm" else 3)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, cin, cout], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=1800, env=env)
    assert r.returncode == 0, r.stdout[-6000:]
    last = r.stdout.strip().splitlines()[-1]
    print(last, flush=True)
    turns = int(last.split(",")[-1].split()[0])
    assert turns > 0, last  # the blocks took turns
