"""trime_sdf_grid_build_noalloc (the grid build for callers that cannot
allocate: its scratch is a static device array per GPU) against
trime_sdf_grid_build, through the C ABI: the same grids bit for bit, on two
calls in a row, the second with a smaller input, so the second call runs on
what the first left in the shared scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2309_13824_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2309_13824_amd import trime
    trime.lib()
    return trime


def grids(T, wl, noalloc):
    from paper_2309_13824_amd.mesher import _geometry
    g = wl.grid
    grid = T.Grid(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, g.dtype_bytes)
    gd = torch.float32 if g.dtype_bytes == 4 else torch.float64
    nn, nc = g.nx * g.ny, (g.nx - 1) * (g.ny - 1)
    out = (torch.full((nn,), -7.0, dtype=gd, device="cuda"), torch.full((nn,), -7.0, dtype=gd, device="cuda"),
           torch.full((nc,), 255, dtype=torch.uint8, device="cuda"),
           torch.full((nc,), -7.0, dtype=torch.float32, device="cuda"),
           torch.full((4,), -7.0, dtype=torch.float64, device="cuda"))
    geo, sz, keep = _geometry(wl)
    fn = T.sdf_grid_build_noalloc if noalloc else T.sdf_grid_build
    fn(geo, sz, grid, wl.n, *out)
    torch.cuda.synchronize()
    del keep
    return [t.cpu().numpy() for t in out]


def test_noalloc_grid_build_equals_grid_build(T):
    for wl in (I.holes20(n=100000, grid_n=1024, iters=1), I.disk()):  # the second is smaller
        print("%s: %d^2 nodes" % (wl.name, wl.grid.nx), flush=True)
        ref = grids(T, wl, False)
        got = grids(T, wl, True)
        for a, b in zip(ref, got):
            assert a.dtype == b.dtype and a.shape == b.shape
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_noalloc_grid_build_refuses_what_needs_allocation(T):
    wl = I.coast(n=2000, segments=64, grid_n=64, iters=1)  # a segment loop
    with pytest.raises(T.TrimeError):
        grids(T, wl, True)
    # more grid cells than the scratch's partial sums can hold
    big = I.disk()
    big.grid = I.GridSpec(20000, 20000, big.grid.x0, big.grid.y0, big.grid.dx, big.grid.dy, 4)
    from paper_2309_13824_amd.mesher import _geometry
    geo, sz, keep = _geometry(big)
    g = big.grid
    grid = T.Grid(g.nx, g.ny, g.x0, g.y0, g.dx, g.dy, g.dtype_bytes)
    fake = C.c_void_p(256)
    rc = T.lib().trime_sdf_grid_build_noalloc(C.byref(geo), C.byref(sz), C.byref(grid), 1000, fake, fake, fake,
                                             fake, fake, None)
    assert rc == 3  # TRIME_ECAPACITY, before any device work
