"""Which kernel family a sweep call runs (mc_sweep_path, host only, no GPU),
for the workloads' shapes and the edges of each family: the dispatcher takes
the fused tiles when it can (and a workspace is given), then the whole-
lattice kernels, then the multi-spin-coded kernel, else the generic
half-sweeps."""
import ctypes

import pytest

mcs = pytest.importorskip("paper_1709_04394_amd")
F2, F3, SB, SM, MSC, GEN = 1, 2, 3, 4, 5, 6


@pytest.fixture(scope="module")
def ctx():
    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    yield h
    mcs._lib.mc_ctx_destroy(h)


def _path(ctx, dims, L, rule=mcs.METROPOLIS, J=False, per=False, layout=mcs.INT8, count=1, ws=True):
    g = mcs.make_geom(dims, L, layout=layout, count=count)
    wsb = mcs._lib.mc_sweep_workspace_bytes(ctypes.byref(g)) if ws else 0
    p = ctypes.c_int32()
    rc = mcs._lib.mc_sweep_path(ctx, ctypes.byref(g), rule, int(J), int(per), ctypes.c_size_t(wsb), ctypes.byref(p))
    return rc if rc else p.value


@pytest.mark.parametrize("args,kw,want", [
    ((2, 4096), dict(count=3), F2),                                   # the headline workload
    ((2, 4096), dict(count=3, ws=False), GEN),                        # no workspace: too big for one workgroup
    ((2, 4096), dict(rule=mcs.HEATBATH), GEN),                         # the 2D tiles do Metropolis only
    ((2, 4096), dict(J=True), GEN),                                    # ... and J = 1 only
    ((3, 256), dict(rule=mcs.HEATBATH), F3),                           # 3D heat-bath 256^3
    ((3, 256), dict(rule=mcs.HEATBATH, per=True, count=4), F3),        # its four runs in one call
    ((3, 32), dict(J=True), SB),                                       # the spin-glass 32^3
    ((2, 32), dict(per=True), SB),                                     # per-lattice tables, no fused tiles:
    ((2, 32), dict(per=True, count=3), SB),                            # ... each lattice alone on its own path
    ((2, 4096), dict(count=3, per=True), F2),                          # the headline call (mc_sweep_betas)
    ((2, 4096), dict(count=3, per=True, ws=False), GEN),               # ... without a workspace
    ((3, 256), dict(rule=mcs.HEATBATH, per=True, count=4, ws=False), GEN),
    ((2, 64), dict(per=True, count=3), F2),
    ((2, 64), dict(per=True, count=3, ws=False), SM),
    ((2, (36, 20)), dict(per=True, count=3), SM),                      # Lx not a multiple of 64
    ((3, 32), dict(per=True, count=2, J=True), SB),
    ((2, 64), dict(ws=False), SM),                                     # a whole small lattice in LDS
    ((2, (96, 64)), dict(), SM),
    ((2, 4096), dict(layout=mcs.MSC64), MSC),                          # 64-lane words, Lx a multiple of 128
    ((3, 256), dict(layout=mcs.MSC64, rule=mcs.HEATBATH), MSC),
    ((2, (96, 96)), dict(layout=mcs.MSC64), GEN),
    ((2, (2048, 2048)), dict(rule=mcs.HEATBATH, J=True), GEN),         # above the small kernels' LDS
])
def test_paths(ctx, args, kw, want):
    assert _path(ctx, *args, **kw) == want


def test_errors(ctx):
    assert _path(ctx, 2, 64, layout=mcs.MSC64, per=True) == mcs.MC_E_LAYOUT
    assert _path(ctx, 2, 64, rule=7) == mcs.MC_E_INVAL
    g = mcs.make_geom(2, 64)
    assert mcs._lib.mc_sweep_path(ctx, ctypes.byref(g), 0, 0, 0, 0, None) == mcs.MC_E_INVAL
    bad = mcs.Geom(2, 5, 8, 1, mcs.INT8, 1)
    p = ctypes.c_int32()
    assert mcs._lib.mc_sweep_path(ctx, ctypes.byref(bad), 0, 0, 0, 0, ctypes.byref(p)) == mcs.MC_E_SHAPE
