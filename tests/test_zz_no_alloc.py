"""mc_sweep_noalloc (the sweep with the library's fixed device scratch instead
of a caller workspace) against mc_sweep with a workspace, through the C ABI:
two calls in a row on the same device, the second with a smaller input, so
the second call finds the first call's intermediate lattices in the scratch;
2D and 3D fused geometries, several lattices per call, per-sweep (E, M).
Also: a geometry whose fused scratch is larger than the array is refused
before any device work; geometries without a fused path run without scratch.
Results must be bit-identical (integer spins and energies)."""
import ctypes

import numpy as np
import pytest
import torch

mcs = pytest.importorskip("paper_1709_04394_amd")


def _args(beta, seed, nsw, sweep0=0, replica0=0, rule=0):
    return mcs.SweepArgs(rule, float(beta), seed, replica0, sweep0, nsw)


def _run(ctx_h, dims, shape, count, beta, seed, nsw, rule, noalloc, sweep0=0, replica0=0):
    g = mcs.make_geom(dims, shape, count=count)
    spins = mcs.lattice_tensor(g)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert mcs._lib.mc_init(ctx_h, ctypes.byref(g), ctypes.c_void_p(spins.data_ptr()), mcs.HOT, seed, replica0,
                            stream) == 0
    EM = torch.empty((nsw, count, 2), dtype=torch.int64, device="cuda")
    a = _args(beta, seed, nsw, sweep0, replica0, rule)
    if noalloc:
        rc = mcs._lib.mc_sweep_noalloc(ctx_h, ctypes.byref(g), ctypes.c_void_p(spins.data_ptr()), None,
                                       ctypes.byref(a), ctypes.c_void_p(EM.data_ptr()), stream)
    else:
        ws = torch.empty(max(1, mcs._lib.mc_sweep_workspace_bytes(ctypes.byref(g))), dtype=torch.uint8,
                         device="cuda")
        rc = mcs._lib.mc_sweep(ctx_h, ctypes.byref(g), ctypes.c_void_p(spins.data_ptr()), None, ctypes.byref(a),
                               ctypes.c_void_p(EM.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream)
    assert rc == 0, mcs._lib.mc_ctx_last_error(ctx_h)
    torch.cuda.synchronize()
    return spins.cpu().numpy(), EM.cpu().numpy()


@pytest.fixture(scope="module")
def ctx_h():
    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    yield h
    mcs._lib.mc_ctx_destroy(h)


def test_scratch_size_reported():
    assert mcs._lib.mc_static_scratch_bytes() == 20 << 20


def test_too_large_geometry_refused_before_device_work(ctx_h):
    # five 4096^2 lattices need 2 * 5 * 4096^2 / 8 B = 20 MiB of packed rows and
    # 2 * 640 KiB of (E, M) slots
    g = mcs.make_geom(2, 4096, count=5)
    a = _args(0.44, 1, 3)
    fake = ctypes.c_void_p(1)
    rc = mcs._lib.mc_sweep_noalloc(ctx_h, ctypes.byref(g), fake, None, ctypes.byref(a), None, None)
    assert rc == mcs.MC_E_RANGE
    assert b"static scratch" in mcs._lib.mc_ctx_last_error(ctx_h)
    # the argument checks of mc_sweep come first
    assert mcs._lib.mc_sweep_noalloc(ctx_h, ctypes.byref(g), None, None, ctypes.byref(a), None, None) == \
        mcs.MC_E_INVAL
    assert mcs._lib.mc_sweep_noalloc(None, ctypes.byref(g), fake, None, ctypes.byref(a), None, None) == \
        mcs.MC_E_INVAL


@pytest.mark.gpu
@pytest.mark.parametrize("case", [
    # (dims, first shape, first count, second shape, second count, rule, beta)
    (2, (512, 260), 3, (256, 68), 2, mcs.METROPOLIS, 0.4406868),
    (3, (128, 20, 18), 2, (64, 12, 8), 1, mcs.HEATBATH, 0.2216546),
    (2, (4096, 4096), 4, (1024, 1024), 1, mcs.METROPOLIS, 0.5),
])
def test_noalloc_equals_sweep_with_workspace(ctx_h, case):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dims, shape1, count1, shape2, count2, rule, beta = case
    for shape, count, nsw, seed in ((shape1, count1, 9, 21), (shape2, count2, 7, 22)):
        want = _run(ctx_h, dims, shape, count, beta, seed, nsw, rule, noalloc=False, sweep0=5, replica0=2)
        got = _run(ctx_h, dims, shape, count, beta, seed, nsw, rule, noalloc=True, sweep0=5, replica0=2)
        assert np.array_equal(got[1], want[1]), ("E, M", shape, count)
        assert np.array_equal(got[0], want[0]), ("spins", shape, count)


@pytest.mark.gpu
def test_noalloc_without_fused_path(ctx_h):
    # a lattice with no fused path (Lx not a multiple of 64) needs no scratch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    want = _run(ctx_h, 2, (36, 20), 2, 0.44, 3, 5, mcs.METROPOLIS, noalloc=False)
    got = _run(ctx_h, 2, (36, 20), 2, 0.44, 3, 5, mcs.METROPOLIS, noalloc=True)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
