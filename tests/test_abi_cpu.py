"""Host-side checks of the C ABI (no GPU needed, no compute call made).

* libmcspin.so loads and exports every function declared in include/*.h;
* argument validation returns the documented codes before any device work
  (only invalid calls are made here, so no pointer is ever dereferenced).
"""
import ctypes
import glob
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
mcs = pytest.importorskip("paper_1709_04394_amd")

FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(mc_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_all_declared_symbols_exported():
    lib = ctypes.CDLL(mcs.LIB_PATH)
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(mcs.exported_symbols()) <= names


def test_abi_version_and_strerror():
    assert mcs.abi_version() == 1
    for code in range(0, -8, -1):
        assert mcs.strerror(code)
    assert "unknown" in mcs.strerror(-99)


@pytest.fixture
def ctx():
    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    yield h
    mcs._lib.mc_ctx_destroy(h)


def _sweep(ctx, geom, args, spins=FAKE):
    return mcs._lib.mc_sweep(ctx, ctypes.byref(geom), spins, None, ctypes.byref(args), None, None, 0, None)


def test_ctx_create_rejects_bad_arguments():
    assert mcs._lib.mc_ctx_create(None, 0) == mcs.MC_E_INVAL
    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), -1) == mcs.MC_E_INVAL


@pytest.mark.parametrize("shape,code", [((2, 5, 8, 1), mcs.MC_E_SHAPE), ((2, 2, 8, 1), mcs.MC_E_SHAPE),
                                        ((2, 8, 8, 3), mcs.MC_E_SHAPE), ((3, 8, 8, 7), mcs.MC_E_SHAPE),
                                        ((4, 8, 8, 8), mcs.MC_E_SHAPE)])
def test_shape_errors(ctx, shape, code):
    g = mcs.Geom(shape[0], shape[1], shape[2], shape[3], mcs.INT8, 1)
    a = mcs.SweepArgs(0, 0.4, 1, 0, 0, 1)
    assert _sweep(ctx, g, a) == code
    assert b"extent" in mcs._lib.mc_ctx_last_error(ctx) or b"dims" in mcs._lib.mc_ctx_last_error(ctx) \
        or b"Lz" in mcs._lib.mc_ctx_last_error(ctx)


@pytest.mark.parametrize("beta", [-0.1, math.nan, math.inf])
def test_beta_range(ctx, beta):
    g = mcs.make_geom(2, 8)
    assert _sweep(ctx, g, mcs.SweepArgs(0, beta, 1, 0, 0, 1)) == mcs.MC_E_RANGE


def test_other_argument_errors(ctx):
    g = mcs.make_geom(2, 8)
    assert _sweep(ctx, g, mcs.SweepArgs(0, 0.4, 1, 0, 0, -1)) == mcs.MC_E_RANGE
    assert _sweep(ctx, g, mcs.SweepArgs(7, 0.4, 1, 0, 0, 1)) == mcs.MC_E_INVAL
    assert _sweep(ctx, g, mcs.SweepArgs(0, 0.4, 1, 0, 0, 1), spins=None) == mcs.MC_E_INVAL
    assert _sweep(ctx, g, mcs.SweepArgs(0, 0.4, 1, 0, 1 << 55, 1)) == mcs.MC_E_RANGE
    gm = mcs.make_geom(2, 8, layout=mcs.MSC64, count=2)
    assert _sweep(ctx, gm, mcs.SweepArgs(0, 0.4, 1, 2 ** 32 - 64, 0, 1)) == mcs.MC_E_RANGE
    bad_layout = mcs.Geom(2, 8, 8, 1, 5, 1)
    assert _sweep(ctx, bad_layout, mcs.SweepArgs(0, 0.4, 1, 0, 0, 1)) == mcs.MC_E_INVAL
    zero = mcs.Geom(2, 8, 8, 1, mcs.INT8, 0)
    assert _sweep(ctx, zero, mcs.SweepArgs(0, 0.4, 1, 0, 0, 1)) == mcs.MC_E_RANGE
    many = mcs.Geom(2, 8, 8, 1, mcs.INT8, 65536)  # one launch dimension per lattice: at most 65535
    assert _sweep(ctx, many, mcs.SweepArgs(0, 0.4, 1, 0, 0, 1)) == mcs.MC_E_RANGE
    assert mcs._lib.mc_init(ctx, ctypes.byref(many), FAKE, 1, 1, 0, None) == mcs.MC_E_RANGE
    assert mcs._lib.mc_measure(ctx, ctypes.byref(many), FAKE, None, FAKE, None) == mcs.MC_E_RANGE
    assert mcs._lib.mc_init(ctx, ctypes.byref(g), FAKE, 2, 1, 0, None) == mcs.MC_E_INVAL
    assert mcs._lib.mc_init(ctx, ctypes.byref(g), None, 1, 1, 0, None) == mcs.MC_E_INVAL
    assert mcs._lib.mc_measure(ctx, ctypes.byref(g), FAKE, None, None, None) == mcs.MC_E_INVAL
    assert mcs._lib.mc_couplings(ctx, ctypes.byref(g), None, 1, None) == mcs.MC_E_INVAL
    assert mcs._lib.mc_sweep(None, ctypes.byref(g), FAKE, None, None, None, None, 0, None) == mcs.MC_E_INVAL


def test_mlp_training_set_matches_oracle(ctx):
    # host-only call: features and targets from converged weights, bit-equal
    # to the oracle's FP64 values rounded to FP32; level k = 1 left out
    import numpy as np
    from oracle import mlp

    rng = np.random.default_rng(3)
    lnW = {L: np.cumsum(rng.normal(0, 2, L * L // 2 + 1)) for L in (4, 6, 12)}
    Ls = sorted(lnW)
    cap = sum(L * L // 2 for L in Ls)
    X = np.zeros((cap, 2), dtype=np.float32)
    Y = np.zeros(cap, dtype=np.float32)
    n = ctypes.c_int32()
    Larr = (ctypes.c_int32 * 3)(*Ls)
    parr = (ctypes.POINTER(ctypes.c_double) * 3)(*[lnW[L].ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for L in Ls])
    fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    assert mcs._lib.mc_mlp_training_set(ctx, 3, Larr, parr, fp(X), fp(Y), cap, ctypes.byref(n)) == 0
    Xo, Yo = mlp.training_set(lnW)
    assert n.value == cap == len(Yo)
    assert np.array_equal(X, Xo.astype(np.float32)) and np.array_equal(Y, Yo.astype(np.float32))
    # too small a buffer, a non-finite weight, an odd L
    assert mcs._lib.mc_mlp_training_set(ctx, 3, Larr, parr, fp(X), fp(Y), cap - 1, ctypes.byref(n)) == mcs.MC_E_RANGE
    lnW[6][5] = np.nan
    assert mcs._lib.mc_mlp_training_set(ctx, 3, Larr, parr, fp(X), fp(Y), cap, ctypes.byref(n)) == mcs.MC_E_RANGE
    lnW[6][5] = 0.0
    lnW[6][1] = np.inf  # the empty level is ignored
    assert mcs._lib.mc_mlp_training_set(ctx, 3, Larr, parr, fp(X), fp(Y), cap, ctypes.byref(n)) == 0
    Larr[0] = 5
    assert mcs._lib.mc_mlp_training_set(ctx, 3, Larr, parr, fp(X), fp(Y), cap, ctypes.byref(n)) == mcs.MC_E_SHAPE


def test_pa_group_setting(ctx):
    """Replicas per workgroup of population annealing: the built-in rule, the
    limits (G <= 64, at most 48 KB of packed lattices per workgroup) and reset."""
    G = ctypes.c_int32()
    builtin = {16: 16, 32: 8, 64: 4, 128: 1, 512: 1}
    for L, g in builtin.items():
        assert mcs._lib.mc_get_pa_group(ctx, L, ctypes.byref(G)) == 0 and G.value == g
    assert mcs._lib.mc_set_pa_group(ctx, 16, 64) == 0
    assert mcs._lib.mc_get_pa_group(ctx, 16, ctypes.byref(G)) == 0 and G.value == 64
    assert mcs._lib.mc_get_pa_group(ctx, 32, ctypes.byref(G)) == 0 and G.value == 8  # other L untouched
    assert mcs._lib.mc_set_pa_group(ctx, 16, 0) == 0
    assert mcs._lib.mc_get_pa_group(ctx, 16, ctypes.byref(G)) == 0 and G.value == 16
    assert mcs._lib.mc_set_pa_group(ctx, 16, 65) == mcs.MC_E_RANGE
    assert mcs._lib.mc_set_pa_group(ctx, 16, -1) == mcs.MC_E_RANGE
    # L = 128: 2 L * 2 words * 4 B = 2 KB per replica -> 24 fit in 48 KB, 25 do not
    assert mcs._lib.mc_set_pa_group(ctx, 128, 24) == 0
    assert mcs._lib.mc_set_pa_group(ctx, 128, 25) == mcs.MC_E_RANGE
    # L = 512: 32 KB per replica -> only G = 1
    assert mcs._lib.mc_set_pa_group(ctx, 512, 2) == mcs.MC_E_RANGE
    assert mcs._lib.mc_set_pa_group(ctx, 12, 1) == mcs.MC_E_SHAPE
    assert mcs._lib.mc_get_pa_group(ctx, 12, ctypes.byref(G)) == mcs.MC_E_SHAPE
    assert mcs._lib.mc_get_pa_group(ctx, 16, None) == mcs.MC_E_INVAL
    assert mcs._lib.mc_set_pa_group(None, 16, 4) == mcs.MC_E_INVAL


def test_pa_tune_argument_errors(ctx):
    Ls = (ctypes.c_int32 * 2)(16, 16)
    beta = (ctypes.c_double * 3)(0.0, 0.1, 0.2)
    a = mcs.PAArgs(2, Ls, 64, 1, 1, 1, 2, beta)
    ptrs = (ctypes.c_void_p * 2)(FAKE, FAKE)
    ws = FAKE
    # the same extent twice
    assert mcs._lib.mc_tune_pa(ctx, ctypes.byref(a), ptrs, ws, 1 << 30, None, None) == mcs.MC_E_INVAL
    Ls[1] = 32
    assert mcs._lib.mc_tune_pa(ctx, ctypes.byref(a), None, ws, 1 << 30, None, None) == mcs.MC_E_INVAL
    # workspace too small
    assert mcs._lib.mc_tune_pa(ctx, ctypes.byref(a), ptrs, ws, 16, None, None) == mcs.MC_E_WORKSPACE
    # a NULL workspace of a claimed size
    assert mcs._lib.mc_tune_pa(ctx, ctypes.byref(a), ptrs, None, 1 << 30, None, None) == mcs.MC_E_WORKSPACE
    # the workspace fits the first population's timing run but not the second's:
    # rejected before any run
    a1 = mcs.PAArgs(1, Ls, 64, 1, 1, 1, 2, beta)
    need16 = mcs._lib.mc_pa_workspace_bytes(ctypes.byref(a1))
    assert 0 < need16
    assert mcs._lib.mc_tune_pa(ctx, ctypes.byref(a), ptrs, ws, need16, None, None) == mcs.MC_E_WORKSPACE
    assert b"L=32" in mcs._lib.mc_ctx_last_error(ctx)
    # no step to time
    a0 = mcs.PAArgs(2, Ls, 64, 1, 1, 1, 0, beta)
    assert mcs._lib.mc_tune_pa(ctx, ctypes.byref(a0), ptrs, ws, 1 << 30, None, None) == mcs.MC_E_RANGE
    G = ctypes.c_int32()
    assert mcs._lib.mc_get_pa_group(ctx, 16, ctypes.byref(G)) == 0 and G.value == 16  # nothing was set


def _plan(ctx, g):
    H, K, T = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert mcs._lib.mc_get_tile_plan(ctx, ctypes.byref(g), ctypes.byref(H), ctypes.byref(K), ctypes.byref(T)) == 0
    return H.value, K.value, T.value


def test_tile_plans_default_set_and_limits(ctx):
    """Launch shapes of the fused sweeps (host logic only): the built-in plans,
    set/get per geometry, and the limits a plan must meet (threads a multiple
    of 64 up to 1024; 2D: H >= 4, K <= 8, (H + 4K) rows x 2 Lx/64 words of LDS <= 64 KB;
    3D: H >= 2, K <= 4, H <= min(Ly, Lz), the tile with couplings <= 96 KB)."""
    g2 = mcs.make_geom(2, 4096, count=3)
    g3 = mcs.make_geom(3, 256)
    # 2D: 256 bands over the three lattices -> H = 4096 // 85 = 48, two sweeps
    # per launch, (48 + 4) rows x 64 words of tasks -> 1024 threads
    assert _plan(ctx, g2) == (48, 2, 1024)
    # 3D: 16 x 16 tiles (one per CU at 256^3), two sweeps, 768 threads; 256
    # threads with four tiles per CU
    assert _plan(ctx, g3) == (16, 2, 768)
    assert _plan(ctx, mcs.make_geom(3, 256, count=4)) == (16, 2, 256)
    assert _plan(ctx, mcs.make_geom(3, 256, count=2)) == (16, 2, 512)
    set_ = lambda g, H, K, T: mcs._lib.mc_set_tile_plan(ctx, ctypes.byref(g), H, K, T)
    assert set_(g2, 16, 4, 512) == 0
    assert _plan(ctx, g2) == (16, 4, 512)
    assert _plan(ctx, mcs.make_geom(2, 4096, count=2)) != (16, 4, 512)  # keyed by count too
    for H, K, T in [(16, 4, 96), (16, 4, 32), (16, 4, 2048), (16, 9, 512), (0, 2, 512), (16, 0, 512),
                    (3, 1, 512), (200, 8, 1024)]:  # the last: (200 + 32) x 128 words x 4 B = 116 KB of LDS
        assert set_(g2, H, K, T) == mcs.MC_E_RANGE, (H, K, T)
    assert _plan(ctx, g2) == (16, 4, 512)  # a rejected plan leaves the set one
    for H, K, T in [(16, 5, 1024), (257, 1, 1024), (1, 1, 256), (32, 4, 1024)]:  # the last: 48^2 x 8 words x 4 B > 96 KB
        assert set_(g3, H, K, T) == mcs.MC_E_RANGE, (H, K, T)
    assert set_(g3, 8, 4, 256) == 0 and _plan(ctx, g3) == (8, 4, 256)
    bad = mcs.Geom(2, 5, 8, 1, mcs.INT8, 1)
    assert set_(bad, 4, 1, 64) == mcs.MC_E_SHAPE


@pytest.mark.parametrize("dims,L,layout,count", [
    (2, (4096, 4096), mcs.INT8, 3), (3, (256, 256, 256), mcs.INT8, 1), (2, (128, 64), mcs.INT8, 1),
    (2, (16384, 8), mcs.INT8, 1), (3, (64, 4, 8), mcs.INT8, 2), (3, (4096, 4, 4), mcs.INT8, 1),
    (2, (96, 96), mcs.INT8, 1), (2, (4096, 4096), mcs.MSC64, 1), (3, (8192, 8, 8), mcs.INT8, 1),
    (3, (64, 6, 10), mcs.INT8, 1),
    (2, (32768, 4), mcs.INT8, 1), (3, (64, 2, 8), mcs.INT8, 1)])
def test_sweep_workspace_bytes_follow_the_header(dims, L, layout, count):
    """Two packed copies of the lattices (count N / 8 bytes each), in 3D three
    packed coupling planes (N / 8 each), then two arrays of per-tile (E, M)
    sums, each rounded up to 256 bytes (2D: 8 sweeps x count x ceil(Ly / 4)
    bands x 16 bytes; 3D: 4 sweeps x count x ceil(Ly / 2) ceil(Lz / 2) tiles
    x 16 bytes); zero where no fused kernel applies (MSC64, Lx not a multiple
    of 64, 2D Lx > 16384, 3D Lx > 4096 or Ly, Lz < 4)."""
    g = mcs.make_geom(dims, L, layout=layout, count=count)
    N = L[0] * L[1] * (L[2] if dims == 3 else 1)
    fused = layout == mcs.INT8 and L[0] % 64 == 0 and (
        L[0] <= 16384 if dims == 2 else (L[0] <= 4096 and min(L[1], L[2]) >= 4))
    up = lambda b: -(-b // 256) * 256
    slots = up(4 * count * -(-L[1] // 2) * -(-L[2] // 2) * 16) if dims == 3 else up(8 * count * -(-L[1] // 4) * 16)
    head = up(2 * count * N // 8 + 3 * N // 8) if dims == 3 else 2 * count * N // 8  # slots 256-aligned in 3D
    expect = (head + 2 * slots) if fused else 0
    assert mcs._lib.mc_sweep_workspace_bytes(ctypes.byref(g)) == expect


def test_muca_preparation_walker_limit(ctx):
    """Walker preparation sweeps run per group of walkers / 16 lattices, one
    launch dimension of at most 65535 lattices: more walkers are rejected up
    front; the same count without preparation passes this check (and fails
    only at the NULL workspace)."""
    dp = ctypes.cast(FAKE, ctypes.POINTER(ctypes.c_double))
    ip = ctypes.cast(FAKE, ctypes.POINTER(ctypes.c_int64))
    st = mcs.MucaStats()

    def run(walkers, prep):
        a = mcs.MucaArgs(8, walkers, 2, 10, 10, 0, 0.8, 1, mcs.MUCA_HOT, 0, 0, prep, 0, mcs.PROGRESS_FN(), None)
        return mcs._lib.mc_muca_run(ctx, ctypes.byref(a), None, FAKE, dp, ip, dp, dp, ctypes.byref(st), None, 0, None)

    assert run(16 * 65535 + 1, 1) == mcs.MC_E_RANGE
    assert b"walkers" in mcs._lib.mc_ctx_last_error(ctx)
    assert run(16 * 65535 + 1, 0) == mcs.MC_E_WORKSPACE
    assert run(16 * 65535, 1) == mcs.MC_E_WORKSPACE


def test_import_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libmcspin.so must refuse to import: there
    is no fallback path."""
    import shutil
    import subprocess
    import sys

    pkg = tmp_path / "paper_1709_04394_amd"
    pkg.mkdir()
    for name in ("__init__.py", "learned_muca.py"):
        shutil.copy(os.path.join(ROOT, "paper_1709_04394_amd", name), pkg / name)
    code = "import paper_1709_04394_amd"
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, PYTHONPATH=str(tmp_path)))
    assert r.returncode != 0 and "ImportError" in r.stderr and "libmcspin.so is not built" in r.stderr, r.stderr


def test_dcb_argument_checks():
    """mc_sweep_dcb validates before any device work (no GPU needed)."""
    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    try:
        fake = ctypes.c_void_p(1)

        def call(g, tile=128, hits=2, rule=0, nsw=3, wsb=None, sweep0=0):
            a = mcs.SweepArgs(rule, 0.4, 1, 0, sweep0, nsw)
            wsb = mcs._lib.mc_dcb_workspace_bytes(ctypes.byref(g)) if wsb is None else wsb
            return mcs._lib.mc_sweep_dcb(h, ctypes.byref(g), fake, ctypes.byref(a), tile, hits, None, fake, wsb, None)

        g = mcs.make_geom(2, 512, count=2)
        # the packed lattices (256-byte aligned) and two arrays of an (E, M)
        # slot per tile of the smallest tile side, 64
        assert mcs._lib.mc_dcb_workspace_bytes(ctypes.byref(g)) == 2 * 512 * 512 // 8 + 2 * 2 * (512 // 64) ** 2 * 16
        assert mcs._lib.mc_dcb_workspace_bytes(ctypes.byref(mcs.make_geom(2, (512, 256)))) == 0
        assert mcs._lib.mc_dcb_workspace_bytes(ctypes.byref(mcs.make_geom(3, 64))) == 0
        assert call(g, rule=mcs.HEATBATH) == mcs.MC_E_LAYOUT
        assert call(mcs.make_geom(3, 64)) == mcs.MC_E_LAYOUT
        assert call(mcs.make_geom(2, 512, layout=mcs.MSC64)) == mcs.MC_E_LAYOUT
        assert call(mcs.make_geom(2, (512, 256))) == mcs.MC_E_SHAPE
        assert call(mcs.make_geom(2, 96)) == mcs.MC_E_SHAPE
        assert call(g, tile=96) == mcs.MC_E_SHAPE
        assert call(mcs.make_geom(2, 384), tile=128) == mcs.MC_E_SHAPE  # 3 tiles per side: odd
        assert call(g, hits=0) == mcs.MC_E_RANGE and call(g, hits=1001) == mcs.MC_E_RANGE
        assert call(g, hits=1000, sweep0=(1 << 55) // 1000) == mcs.MC_E_RANGE
        assert call(g, wsb=2 * 512 * 512 // 8 - 1) == mcs.MC_E_WORKSPACE
        assert call(g, nsw=0) == 0  # nothing to do: no device work
    finally:
        mcs._lib.mc_ctx_destroy(h)


def test_sg_msc64_argument_checks():
    """mc_couplings_msc64 and mc_sweep_sg_msc64 validate before any device
    work (no GPU needed)."""
    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    try:
        fake = ctypes.c_void_p(1)
        g = mcs.make_geom(3, 32, layout=mcs.MSC64)
        a = mcs.SweepArgs(0, 1.0, 1, 0, 0, 2)
        assert mcs._lib.mc_sweep_sg_msc64(h, ctypes.byref(mcs.make_geom(3, 32)), fake, fake, ctypes.byref(a), None,
                                          None) == mcs.MC_E_LAYOUT
        assert mcs._lib.mc_sweep_sg_msc64(h, ctypes.byref(g), fake, None, ctypes.byref(a), None, None) == mcs.MC_E_INVAL
        small = mcs.make_geom(2, (8, 4), layout=mcs.MSC64)  # 16 sites of a colour: not a multiple of 64
        assert mcs._lib.mc_sweep_sg_msc64(h, ctypes.byref(small), fake, fake, ctypes.byref(a), None,
                                          None) == mcs.MC_E_SHAPE
        assert mcs._lib.mc_couplings_msc64(h, ctypes.byref(mcs.make_geom(3, 32)), fake, 1, 0, None) == mcs.MC_E_LAYOUT
        assert mcs._lib.mc_couplings_msc64(h, ctypes.byref(g), None, 1, 0, None) == mcs.MC_E_INVAL
        assert mcs._lib.mc_couplings_msc64(h, ctypes.byref(g), fake, 1, 0xFFFFFFC1, None) == mcs.MC_E_RANGE
    finally:
        mcs._lib.mc_ctx_destroy(h)


def test_wang_landau_argument_checks():
    """mc_win_drive, mc_wl_sweeps and mc_wl_run validate before any device
    work (no GPU needed)."""
    import numpy as np

    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    try:
        fake = ctypes.c_void_p(1)
        lo = np.array([0, 14], dtype=np.int32)
        hi = np.array([20, 32], dtype=np.int32)
        a, keep = mcs.Context._wl_args(8, lo, hi, 64, 1, lnf_final=1e-4)
        n = mcs._lib.mc_wl_workspace_bytes(ctypes.byref(a))
        assert n > 0

        def drive(L=8, lo=lo, hi=hi, M=64, max_pass=10, ws=fake, nb=n):
            return mcs._lib.mc_win_drive(h, L, lo.size, lo.ctypes.data, hi.ctypes.data, M, 1, max_pass, fake, fake,
                                         ws, nb, None)

        assert drive(L=10) == mcs.MC_E_SHAPE
        assert drive(M=32) == mcs.MC_E_RANGE              # not a multiple of 64
        assert drive(lo=np.array([0, 20], dtype=np.int32), hi=np.array([20, 20], dtype=np.int32)) == mcs.MC_E_RANGE
        assert drive(hi=np.array([20, 33], dtype=np.int32)) == mcs.MC_E_RANGE   # above E = 0
        assert drive(max_pass=0) == mcs.MC_E_RANGE
        assert drive(ws=None) == mcs.MC_E_WORKSPACE
        assert drive(nb=n - 1) == mcs.MC_E_WORKSPACE
        big_lo = np.array([0], dtype=np.int32)
        big_hi = np.array([200], dtype=np.int32)
        assert drive(L=32, lo=big_lo, hi=big_hi) == mcs.MC_E_RANGE   # wider than 192 levels

        inc = np.array([1 << 32, 1 << 31], dtype=np.int64)
        act = np.array([1, 1], dtype=np.uint8)

        def sweeps(inc=inc, flat=0.8, nsw=2):
            return mcs._lib.mc_wl_sweeps(h, 8, 2, lo.ctypes.data, hi.ctypes.data, 64, inc.ctypes.data,
                                         act.ctypes.data, flat, 1, 0, nsw, fake, fake, fake, fake, fake, fake, n,
                                         None)

        assert sweeps(inc=np.array([(1 << 32) + 1, 0], dtype=np.int64)) == mcs.MC_E_RANGE
        assert sweeps(flat=0.0) == mcs.MC_E_RANGE
        assert sweeps(nsw=-1) == mcs.MC_E_RANGE

        st = (mcs.WlWindowStats * 2)()
        pieces = np.zeros((2, 21))
        lng = np.zeros(33)
        dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

        def run(a):
            return mcs._lib.mc_wl_run(h, ctypes.byref(a), fake, fake, dp(pieces), dp(lng), st, fake, n, None)

        for kw in (dict(lnf_final=2.0), dict(lnf_final=1e-12), dict(flat=1.5), dict(check_sweeps=0)):
            b, keep2 = mcs.Context._wl_args(8, lo, hi, 64, 1, **dict(dict(lnf_final=1e-4), **kw))
            assert run(b) == mcs.MC_E_RANGE, kw
        # windows that leave a gap, or do not cover 0..N/2
        for l2, h2 in (([0, 21], [20, 32]), ([2, 14], [20, 32]), ([0, 14], [20, 30]), ([0, 1], [1, 32])):
            b, keep2 = mcs.Context._wl_args(8, l2, h2, 64, 1, lnf_final=1e-4)
            assert run(b) == mcs.MC_E_RANGE, (l2, h2)
    finally:
        mcs._lib.mc_ctx_destroy(h)


def test_windowed_multicanonical_argument_checks():
    import numpy as np

    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    try:
        fake = ctypes.c_void_p(1)
        lo = np.array([0, 14], dtype=np.int32)
        hi = np.array([20, 32], dtype=np.int32)
        i32p = ctypes.POINTER(ctypes.c_int32)

        def args(**kw):
            d = dict(eq=2, rec=10, it=5, flat=0.8, mp=10, lo=lo, hi=hi, M=64)
            d.update(kw)
            return mcs.MucaWinArgs(8, d["lo"].size, d["lo"].ctypes.data_as(i32p), d["hi"].ctypes.data_as(i32p), d["M"],
                                   d["eq"], d["rec"], d["it"], d["flat"], d["mp"], 1, mcs.WL_PROGRESS_FN(), None)

        a = args()
        n = mcs._lib.mc_muca_windows_workspace_bytes(ctypes.byref(a))
        assert n > 0
        st = (mcs.MucaWinStats * 2)()
        pieces = np.zeros((2, 21))
        lng = np.zeros(33)
        dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        run = lambda b, ws=fake, nb=n: mcs._lib.mc_muca_windows_run(h, ctypes.byref(b), fake, fake, dp(pieces),
                                                                     dp(lng), st, ws, nb, None)
        for kw in (dict(rec=0), dict(eq=-1), dict(it=-1), dict(flat=0.0), dict(mp=0), dict(M=96)):
            assert run(args(**kw)) == mcs.MC_E_RANGE, kw
        assert run(args(), ws=None) == mcs.MC_E_WORKSPACE
        assert run(args(lo=np.array([0, 22], dtype=np.int32))) == mcs.MC_E_RANGE   # no overlap
    finally:
        mcs._lib.mc_ctx_destroy(h)
