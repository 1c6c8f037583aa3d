"""GPU parity of the sweep path against the CPU oracle, through the C ABI.

Bit-exact: initial lattices, couplings, spins after every call, and the
per-sweep (E, M) records.  Shapes span several tiles and ragged tails, square
and rectangular, 2D and 3D, both update rules, the +-J model, int8 and the
64-lane multi-spin-coded layout (lane b must equal the int8 run of replica
replica0 + 64 l + b), with and without the fused-sweep workspace.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact

pytestmark = pytest.mark.gpu

mcs = pytest.importorskip("paper_1709_04394_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mcs.Context(0)


def _shape(dims, L):
    return (L,) * dims if isinstance(L, int) else tuple(L)


def _to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _unpack_msc(words, lane):
    w = words.view(np.uint64) if words.dtype != np.uint64 else words
    return np.where((w >> np.uint64(lane)) & np.uint64(1), -1, 1).astype(np.int8)


@pytest.mark.parametrize("dims,L,layout", [(2, 64, 0), (2, (36, 20), 0), (3, (8, 6, 4), 0), (2, 4, 0),
                                           (2, (12, 8), 1), (3, 4, 1)])
def test_init_parity(ctx, dims, L, layout):
    shape = _shape(dims, L)
    count = 3
    g = mcs.make_geom(dims, shape, layout=layout, count=count)
    t = mcs.lattice_tensor(g)
    ctx.init(g, t, mcs.HOT, 77, replica0=5)
    h = _to_host(t)
    for l in range(count):
        if layout == 0:
            assert np.array_equal(h[l], oracle.init(dims, shape, oracle.HOT, 77, 5 + l))
        else:
            for b in (0, 1, 31, 63):
                assert np.array_equal(_unpack_msc(h[l], b), oracle.init(dims, shape, oracle.HOT, 77, 5 + 64 * l + b))
    ctx.init(g, t, mcs.COLD, 77)
    h = _to_host(t)
    assert np.all(h == (1 if layout == 0 else 0))


@pytest.mark.parametrize("dims,L", [(2, (20, 12)), (3, 8)])
def test_couplings_parity(ctx, dims, L):
    shape = _shape(dims, L)
    g = mcs.make_geom(dims, shape)
    J = torch.empty(dims * g.N, dtype=torch.int8, device="cuda")
    ctx.couplings(g, J, 13)
    assert np.array_equal(_to_host(J), oracle.couplings(dims, shape, 13))


def _run_both(ctx, dims, shape, rule, beta, seed, nsweeps, sweep0=0, count=1, replica0=0, J=None, start=1,
               use_ws=False, calls=1):
    g = mcs.make_geom(dims, shape, count=count)
    spins = mcs.lattice_tensor(g)
    ctx.init(g, spins, start, seed, replica0)
    Jd = None if J is None else torch.from_numpy(J).cuda()
    ws = None
    if use_ws:
        nb = ctx.sweep_workspace_bytes(g)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    EMs = []
    per = nsweeps // calls
    for k in range(calls):
        EM = torch.empty((per, count, 2), dtype=torch.int64, device="cuda")
        ctx.sweep(g, spins, beta, seed, per, sweep0=sweep0 + k * per, replica0=replica0, rule=rule, J=Jd, EM=EM,
                  ws=ws)
        EMs.append(_to_host(EM))
    gpu = _to_host(spins)
    gEM = np.concatenate(EMs, axis=0)
    for l in range(count):
        s = oracle.init(dims, shape, start, seed, replica0 + l)
        EM = oracle.sweep(dims, shape, s, beta, seed, replica0 + l, sweep0, per * calls, rule=rule, J=J)
        assert np.array_equal(gpu[l], s), ("spins differ", l)
        assert np.array_equal(gEM[:, l, :], EM), ("EM differ", l)


def test_config_tiny_64x64_betac_1000_sweeps(ctx):
    # 2D Ising 64x64, hot start seed 1, replica 0, Metropolis at beta_c, 1000
    # sweeps, (E, M) after every sweep
    _run_both(ctx, 2, (64, 64), mcs.METROPOLIS, exact.BETA_C, 1, 1000)


@pytest.mark.parametrize("shape,beta,rule", [((4, 4), 0.3, 0), ((36, 20), 0.44, 0), ((68, 132), 0.5, 0),
                                             ((260, 12), 0.2, 1), ((16, 16), 0.0, 0), ((16, 16), 0.0, 1),
                                             ((8, 8), 40.0, 0)])
def test_2d_shapes_rules(ctx, shape, beta, rule):
    _run_both(ctx, 2, shape, rule, beta, 3, 30, sweep0=(1 << 33) + 5, count=2, replica0=11)


@pytest.mark.parametrize("shape,rule,beta", [((8, 8, 8), 1, 0.2216546), ((12, 6, 4), 1, 0.25), ((6, 8, 10), 0, 0.3)])
def test_3d(ctx, shape, rule, beta):
    _run_both(ctx, 3, shape, rule, beta, 11, 20, count=2)
    _run_both(ctx, 3, shape, rule, beta, 11, 6, start=0)


@pytest.mark.parametrize("dims,shape,rule,J", [(2, (516, 310), 0, False), (3, (34, 38, 124), 1, True)])
def test_generic_kernels_large_odd_shapes(ctx, dims, shape, rule, J):
    # too large for one workgroup's LDS and not a multiple of 64 wide: the
    # generic half-sweep kernels
    Jh = oracle.couplings(dims, shape, 3) if J else None
    _run_both(ctx, dims, shape, rule, 0.3, 17, 4, J=Jh)


def test_config_edwards_anderson_32(ctx):
    # 3D +-J spin glass at L = 32, couplings and spins from seed 13, Metropolis
    # at beta = 1, the workload's whole 2000 sweeps (the bit-packed whole-
    # lattice kernel: one workgroup)
    J = oracle.couplings(3, 32, 13)
    _run_both(ctx, 3, (32, 32, 32), mcs.METROPOLIS, 1.0, 13, 2000, J=J)


def test_edwards_anderson(ctx):
    J = oracle.couplings(3, 8, 13)
    _run_both(ctx, 3, (8, 8, 8), mcs.METROPOLIS, 1.0, 13, 25, J=J)
    J2 = oracle.couplings(2, (20, 12), 14)
    _run_both(ctx, 2, (20, 12), mcs.HEATBATH, 0.7, 14, 15, J=J2)


def test_split_calls_and_workspace(ctx):
    # three calls of 10 sweeps == one call of 30 (global sweep numbering), with
    # and without the fused-sweep workspace
    _run_both(ctx, 2, (64, 64), 0, 0.44, 5, 30, calls=3)
    _run_both(ctx, 2, (64, 64), 0, 0.44, 5, 30, use_ws=True)
    _run_both(ctx, 2, (256, 64), 0, 0.4, 6, 21, use_ws=True, count=2)


@pytest.mark.parametrize("dims,shape,rule,beta,Jseed", [(2, (16, 12), 0, 0.44, None), (3, (6, 4, 8), 1, 0.22, None),
                                                        (3, (4, 4, 4), 0, 1.0, 13)])
def test_msc64_lanes_equal_int8_replicas(ctx, dims, shape, rule, beta, Jseed):
    count, seed, r0, nsw = 2, 7, 64, 8
    g = mcs.make_geom(dims, shape, layout=mcs.MSC64, count=count)
    w = mcs.lattice_tensor(g)
    ctx.init(g, w, mcs.HOT, seed, r0)
    J = None if Jseed is None else oracle.couplings(dims, shape, Jseed)
    Jd = None if J is None else torch.from_numpy(J).cuda()
    EM = torch.empty((nsw, count * 64, 2), dtype=torch.int64, device="cuda")
    ctx.sweep(g, w, beta, seed, nsw, sweep0=3, replica0=r0, rule=rule, J=Jd, EM=EM)
    wh = _to_host(w)
    emh = _to_host(EM)
    for l in range(count):
        for b in (0, 1, 2, 31, 32, 63):
            r = r0 + 64 * l + b
            s = oracle.init(dims, shape, oracle.HOT, seed, r)
            ref = oracle.sweep(dims, shape, s, beta, seed, r, 3, nsw, rule=rule, J=J)
            assert np.array_equal(_unpack_msc(wh[l], b), s), (l, b)
            assert np.array_equal(emh[:, 64 * l + b, :], ref), (l, b)


def test_measure_parity(ctx):
    for dims, shape, Js in [(2, (20, 36), None), (3, (6, 8, 4), 21)]:
        g = mcs.make_geom(dims, shape, count=3)
        t = mcs.lattice_tensor(g)
        ctx.init(g, t, mcs.HOT, 9)
        J = None if Js is None else oracle.couplings(dims, shape, Js)
        EM = torch.empty((3, 2), dtype=torch.int64, device="cuda")
        ctx.measure(g, t, EM, J=None if J is None else torch.from_numpy(J).cuda())
        emh = _to_host(EM)
        for l in range(3):
            s = oracle.init(dims, shape, oracle.HOT, 9, l)
            assert tuple(emh[l]) == oracle.measure(dims, shape, s, J)
