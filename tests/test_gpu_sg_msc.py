"""GPU spin glasses multi-spin coded across 64 disorder realisations, one
random number per site shared by the coded copies (mc_couplings_msc64,
mc_sweep_sg_msc64), against the int8 oracle: bit b of word lattice l is the
realisation with couplings oracle.couplings(.., realisation0 + 64 l + b),
started from the hot start of replica replica0 + 64 l + b and swept with the
draws of replica id replica0 + l; spins and per-sweep (E, M) of every
realisation, 2D and 3D, Metropolis and heat-bath, several word lattices, and
the 32^3 workload over the full 2000 sweeps on sampled realisations."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
mcs = pytest.importorskip("paper_1709_04394_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mcs.Context(0)


def _lane(words, b):
    return np.where((words >> np.uint64(b)) & np.uint64(1), -1, 1).astype(np.int8)


def _jlane(words, b):
    return np.where((words >> np.uint64(b)) & np.uint64(1), -1, 1).astype(np.int8)


@pytest.mark.parametrize("dims,shape,count", [(3, (8, 8, 8), 2), (2, (16, 8), 1), (3, (32, 32, 32), 1)])
def test_couplings_msc64_equal_realisations(ctx, dims, shape, count):
    g = mcs.make_geom(dims, shape, layout=mcs.MSC64, count=count)
    J = torch.empty((count, dims * g.N), dtype=torch.int64, device="cuda")
    ctx.couplings_msc64(g, J, 13, 5)
    Jh = J.cpu().numpy().view(np.uint64)
    for l in range(count):
        for b in (0, 1, 31, 63):
            ref = oracle.couplings(dims, shape, 13, 5 + 64 * l + b)
            assert np.array_equal(_jlane(Jh[l], b), ref), (l, b)


def _run(ctx, dims, shape, count, rule, beta, seed, nsw, lanes, r0=3, z0=0, sweep0=0):
    g = mcs.make_geom(dims, shape, layout=mcs.MSC64, count=count)
    w = mcs.lattice_tensor(g)
    ctx.init(g, w, mcs.HOT, seed, r0)
    J = torch.empty((count, dims * g.N), dtype=torch.int64, device="cuda")
    ctx.couplings_msc64(g, J, seed + 100, z0)
    EM = torch.empty((nsw, count * 64, 2), dtype=torch.int64, device="cuda")
    ctx.sweep_sg_msc64(g, w, J, beta, seed, nsw, sweep0=sweep0, replica0=r0, rule=rule, EM=EM)
    torch.cuda.synchronize()
    wh = w.cpu().numpy().view(np.uint64).reshape(count, -1)
    emh = EM.cpu().numpy()
    orule = oracle.HEATBATH if rule == mcs.HEATBATH else oracle.METROPOLIS
    for l in range(count):
        for b in lanes:
            s = oracle.init(dims, shape, oracle.HOT, seed, r0 + 64 * l + b)
            Jb = oracle.couplings(dims, shape, seed + 100, z0 + 64 * l + b)
            ref = oracle.sweep(dims, shape, s, beta, seed, r0 + l, sweep0, nsw, rule=orule, J=Jb)
            assert np.array_equal(emh[:, 64 * l + b, :], ref), ("E, M", l, b)
            assert np.array_equal(_lane(wh[l], b), s), ("spins", l, b)


ALL = list(range(64))


@pytest.mark.parametrize("dims,shape,count,rule,beta", [
    (3, (8, 8, 8), 2, mcs.METROPOLIS, 1.0),
    (3, (8, 4, 4), 1, mcs.HEATBATH, 0.7),
    (2, (16, 8), 1, mcs.METROPOLIS, 0.8),
    (2, (32, 12), 2, mcs.HEATBATH, 2.0),
    (3, (8, 8, 8), 1, mcs.METROPOLIS, 0.0),
])
def test_every_realisation_equals_its_int8_run(ctx, dims, shape, count, rule, beta):
    _run(ctx, dims, shape, count, rule, beta, 21, 6, ALL, sweep0=(1 << 32) - 3)


def test_spin_glass_workload_32_cubed(ctx):
    # 3D +-J at L = 32, Metropolis at beta = 1 (the spin-glass workload),
    # the workload's full 2000 sweeps on sampled realisations
    _run(ctx, 3, (32, 32, 32), 1, mcs.METROPOLIS, 1.0, 13, 2000, [0, 17, 63], r0=0, z0=0)
