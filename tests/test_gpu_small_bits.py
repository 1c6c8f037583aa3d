"""GPU parity of the bit-packed small-lattice kernel (rows of 32 sites held as
two 16-bit parity words in one workgroup's LDS, all sweeps in one launch)
against the CPU oracle, through the C ABI: spins and per-sweep (E, M) bit for
bit, 2D and 3D, J = 1 and +-J, Metropolis and heat-bath, temperatures from
infinite (every threshold 2^32) to ones where thresholds round to 0 or 2^32,
several lattices per launch, more rows than threads, sweep numbers across
2^32, cold and hot starts, and the 32^3 spin-glass workload.
"""
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


def _run(ctx, dims, shape, rule, beta, seed, nsweeps, sweep0=0, count=1, replica0=0, Jseed=None, start=mcs.HOT):
    g = mcs.make_geom(dims, shape, count=count)
    spins = mcs.lattice_tensor(g)
    ctx.init(g, spins, start, seed, replica0)
    J = None if Jseed is None else oracle.couplings(dims, shape, Jseed)
    Jd = None if J is None else torch.from_numpy(J).cuda()
    EM = torch.empty((nsweeps, count, 2), dtype=torch.int64, device="cuda")
    ctx.sweep(g, spins, beta, seed, nsweeps, sweep0=sweep0, replica0=replica0, rule=rule, J=Jd, EM=EM)
    torch.cuda.synchronize()
    gs, gem = spins.cpu().numpy().reshape(count, -1), EM.cpu().numpy()
    for l in range(count):
        s = oracle.init(dims, shape, start, seed, replica0 + l)
        em = oracle.sweep(dims, shape, s, beta, seed, replica0 + l, sweep0, nsweeps, rule=rule, J=J)
        assert np.array_equal(gs[l], s), ("spins", l)
        assert np.array_equal(gem[:, l, :], em), ("E, M", l)


@pytest.mark.parametrize("rule", [mcs.METROPOLIS, mcs.HEATBATH])
@pytest.mark.parametrize("shape,beta", [((32, 4), 0.3), ((32, 10), 0.44068679350977147), ((32, 36), 0.0),
                                        ((32, 8), 4.0), ((32, 6), 40.0)])
def test_2d(ctx, rule, shape, beta):
    _run(ctx, 2, shape, rule, beta, 3, 12, sweep0=(1 << 32) - 5, count=3, replica0=2)


@pytest.mark.parametrize("rule", [mcs.METROPOLIS, mcs.HEATBATH])
@pytest.mark.parametrize("shape,beta", [((32, 4, 6), 0.2216546), ((32, 8, 4), 0.0), ((32, 6, 8), 3.0),
                                        ((32, 64, 20), 0.25)])
def test_3d(ctx, rule, shape, beta):
    _run(ctx, 3, shape, rule, beta, 11, 7, sweep0=(1 << 33) + 1, count=2, replica0=5)


@pytest.mark.parametrize("rule", [mcs.METROPOLIS, mcs.HEATBATH])
@pytest.mark.parametrize("dims,shape,beta", [(2, (32, 8), 1.0), (2, (32, 12), 0.0), (3, (32, 6, 4), 1.0),
                                             (3, (32, 4, 10), 5.0), (3, (32, 40, 30), 0.6)])
def test_couplings(ctx, rule, dims, shape, beta):
    _run(ctx, dims, shape, rule, beta, 13, 6, count=2, Jseed=17)


@pytest.mark.parametrize("start", [mcs.COLD, mcs.HOT])
def test_starts(ctx, start):
    _run(ctx, 3, (32, 8, 8), mcs.METROPOLIS, 0.5, 9, 10, start=start, Jseed=4)


def test_spin_glass_32_cubed(ctx):
    # +-J couplings from seed 13, hot spins from seed 13, Metropolis at beta = 1
    _run(ctx, 3, (32, 32, 32), mcs.METROPOLIS, 1.0, 13, 300, Jseed=13)
