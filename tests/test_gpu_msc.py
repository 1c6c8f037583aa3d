"""GPU parity of the 64-lane multi-spin-coded half-sweep kernel (one lane per
site, 64 replicas per word, random planes transposed across the wave, fused
per-replica E and M) against the CPU oracle: lane b of word lattice l must
equal the int8 oracle run of replica replica0 + 64 l + b, spins and per-sweep
(E, M) alike.  Covers 2D and 3D, Metropolis and heat-bath, +-J couplings,
several word lattices, sweep numbers above 2^32, and the 4096^2 workload's
first sweeps on sampled lanes.
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


def _lane(words, b):
    return np.where((words >> np.uint64(b)) & np.uint64(1), -1, 1).astype(np.int8)


def _run(ctx, dims, shape, rule, beta, seed, nsw, lanes, count=1, r0=0, Jseed=None, sweep0=3, start=mcs.HOT):
    g = mcs.make_geom(dims, shape, layout=mcs.MSC64, count=count)
    w = mcs.lattice_tensor(g)
    ctx.init(g, w, start, seed, r0)
    J = None if Jseed is None else oracle.couplings(dims, shape, Jseed)
    Jd = None if J is None else torch.from_numpy(J).cuda()
    EM = torch.empty((nsw, count * 64, 2), dtype=torch.int64, device="cuda")
    ctx.sweep(g, w, beta, seed, nsw, sweep0=sweep0, replica0=r0, rule=rule, J=Jd, EM=EM)
    torch.cuda.synchronize()
    wh = w.cpu().numpy().view(np.uint64).reshape(count, -1)
    emh = EM.cpu().numpy()
    for l in range(count):
        for b in lanes:
            r = r0 + 64 * l + b
            s = oracle.init(dims, shape, start, seed, r)
            ref = oracle.sweep(dims, shape, s, beta, seed, r, sweep0, nsw, rule=rule, J=J)
            assert np.array_equal(_lane(wh[l], b), s), ("spins", l, b)
            assert np.array_equal(emh[:, 64 * l + b, :], ref), ("E, M", l, b)


ALL = list(range(64))


@pytest.mark.parametrize("dims,shape,rule,beta,Jseed", [
    (2, (128, 6), mcs.METROPOLIS, 0.44068679350977147, None),
    (2, (128, 4), mcs.HEATBATH, 0.3, None),
    (2, (256, 10), mcs.METROPOLIS, 0.0, None),
    (2, (128, 8), mcs.HEATBATH, 0.9, 5),
    (3, (128, 4, 6), mcs.HEATBATH, 0.2216546, None),
    (3, (128, 6, 4), mcs.METROPOLIS, 1.0, 13),
    (3, (128, 4, 4), mcs.METROPOLIS, 0.25, None),
    (3, (256, 4, 4), mcs.HEATBATH, 3.0, 7),
])
def test_all_lanes_equal_int8_replicas(ctx, dims, shape, rule, beta, Jseed):
    _run(ctx, dims, shape, rule, beta, 7, 5, ALL, r0=64, Jseed=Jseed, sweep0=(1 << 32) - 2)


def test_several_word_lattices_cold(ctx):
    _run(ctx, 2, (128, 12), mcs.METROPOLIS, 0.5, 3, 6, [0, 5, 63], count=3, r0=1, start=mcs.COLD)


def test_workload_prefix_4096(ctx):
    # the 4096^2 multi-spin workload at beta_c: lanes 0, 1, 31, 63, first sweeps
    _run(ctx, 2, (4096, 4096), mcs.METROPOLIS, 0.44068679350977147, 7, 2, [0, 1, 31, 63], sweep0=0)


def test_workload_prefix_256_cubed(ctx):
    _run(ctx, 3, (256, 256, 256), mcs.HEATBATH, 0.2216546, 11, 1, [0, 63], sweep0=0)
