"""GPU parity of the fused multi-sweep 3D kernel (tiles of rows in y, z with a
redone halo, bit-packed in LDS, per-class thresholds) against the CPU oracle:
Metropolis and heat-bath, ferromagnet and +-J couplings, every admissible
tile plan giving the same bits (ragged tiles, tiles larger than the lattice,
several lattices per launch with their own temperatures, single sweeps, sweep
numbers above 2^32), cold and hot starts, and the 256^3 workload's first
sweeps compared in full.
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


def _run(ctx, shape, rule, beta, seed, nsweeps, plan=None, count=1, replica0=0, J=None, start=mcs.HOT, sweep0=0,
         betas=None, measure=True):
    g = mcs.make_geom(3, shape, count=count)
    spins = mcs.lattice_tensor(g)
    ctx.init(g, spins, start, seed, replica0)
    ws = torch.empty(ctx.sweep_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    assert ws.numel() > 0
    if plan is not None:
        ctx.set_tile_plan(g, *plan)
    Jd = None if J is None else torch.from_numpy(J).cuda()
    EM = torch.empty((nsweeps, count, 2), dtype=torch.int64, device="cuda") if measure else None
    if betas is None:
        ctx.sweep(g, spins, beta, seed, nsweeps, sweep0=sweep0, replica0=replica0, rule=rule, J=Jd, EM=EM, ws=ws)
    else:
        ctx.sweep_betas(g, spins, betas, seed, nsweeps, sweep0=sweep0, replica0=replica0, rule=rule, J=Jd, EM=EM,
                        ws=ws)
    torch.cuda.synchronize()
    gs = spins.cpu().numpy().reshape(count, -1)
    gem = EM.cpu().numpy() if measure else None
    for l in range(count):
        b = beta if betas is None else betas[l]
        s = oracle.init(3, shape, start, seed, replica0 + l)
        em = oracle.sweep(3, shape, s, b, seed, replica0 + l, sweep0, nsweeps, rule=rule, J=J)
        assert np.array_equal(gs[l], s), ("spins", l)
        if measure:
            assert np.array_equal(gem[:, l, :], em), ("E, M", l)


@pytest.mark.parametrize("rule", [mcs.METROPOLIS, mcs.HEATBATH])
@pytest.mark.parametrize("shape,plan", [((64, 8, 8), (4, 1, 64)), ((64, 8, 8), (8, 2, 128)), ((64, 12, 10), (5, 3, 256)),
                                        ((128, 6, 10), (4, 4, 512)), ((64, 16, 16), (16, 1, 1024)),
                                        ((192, 6, 10), (4, 2, 64)), ((64, 20, 12), None),
                                        ((64, 4, 4), (4, 3, 64)), ((64, 64, 64), (4, 1, 64)),
                                        ((64, 6, 10), (2, 1, 64)), ((128, 6, 10), (3, 2, 128))])
@pytest.mark.parametrize("nsweeps", [1, 4, 9])
def test_fused3d_matches_oracle(ctx, rule, shape, plan, nsweeps):
    _run(ctx, shape, rule, 0.2216546, 11, nsweeps, plan=plan, count=2, replica0=3, sweep0=(1 << 32) - 3)


@pytest.mark.parametrize("rule,beta", [(mcs.METROPOLIS, 1.0), (mcs.METROPOLIS, 0.3), (mcs.HEATBATH, 1.0),
                                       (mcs.HEATBATH, 0.0), (mcs.METROPOLIS, 0.0), (mcs.HEATBATH, 4.0)])
def test_fused3d_couplings(ctx, rule, beta):
    shape = (64, 10, 8)
    J = oracle.couplings(3, shape, 13)
    _run(ctx, shape, rule, beta, 13, 6, plan=(4, 2, 128), J=J)


@pytest.mark.parametrize("start", [mcs.COLD, mcs.HOT])
def test_fused3d_starts_and_betas(ctx, start):
    _run(ctx, (64, 8, 12), mcs.HEATBATH, None, 5, 5, plan=(6, 2, 256), count=3, start=start,
         betas=[0.2216546, 0.25, 0.1])


def test_fused3d_workload_prefix(ctx):
    # the 256^3 heat-bath workload near the critical point: first sweeps in full
    _run(ctx, (256, 256, 256), mcs.HEATBATH, 0.2216546, 11, 2, start=mcs.HOT)


def test_tuner_3d(ctx):
    g = mcs.make_geom(3, (64, 16, 16))
    a, b = mcs.lattice_tensor(g), mcs.lattice_tensor(g)
    plan = ctx.tune_sweep(g, a, b, 0.25, sweeps=4, rule=mcs.HEATBATH)
    assert plan[0] >= 1
    _run(ctx, (64, 16, 16), mcs.HEATBATH, 0.25, 3, 5, plan=plan)


@pytest.mark.parametrize("rule", [mcs.METROPOLIS, mcs.HEATBATH])
def test_fused3d_without_measurement(ctx, rule):
    # no EM: the launches store no tile sums and add none up; the spins are
    # those of the measured run
    _run(ctx, (64, 12, 10), rule, 0.2216546, 17, 7, plan=(4, 2, 128), count=2, measure=False)
