"""GPU double-checkerboard sweeps with k hits per tile (mc_sweep_dcb: tiles
of one coarse colour per launch, k rounds of each tile's own checkerboard in
LDS, in place on bit-packed lattices) against the oracle's sweep_dcb, bit for
bit: spins and per-sweep (E, M) of several lattices per call, for every tile
size, one to many hits, temperatures from 0 to deep in the ordered phase,
sweep numbers that cross 2^32 after multiplying by the hits, a run split over
calls, and the 4096^2 benchmark lattice's first sweeps."""
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


def _run(ctx, L, T, k, beta, seed, nsw, count=2, replica0=3, sweep0=0, calls=1, start=None):
    start = mcs.HOT if start is None else start
    g = mcs.make_geom(2, L, count=count)
    spins = mcs.lattice_tensor(g)
    ctx.init(g, spins, start, seed, replica0)
    ws = torch.empty(ctx.dcb_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    # one packed copy and two arrays of an (E, M) slot per tile of side 64,
    # each 256-byte aligned
    up = lambda b: (b + 255) // 256 * 256
    assert ws.numel() == up(count * L * L // 8) + 2 * up(count * (L // 64) ** 2 * 16)
    per = nsw // calls
    EMs = []
    for c in range(calls):
        EM = torch.empty((per, count, 2), dtype=torch.int64, device="cuda")
        ctx.sweep_dcb(g, spins, beta, seed, per, T, k, sweep0=sweep0 + c * per, replica0=replica0, EM=EM, ws=ws)
        EMs.append(EM.cpu().numpy())
    torch.cuda.synchronize()
    gs, gem = spins.cpu().numpy(), np.concatenate(EMs, axis=0)
    for l in range(count):
        s = oracle.init(2, L, oracle.HOT if start == mcs.HOT else oracle.COLD, seed, replica0 + l)
        em = oracle.sweep_dcb(L, s, beta, seed, replica0 + l, sweep0, per * calls, T, k)
        assert np.array_equal(gem[:, l, :], em), ("E, M", l)
        assert np.array_equal(gs[l], s), ("spins", l)


@pytest.mark.parametrize("L,T,k", [(128, 64, 1), (128, 64, 3), (256, 128, 2), (256, 64, 10), (512, 128, 5),
                                   (512, 256, 1), (1024, 512, 2)])
def test_dcb_matches_oracle(ctx, L, T, k):
    _run(ctx, L, T, k, 0.4406868, 61, 4, sweep0=(1 << 32) // k - 1)


@pytest.mark.parametrize("beta", [0.0, 0.3, 1.0])
def test_dcb_temperatures_and_cold_start(ctx, beta):
    _run(ctx, 256, 64, 3, beta, 62, 3, count=1)
    _run(ctx, 128, 64, 2, beta, 62, 3, count=3, start=mcs.COLD)


def test_dcb_split_calls(ctx):
    _run(ctx, 256, 128, 4, 0.44, 63, 6, calls=3)
    _run(ctx, 256, 64, 2, 0.44, 64, 3, calls=3)  # one sweep per call


def test_dcb_many_tiles_per_lattice(ctx):
    # 1024 tiles of 64 per lattice: the slots of a sweep outnumber the threads
    # of the workgroup that adds them up
    _run(ctx, 2048, 64, 1, 0.44068679350977147, 65, 3, count=1)


def test_dcb_benchmark_lattice_prefix(ctx):
    # 4096^2 at beta_c with tiles of 128 and 10 hits: the benchmark rows' shape
    _run(ctx, 4096, 128, 10, 0.44068679350977147, 7, 2, count=1, replica0=0)
