"""GPU parity of the workloads exactly as the benchmark runs them, at full
size, against the CPU oracle (spins and per-sweep (E, M) element by element):

- the 2D headline call: three 4096^2 lattices at beta 0.40, beta_c, 0.50 in
  one mc_sweep_betas call with the tuned launch shape (bands of 16 rows, 4
  sweeps per launch, 512 threads), 12 sweeps, so that one launch of the call
  reads and writes bit-packed rows (int8 -> packed -> packed -> int8);
- the 3D call: four 256^3 heat-bath lattices (beta 0.2216546 and 0.25, each
  from a cold and a hot start, seed 11) in one call, 6 sweeps (three launches
  of two sweeps);
- 64-replica multi-spin coding at 4096^2 (Metropolis at beta_c) and 256^3
  (heat-bath at beta 0.2216546): every lane's spins and (E, M) against the
  int8 oracle run of that replica;
- the whole 200-step population anneal of the L = 32 population of the
  4 x 16384-replica workload (the L = 16 population is in test_gpu_pa.py).

The oracle's share of the long runs is split over several tests so that each
finishes (and reports) within a minute or so on the host cores.
"""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
mcs = pytest.importorskip("paper_1709_04394_amd")

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mcs.Context(0)


@pytest.mark.parametrize("plan", [(16, 2, 512), (16, 4, 512)])
def test_headline_call_3x4096_betas_tuned_plan(ctx, plan):
    # the benchmark's launch shape (16, 2, 512) and the earlier (16, 4, 512)
    L, betas, seed, nsw, sweep0 = 4096, [0.40, BETA_C, 0.50], 7, 12, 100
    g = mcs.make_geom(2, L, count=3)
    lat = mcs.lattice_tensor(g)
    ctx.init(g, lat, mcs.HOT, seed, 0)
    ws = torch.empty(ctx.sweep_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    ctx.set_tile_plan(g, *plan)
    EM = torch.empty((nsw, 3, 2), dtype=torch.int64, device="cuda")
    ctx.sweep_betas(g, lat, betas, seed, nsw, sweep0=sweep0, replica0=0, EM=EM, ws=ws)
    torch.cuda.synchronize()
    gs, gem = lat.cpu().numpy(), EM.cpu().numpy()
    del lat, ws, EM
    for l, b in enumerate(betas):
        s = oracle.init(2, L, oracle.HOT, seed, l)
        em = oracle.sweep(2, L, s, b, seed, l, sweep0, nsw)
        assert np.array_equal(gem[:, l, :], em), ("E, M", l)
        assert np.array_equal(gs[l], s), ("spins", l)


def test_3d_call_4x256_heatbath_cold_and_hot(ctx):
    L, seed, nsw = 256, 11, 6
    betas = [0.2216546, 0.25, 0.2216546, 0.25]
    starts = [mcs.COLD, mcs.COLD, mcs.HOT, mcs.HOT]
    g4, g2 = mcs.make_geom(3, L, count=4), mcs.make_geom(3, L, count=2)
    lat = mcs.lattice_tensor(g4)
    ctx.init(g2, lat[:2], mcs.COLD, seed, 0)
    ctx.init(g2, lat[2:], mcs.HOT, seed, 2)
    ws = torch.empty(ctx.sweep_workspace_bytes(g4), dtype=torch.uint8, device="cuda")
    assert ctx.get_tile_plan(g4)[1] == 2  # two sweeps per launch: the 6 sweeps are three launches
    EM = torch.empty((nsw, 4, 2), dtype=torch.int64, device="cuda")
    ctx.sweep_betas(g4, lat, betas, seed, nsw, rule=mcs.HEATBATH, EM=EM, ws=ws)
    torch.cuda.synchronize()
    gs, gem = lat.cpu().numpy(), EM.cpu().numpy()
    del lat, ws, EM
    for l in range(4):
        s = oracle.init(3, L, oracle.COLD if starts[l] == mcs.COLD else oracle.HOT, seed, l)
        em = oracle.sweep(3, L, s, betas[l], seed, l, 0, nsw, rule=oracle.HEATBATH)
        assert np.array_equal(gem[:, l, :], em), ("E, M", l)
        assert np.array_equal(gs[l], s), ("spins", l)


def _lane(words, b):
    return np.where((words >> np.uint64(b)) & np.uint64(1), -1, 1).astype(np.int8)


MSC_CASES = {
    "2d": (2, (4096, 4096), mcs.METROPOLIS, BETA_C, 7, 4),
    "3d": (3, (256, 256, 256), mcs.HEATBATH, 0.2216546, 11, 2),
}


@pytest.fixture(scope="module")
def msc_runs(ctx):
    """GPU runs of the two multi-spin-coded workloads (lanes = replicas
    0..63), computed once; the lanes are compared in groups below."""
    out = {}
    for name, (dims, shape, rule, beta, seed, nsw) in MSC_CASES.items():
        g = mcs.make_geom(dims, shape, layout=mcs.MSC64)
        w = mcs.lattice_tensor(g)
        ctx.init(g, w, mcs.HOT, seed, 0)
        EM = torch.empty((nsw, 64, 2), dtype=torch.int64, device="cuda")
        ctx.sweep(g, w, beta, seed, nsw, rule=rule, EM=EM)
        torch.cuda.synchronize()
        out[name] = (w.cpu().numpy().view(np.uint64).reshape(-1), EM.cpu().numpy())
        del w, EM
    return out


@pytest.mark.parametrize("name", list(MSC_CASES))
@pytest.mark.parametrize("lanes", [range(0, 16), range(16, 32), range(32, 48), range(48, 64)])
def test_msc64_workloads_every_lane(msc_runs, name, lanes):
    dims, shape, rule, beta, seed, nsw = MSC_CASES[name]
    words, em = msc_runs[name]
    orule = oracle.HEATBATH if rule == mcs.HEATBATH else oracle.METROPOLIS
    for b in lanes:
        s = oracle.init(dims, shape, oracle.HOT, seed, b)
        ref = oracle.sweep(dims, shape, s, beta, seed, b, 0, nsw, rule=orule)
        assert np.array_equal(em[:, b, :], ref), ("E, M", name, b)
        assert np.array_equal(_lane(words, b), s), ("spins", name, b)


# ------------------------------------------------------------------ annealing
PA_LS, PA_R, PA_THETA, PA_SEED = [16, 32, 64, 128], 16384, 10, 17


@pytest.fixture(scope="module")
def pa_full(ctx):
    """The whole anneal of the four populations in one call (as the benchmark
    runs it), and the oracle's L = 32 population (population index 1), which
    the tests below advance 50 steps at a time."""
    beta = oracle.pa_schedule(200, 1.0)
    pops = ctx.pa_population_tensors(PA_LS, PA_R)
    res = ctx.pa_anneal(PA_LS, PA_R, PA_THETA, PA_SEED, beta, pops)
    torch.cuda.synchronize()
    final32 = pops[1][:PA_R * 32 * 32].cpu().numpy()
    del pops
    op = oracle.PAPopulation(32, PA_R, 1, PA_SEED)
    return dict(beta=beta, res=res, final32=final32, op=op)


@pytest.mark.parametrize("chunk", [0, 1, 2, 3])
def test_pa_full_config_L32_whole_anneal(pa_full, chunk):
    op, res, beta = pa_full["op"], pa_full["res"], pa_full["beta"]
    if op.step < 50 * chunk:  # a chunk run on its own first catches up
        op.advance(beta, PA_THETA, 50 * chunk - op.step)
    if op.step == 50 * chunk:
        op.advance(beta, PA_THETA, 50)
    lo, hi = 50 * chunk, 50 * chunk + 50
    assert np.array_equal(res["Ctot"][1][lo:hi], np.array(op.Ctot[lo:hi])), "C_total"
    assert np.array_equal(res["lnQ"][1][lo:hi], np.array(op.lnQ[lo:hi])), "ln Q"
    assert np.array_equal(res["lnZ"][1][lo:hi + 1], np.array(op.lnZ[lo:hi + 1])), "ln Z"
    for s in range(lo, hi + 1):
        assert np.array_equal(res["hist"][1][s], op.hist[s]), ("histogram", s)
    if chunk == 3:
        assert np.array_equal(pa_full["final32"], op.spins), "final population"
