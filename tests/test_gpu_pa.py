"""GPU population annealing against the CPU oracle, through the C ABI.

Bit-exact: FP64 C_total of every step (fixed-order prefix sum), ln Q and ln Z
(same host arithmetic on the same C_total), every energy histogram, and the
final populations, for populations of several L in one call (4 .. 128,
replica counts that are not multiples of 64, several scan levels), and for a
run split into two calls (step_first > 1).  At the full configuration
(4 populations x 16384 replicas, L = 16, 32, 64, 128, theta = 10, beta_i =
i / 200) the first steps are compared for every population and the whole
200-step anneal for L = 16; ln Z(beta = 1) is checked against Kaufman.
"""
import math

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


def _compare(Ls, R, res, pops_gpu, opops, nsteps):
    for p, L in enumerate(Ls):
        N = L * L
        op = opops[p]
        assert np.array_equal(res["Ctot"][p], np.array(op.Ctot[-nsteps:])), ("Ctot", L)
        assert np.array_equal(res["lnQ"][p], np.array(op.lnQ[-nsteps:])), ("lnQ", L)
        assert np.array_equal(res["lnZ"][p], np.array(op.lnZ[-(nsteps + 1):])), ("lnZ", L)
        for s in range(nsteps + 1):
            assert np.array_equal(res["hist"][p][s], op.hist[len(op.hist) - nsteps - 1 + s]), ("hist", L, s)
        torch.cuda.synchronize()
        g = pops_gpu[p][:R * N].cpu().numpy()
        assert np.array_equal(g, op.spins), ("spins", L)


@pytest.mark.parametrize("Ls,R,theta,nsteps,dbeta", [([4, 16], 100, 3, 5, 0.04), ([8, 32, 64], 130, 2, 4, 0.03),
                                                     ([128], 70, 2, 3, 0.005), ([16], 4096 + 7, 2, 3, 0.04),
                                                     ([32, 16], 1, 1, 3, 0.02)])
def test_pa_matches_oracle(ctx, Ls, R, theta, nsteps, dbeta):
    seed = 17
    beta = np.array([i * dbeta for i in range(nsteps + 1)])
    pops = ctx.pa_population_tensors(Ls, R)
    res = ctx.pa_anneal(Ls, R, theta, seed, beta, pops)
    opops = [oracle.PAPopulation(L, R, p, seed).advance(beta, theta, nsteps) for p, L in enumerate(Ls)]
    _compare(Ls, R, res, pops, opops, nsteps)


def test_pa_split_calls(ctx):
    Ls, R, theta, seed = [16, 64], 200, 2, 5
    beta = np.array([i * 0.02 for i in range(6)])
    pops = ctx.pa_population_tensors(Ls, R)
    r1 = ctx.pa_anneal(Ls, R, theta, seed, beta, pops, step_first=1, nsteps=2)
    r2 = ctx.pa_anneal(Ls, R, theta, seed, beta, pops, step_first=3, nsteps=3, lnZ0=r1["lnZ"][:, -1])
    opops = [oracle.PAPopulation(L, R, p, seed).advance(beta, theta, 5) for p, L in enumerate(Ls)]
    _compare(Ls, R, r2, pops, opops, 3)


@pytest.fixture(scope="module")
def full_run(ctx):
    # 4 populations x 16384 replicas, L = 16, 32, 64, 128, beta_i = i/200, theta = 10
    Ls, R, theta, seed = [16, 32, 64, 128], 16384, 10, 17
    beta = oracle.pa_schedule(200, 1.0)
    pops = ctx.pa_population_tensors(Ls, R)
    res = ctx.pa_anneal(Ls, R, theta, seed, beta, pops)
    return Ls, R, theta, seed, beta, res, pops


def test_pa_full_config_first_steps(ctx):
    Ls, R, theta, seed = [16, 32, 64, 128], 16384, 10, 17
    beta = oracle.pa_schedule(200, 1.0)
    pops = ctx.pa_population_tensors(Ls, R)
    res = ctx.pa_anneal(Ls, R, theta, seed, beta, pops, nsteps=1)
    opops = [oracle.PAPopulation(L, R, p, seed).advance(beta, theta, 1) for p, L in enumerate(Ls)]
    _compare(Ls, R, res, pops, opops, 1)


def test_pa_full_config_L16_whole_anneal(full_run):
    Ls, R, theta, seed, beta, res, pops = full_run
    op = oracle.PAPopulation(16, R, 0, seed).advance(beta, theta, 200)
    sub = dict(Ctot=res["Ctot"][:1], lnQ=res["lnQ"][:1], lnZ=res["lnZ"][:1], hist=res["hist"][:1])
    _compare([16], R, sub, pops[:1], [op], 200)


def test_pa_full_config_free_energy_vs_kaufman(full_run):
    Ls, R, theta, seed, beta, res, pops = full_run
    for p, L in enumerate(Ls):
        N = L * L
        for i in (100, 200):
            est = res["lnZ"][p][i] / N
            ex = float(exact.kaufman_lnZ(L, beta[i])) / N
            # population-size bias and noise of R = 16384 at these L: well below 1e-3 per spin
            assert abs(est - ex) < 1e-3, (L, i, est, ex)
        # every histogram counts the whole population
        assert np.all(res["hist"][p].sum(axis=1) == R)


@pytest.mark.parametrize("groups", [{4: 64, 16: 1, 64: 16, 128: 3}, {4: 7, 16: 64, 64: 1, 128: 24}])
def test_pa_replicas_per_workgroup_do_not_change_results(ctx, groups):
    """Any admissible replicas-per-workgroup setting gives the oracle's results
    bit for bit (ragged last workgroup: R = 130 is a multiple of none of them)."""
    Ls, R, theta, nsteps, seed = [4, 16, 64, 128], 130, 2, 3, 23
    beta = np.array([i * 0.005 for i in range(nsteps + 1)])
    try:
        for L, G in groups.items():
            ctx.set_pa_group(L, G)
            assert ctx.get_pa_group(L) == G
        pops = ctx.pa_population_tensors(Ls, R)
        res = ctx.pa_anneal(Ls, R, theta, seed, beta, pops)
    finally:
        for L in groups:
            ctx.set_pa_group(L, 0)
    opops = [oracle.PAPopulation(L, R, p, seed).advance(beta, theta, nsteps) for p, L in enumerate(Ls)]
    _compare(Ls, R, res, pops, opops, nsteps)


def test_pa_tuner_picks_admissible_groups_and_keeps_results(ctx):
    Ls, R, theta, nsteps, seed = [16, 128], 300, 1, 3, 29
    beta = np.array([i * 0.005 for i in range(nsteps + 1)])
    pops = ctx.pa_population_tensors(Ls, R)
    try:
        G = ctx.tune_pa(Ls, R, theta, seed, beta, pops)
        assert G[0] in (4, 8, 16, 32, 64) and G[1] in (1, 2, 4), G
        assert [ctx.get_pa_group(L) for L in Ls] == G
        res = ctx.pa_anneal(Ls, R, theta, seed, beta, pops)
    finally:
        for L in Ls:
            ctx.set_pa_group(L, 0)
    opops = [oracle.PAPopulation(L, R, p, seed).advance(beta, theta, nsteps) for p, L in enumerate(Ls)]
    _compare(Ls, R, res, pops, opops, nsteps)


def test_pa_repeated_identical_calls_reuse_the_graph(ctx):
    """The context keeps the instantiated graph of the last anneal and launches
    it again for a call with the same inputs: three identical calls, with the
    workspace overwritten and other work on the device between them, all give
    the oracle's results; a call with other inputs in between rebuilds it."""
    Ls, R, theta, nsteps, seed = [16, 64], 200, 2, 4, 31
    beta = np.array([i * 0.02 for i in range(nsteps + 1)])
    pops = ctx.pa_population_tensors(Ls, R)
    ws = torch.empty(ctx.pa_workspace_bytes(Ls, R, theta, beta), dtype=torch.uint8, device="cuda")
    opops = [oracle.PAPopulation(L, R, p, seed).advance(beta, theta, nsteps) for p, L in enumerate(Ls)]
    for rep in range(3):
        res = ctx.pa_anneal(Ls, R, theta, seed, beta, pops, ws=ws)
        _compare(Ls, R, res, pops, opops, nsteps)
        ws.fill_(0xA5)
        for t in pops:
            t.fill_(3)
        torch.cuda.synchronize()
        if rep == 1:
            other = ctx.pa_anneal(Ls, R, theta, seed + 1, beta, pops, ws=ws)
            assert not np.array_equal(other["Ctot"], res["Ctot"])
