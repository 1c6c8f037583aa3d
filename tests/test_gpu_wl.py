"""GPU Wang-Landau sampling in energy windows (mc_win_drive, mc_wl_sweeps,
mc_wl_run) against the oracle, bit for bit: the walkers driven into their
windows (spins, E); sweeps from given estimates with several ln f and an
inactive window (spins, E, estimates, counts, flatness flags), at L = 8, 16,
32 and 64, the widest window the kernel takes included; whole runs (stages,
sweeps, every window's piece and the matched ln g), converged and stopped
early; and the run at the bench's shape (L = 64, 32 windows) on sampled
walkers of its first sweeps."""
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


CASES = [
    (8, [0, 14], [20, 32]),
    (16, [0, 40, 90], [60, 110, 128]),
    (32, [0, 160, 330], [180, 340, 512]),
]


@pytest.mark.parametrize("L,lo,hi", CASES)
def test_drive_equals_oracle(ctx, L, lo, hi):
    M = 64
    s, E = ctx.win_drive(L, lo, hi, M, 23)
    so, Eo = oracle.win_drive(L, lo, hi, M, 23)
    assert np.array_equal(s.cpu().numpy(), so)
    assert np.array_equal(E.cpu().numpy(), Eo)


def _sweeps_case(ctx, L, lo, hi, M, nsw, inc, active, seed=31, sweep0=(1 << 32) - 2, gmax=3 << 32):
    lo_a, hi_a = np.array(lo), np.array(hi)
    wmax = int((hi_a - lo_a).max()) + 1
    W = len(lo) * M
    s, E = ctx.win_drive(L, lo, hi, M, seed)
    so, Eo = s.cpu().numpy(), E.cpu().numpy()
    rng = np.random.default_rng(L)
    G0 = rng.integers(0, gmax, size=(W, wmax)).astype(np.int64)
    H0 = rng.integers(0, 50, size=(W, wmax)).astype(np.uint32)
    G = torch.from_numpy(G0.copy()).cuda()
    H = torch.from_numpy(H0.view(np.int32).copy()).cuda()
    flags = torch.full((W,), -1, dtype=torch.int32, device="cuda")
    ctx.wl_sweeps(L, lo, hi, M, inc, active, seed, sweep0, nsw, s, E, G, H, flags)
    torch.cuda.synchronize()
    Go, Ho = G0.copy(), H0.copy()
    oracle.wl_sweeps(L, lo, hi, M, inc, active, seed, sweep0, nsw, so, Eo, Go, Ho)
    assert np.array_equal(s.cpu().numpy(), so)
    assert np.array_equal(E.cpu().numpy(), Eo)
    assert np.array_equal(G.cpu().numpy(), Go)
    assert np.array_equal(H.cpu().numpy().view(np.uint32), Ho)
    fl = flags.cpu().numpy()
    for w in range(W):
        i = w // M
        if active[i]:
            assert fl[w] == int(oracle.wl_flat(Ho[w], lo[i], hi[i], 0.8)), w
        else:
            assert fl[w] == -1


@pytest.mark.parametrize("L,lo,hi", CASES)
def test_sweeps_equal_oracle(ctx, L, lo, hi):
    n = len(lo)
    inc = [(1 << 32) >> (3 * i) for i in range(n)]
    active = [1] * n
    active[-1] = 0 if n > 2 else 1
    _sweeps_case(ctx, L, lo, hi, 64, 3, inc, active)


def test_sweeps_widest_window_at_L64(ctx):
    # 192 levels: the largest estimate block the kernel keeps in LDS
    _sweeps_case(ctx, 64, [0, 180], [191, 371], 64, 2, [1 << 20, 0], [1, 1], gmax=1 << 36)


def test_fixed_weights_sweeps(ctx):
    # ln f = 0: multicanonical sweeps inside the windows
    _sweeps_case(ctx, 16, [0, 40], [60, 128], 128, 4, [0, 0], [1, 1])


@pytest.mark.parametrize("L,lo,hi,lnf,check,max_sweeps", [
    (8, [0, 14], [20, 32], 1e-3, 1, 1 << 30),
    (16, [0, 40, 90], [60, 110, 128], 0.05, 2, 1 << 30),
    (16, [0, 60], [80, 128], 1e-4, 3, 40),   # stops early: not converged
])
def test_run_equals_oracle(ctx, L, lo, hi, lnf, check, max_sweeps):
    M = 64
    r = ctx.wl_run(L, lo, hi, M, 41, lnf, check_sweeps=check, max_sweeps=max_sweeps)
    o = oracle.wl_run(L, lo, hi, M, 41, lnf, check=check, max_sweeps=max_sweeps)
    assert r["stages"] == o["stages"]
    assert r["sweeps"] == o["sweeps"]
    assert r["converged"] == o["converged"]
    for a, b in zip(r["pieces"], o["pieces"]):
        assert np.array_equal(a, b)
    assert np.array_equal(r["lng"], o["lng"])
    assert np.array_equal(r["E"].cpu().numpy(), o["E"])
    assert np.array_equal(r["spins"].cpu().numpy(), o["spins"])


def test_bench_shape_sampled_walkers(ctx):
    # L = 64, 32 windows of 2 x 64 walkers (the bench's run), first sweeps:
    # sampled walkers rebuilt by the oracle from the same driven states
    L, M = 64, 128
    lo, hi = _bench_windows(L, 32)
    W = len(lo) * M
    s, E = ctx.win_drive(L, lo, hi, M, 5)
    so, Eo = s.cpu().numpy(), E.cpu().numpy()
    wmax = max(h - l for l, h in zip(lo, hi)) + 1
    G = torch.zeros((W, wmax), dtype=torch.int64, device="cuda")
    H = torch.zeros((W, wmax), dtype=torch.int32, device="cuda")
    flags = torch.zeros(W, dtype=torch.int32, device="cuda")
    inc = [1 << 32] * len(lo)
    ctx.wl_sweeps(L, lo, hi, M, inc, [1] * len(lo), 5, 0, 3, s, E, G, H, flags)
    torch.cuda.synchronize()
    Gd, Hd, sd, Ed = G.cpu().numpy(), H.cpu().numpy().view(np.uint32), s.cpu().numpy(), E.cpu().numpy()
    for i in (0, 13, 31):
        # the oracle on window i alone: walker ids of that window are i M + m
        lo1, hi1 = lo[:i + 1], hi[:i + 1]
        act = [0] * i + [1]
        sub = slice(0, (i + 1) * M)
        so2, Eo2 = so[sub].copy(), Eo[sub].copy()
        Go = np.zeros(((i + 1) * M, max(h - l for l, h in zip(lo1, hi1)) + 1), dtype=np.int64)
        Ho = np.zeros(Go.shape, dtype=np.uint32)
        oracle.wl_sweeps(L, lo1, hi1, M, inc[:i + 1], act, 5, 0, 3, so2, Eo2, Go, Ho)
        for m in (0, 37, M - 1):
            w = i * M + m
            n = hi[i] - lo[i] + 1
            assert np.array_equal(sd[w], so2[w]) and Ed[w] == Eo2[w]
            assert np.array_equal(Gd[w, :n], Go[w, :n]) and np.array_equal(Hd[w, :n], Ho[w, :n])


def _bench_windows(L, nwin):
    K = L * L // 2
    width = -(-(K + 1 + (nwin - 1) * 8) // nwin)  # equal widths with 8-level overlaps
    lo = [min(i * (width - 8), K - width + 1) for i in range(nwin)]
    hi = [l + width - 1 for l in lo]
    hi[-1] = K
    return lo, hi


@pytest.mark.parametrize("L,lo,hi,rec,max_iter", [
    (8, [0, 14], [20, 32], 200, 100),
    (16, [0, 40, 90], [60, 110, 128], 300, 100),
    (16, [0, 40, 90], [60, 110, 128], 50, 6),   # stops early: not flat
])
def test_windowed_multicanonical_equals_oracle(ctx, L, lo, hi, rec, max_iter):
    M = 64
    r = ctx.muca_windows_run(L, lo, hi, M, 7, rec, max_iter)
    o = oracle.muca_windows_run(L, lo, hi, M, 7, rec, max_iter)
    assert r["iterations"] == o["iterations"]
    assert r["converged"] == o["converged"]
    for a, b in zip(r["pieces"], o["pieces"]):
        assert np.array_equal(a, b)
    assert np.array_equal(r["lng"], o["lng"])
    assert np.array_equal(r["E"].cpu().numpy(), o["E"])
