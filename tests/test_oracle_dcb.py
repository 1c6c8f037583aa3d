"""Pins of the oracle's double-checkerboard sweep with k hits per tile (Sec.
"Checkerboard scheme": tiles in a coarse checkerboard, each tile updated k
times per load; a different Markov chain from the plain checkerboard).

* Deterministic: at beta = 0 every Metropolis move is accepted, so each site
  flips once per hit and a sweep maps s -> (-1)^k s.
* Exact enumeration of the 4 x 4 torus with 2 x 2 tiles: every elementary
  step (one coarse colour, one fine colour) satisfies detailed balance, the
  composed sweep satisfies global balance (to the 2^-32 quantisation of the
  acceptance probabilities) but not detailed balance; long oracle runs sample
  the Boltzmann energy distribution g(E) e^{-beta E} / Z.
* Kaufman's exact finite-lattice energy at L = 16 (tiles of 4 and 8, several
  hits).
* The stream and order: small cases rebuilt tile by tile (each tile of the
  first coarse colour k rounds of its own checkerboard, then each tile of the
  second), from the pinned Philox draws and tables, equal the oracle.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact


def _batch_sigma(x, nb=40):
    x = np.asarray(x, dtype=np.float64)
    n = (x.size // nb) * nb
    b = x[:n].reshape(nb, -1).mean(axis=1)
    return b.std(ddof=1) / math.sqrt(nb)


@pytest.mark.parametrize("L,T,k", [(8, 2, 1), (8, 4, 2), (16, 4, 3), (16, 8, 4), (12, 2, 5)])
def test_beta0_each_site_flips_once_per_hit(L, T, k):
    s = oracle.init(2, L, oracle.HOT, 3, 1)
    s0 = s.copy()
    EM = oracle.sweep_dcb(L, s, 0.0, 3, 1, 0, 2, T, k)
    assert np.array_equal(s, s0)  # two sweeps: (-1)^(2k)
    oracle.sweep_dcb(L, s, 0.0, 3, 1, 2, 1, T, k)
    assert np.array_equal(s, -s0 if k % 2 else s0)
    E0, M0 = oracle.measure(2, L, s0)
    assert EM[0, 0] == E0 and EM[0, 1] == (M0 if k % 2 == 0 else -M0)


def test_rejects_tilings_that_are_not_a_checkerboard():
    s = oracle.init(2, 12, oracle.HOT, 3)
    for T, k in ((4, 1), (5, 1), (3, 1), (2, 0), (12, 1)):  # 12/4 = 3 and 12/12 = 1 tiles per side are odd
        with pytest.raises(ValueError):
            oracle.sweep_dcb(12, s, 0.3, 3, 0, 0, 1, T, k)


def _step_matrix(spins, beta, sites):
    """Flip probabilities of a simultaneous Metropolis update of the given
    (mutually non-adjacent) sites of the 4 x 4 torus, every state at once."""
    L = 4
    T = oracle.metropolis_table(beta).astype(np.float64) / 2.0 ** 32
    idx = np.arange(L * L)
    x, y = idx % L, idx // L
    nb = np.stack([(x + 1) % L + L * y, (x - 1) % L + L * y, x + L * ((y + 1) % L), x + L * ((y - 1) % L)], 1)
    h = spins[:, nb].sum(axis=2)
    dE = 2 * spins * h
    p = np.where(dE <= 0, 1.0, T[np.clip(dE // 4, 0, 3)])[:, sites]
    n = len(sites)
    sub = np.arange(1 << n)
    bits = ((sub[:, None] >> np.arange(n)) & 1).astype(bool)
    F = (bits.astype(np.int64) << np.asarray(sites)).sum(axis=1)
    P = np.ones((spins.shape[0], sub.size))
    for j in range(n):
        P *= np.where(bits[None, :, j], p[:, j:j + 1], 1.0 - p[:, j:j + 1])
    return P, F


def test_balance_4x4_tiles_2x2():
    L, N, T, k, beta = 4, 16, 2, 2, 0.35
    E, _ = exact.enumerate_states(2, (L, L))
    idx = np.arange(1 << N)
    spins = 1 - 2 * ((idx[:, None] >> np.arange(N)) & 1)
    w = np.exp(-beta * (E - E.min()))
    pi = w / w.sum()
    sx, sy = np.arange(N) % L, np.arange(N) // L
    coarse, fine = (sx // T + sy // T) & 1, (sx + sy) & 1
    dist = pi.copy()
    steps = []
    for P in (0, 1):
        for _h in range(k):
            for c in (0, 1):
                sites = np.flatnonzero((coarse == P) & (fine == c))
                Pm, F = _step_matrix(spins, beta, sites)
                succ = idx[:, None] ^ F[None, :]
                # detailed balance of the elementary step (a flip set is its own reverse)
                fwd = pi[:, None] * Pm
                rev = pi[succ] * Pm[succ, np.arange(F.size)[None, :]]
                rel = np.abs(fwd - rev) / np.maximum(fwd, 1e-300)
                assert np.max(np.where(fwd > 1e-30, rel, 0.0)) < 1e-7
                dist = np.bincount(succ.ravel(), weights=(dist[:, None] * Pm).ravel(), minlength=1 << N)
                steps.append((Pm, succ))
    # global balance of the whole sweep
    assert np.max(np.abs(dist - pi) / pi) < 1e-7

    # ... but not detailed balance: transition probabilities between the ground
    # state and a state it reaches, by propagating a point mass
    def sweep_row(s0):
        v = np.zeros(1 << N)
        v[s0] = 1.0
        for Pm, succ in steps:
            v = np.bincount(succ.ravel(), weights=(v[:, None] * Pm).ravel(), minlength=1 << N)
        return v

    s = 0
    row = sweep_row(s)
    target = int(np.argmax(row * (idx != s)))
    back = sweep_row(target)[s]
    lhs, rhs = pi[s] * row[target], pi[target] * back
    assert abs(lhs - rhs) / lhs > 1e-3


@pytest.mark.parametrize("k", [1, 3])
def test_boltzmann_4x4_tiles_2x2(k):
    beta = 0.3
    s = oracle.init(2, 4, oracle.HOT, 51)
    EM = oracle.sweep_dcb(4, s, beta, 51, 0, 0, 150000, 2, k)
    g = exact.enumerate_torus(2, (4, 4))
    levels = np.array(sorted(g))
    w = np.array([g[e] * math.exp(-beta * (e - levels.min())) for e in levels])
    p = w / w.sum()
    Es = EM[1000:, 0]
    for e, pe in zip(levels, p):
        if pe < 1e-3:
            continue
        ind = (Es == e).astype(np.float64)
        assert abs(ind.mean() - pe) < 5 * _batch_sigma(ind) + 1e-4, (k, e, ind.mean(), pe)


@pytest.mark.parametrize("T,k,beta,nsw", [(4, 10, 0.4, 8000), (8, 3, exact.BETA_C, 20000), (4, 1, 0.5, 20000)])
def test_kaufman_energy_L16(T, k, beta, nsw):
    L, N = 16, 256
    s = oracle.init(2, L, oracle.HOT, 53)
    EM = oracle.sweep_dcb(L, s, beta, 53, 0, 0, nsw, T, k)
    e = EM[500:, 0].astype(np.float64) / N
    u_ex, _ = exact.kaufman_u_cv(L, beta, dps=30)
    assert abs(e.mean() - u_ex) < 5 * _batch_sigma(e), (e.mean(), u_ex)


def _rebuild_by_tiles(L, T, k, s, beta, seed, rep, sweep0, nsweeps):
    """The double checkerboard written tile by tile, as the paper's blocks do
    it: each tile of coarse colour 0 takes its k rounds (even sites, then odd),
    then each tile of coarse colour 1; site i's hit h of sweep t draws r32 of
    same-colour index i >> 1 in plain sweep number t k + h."""
    Tm = oracle.metropolis_table(beta)
    nt = L // T
    out = []
    for t in range(sweep0, sweep0 + nsweeps):
        for P in (0, 1):
            for ty in range(nt):
                for tx in range(nt):
                    if (tx + ty) % 2 != P:
                        continue
                    for h in range(k):
                        for c in (0, 1):
                            for y in range(ty * T, ty * T + T):
                                for x in range(tx * T, tx * T + T):
                                    if (x + y) % 2 != c:
                                        continue
                                    i = x + L * y
                                    hf = (s[(x + 1) % L + L * y] + s[(x - 1) % L + L * y] +
                                          s[x + L * ((y + 1) % L)] + s[x + L * ((y - 1) % L)])
                                    dE = 2 * int(s[i]) * int(hf)
                                    r = oracle.draw32(seed, oracle.TAG_SWEEP, oracle.TAG_SWEEP_LO, i >> 1, rep,
                                                      t * k + h, c)
                                    if dE <= 0 or r < int(Tm[dE // 4]):
                                        s[i] = -s[i]
        out.append(oracle.measure(2, L, s))
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("L,T,k,beta,sweep0", [(8, 2, 2, 0.44, 0), (8, 4, 3, 0.3, 5), (12, 2, 1, 0.6, (1 << 32) - 1)])
def test_stream_and_order_rebuilt_tile_by_tile(L, T, k, beta, sweep0):
    seed, rep = 57, 3
    s1 = oracle.init(2, L, oracle.HOT, seed, rep)
    s2 = s1.copy()
    EM = oracle.sweep_dcb(L, s1, beta, seed, rep, sweep0, 2, T, k)
    ref = _rebuild_by_tiles(L, T, k, s2, beta, seed, rep, sweep0, 2)
    assert np.array_equal(s1, s2)
    assert np.array_equal(EM, ref)
