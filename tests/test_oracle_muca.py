"""Pins of the oracle's multicanonical walkers (Sec. "Multicanonical
simulations", Eq. muca, Eq. weight_modification, count-again rule).

* With the exact weights W = 1/g(E) (from the exact density of states) the
  energy histogram in the window [-2N, 0] is flat within statistics.
* With W = exp(-beta E) the walkers sample the canonical P_beta(E) restricted
  to the window.
* Walkers never leave the window; the histogram counts one entry per attempted
  move; the start state lies in the window.
* The plain recursion converges at small L and its ln g agrees with the exact
  density of states.
* Acceptance table: ceil(min(1, W(E')/W(E)) 2^32).
* Stratified walker starts: the integer disorder level equals its rounded
  closed form, and the starting energies follow -2N (1 - c/128)^2.
* Walker preparation: the group temperatures are the weights' slope -d lnW/dE
  (beta0 for canonical weights, -2aE at the group's level for ln W = a E^2,
  0 for flat or rising weights); walkers prepared at canonical weights
  reproduce Kaufman's exact energy at L = 16, and their recorded energies equal
  their measured ones.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact


def _exact_window_lng(L):
    g = exact.exact_g(L)
    K = oracle.muca_levels(L)
    return np.array([exact.big_log(v) if v > 0 else -np.inf for v in g[:K]])


def test_table_closed_form():
    L = 6
    K = oracle.muca_levels(L)
    lnW = -np.linspace(0, 7.5, K) ** 1.3
    T = oracle.muca_table(L, lnW)
    for k in range(K):
        for d, dk in enumerate((-2, -1, 1, 2)):
            k2 = k + dk
            if 0 <= k2 < K:
                p = min(1.0, math.exp(lnW[k2] - lnW[k]))
                assert T[k, d] - 1 < p * 2 ** 32 <= T[k, d]
            else:
                assert T[k, d] == 0


def test_start_in_window_and_counting():
    L, W = 8, 64
    N = L * L
    spins, E = oracle.muca_start(L, W, 3)
    assert np.all(E <= 0)
    for w in range(W):
        assert oracle.measure(2, L, spins[w * N:(w + 1) * N])[0] == E[w]
    H = oracle.muca_sweeps(L, spins, E, np.zeros(oracle.muca_levels(L)), 3, 0, 5, True)
    assert H.sum() == W * N * 5
    assert np.all(E <= 0)
    for w in range(0, W, 7):
        assert oracle.measure(2, L, spins[w * N:(w + 1) * N])[0] == E[w]


def test_exact_weights_give_flat_histogram():
    L, W = 8, 256
    lng = _exact_window_lng(L)
    lnW = np.where(np.isfinite(lng), -lng, 0.0)
    spins, E = oracle.muca_start(L, W, 11)
    oracle.muca_sweeps(L, spins, E, lnW, 11, 0, 50, False)
    H = oracle.muca_sweeps(L, spins, E, lnW, 11, 50, 400, True)
    reach = oracle.muca_flat_levels(L)
    h = H[reach].astype(np.float64)
    # mean count per level and a generous correlated-sampling spread
    assert h.min() / h.max() > 0.85, h.min() / h.max()
    assert abs(h.mean() - H.sum() / reach.sum()) < 1e-9


def test_canonical_weights_reproduce_boltzmann():
    L, W, beta = 8, 64, 0.3
    N = L * L
    K = oracle.muca_levels(L)
    lnW = np.array([-beta * (4 * k - 2 * N) for k in range(K)])
    lng = _exact_window_lng(L)
    logp = np.where(np.isfinite(lng), lng + lnW, -np.inf)
    p = np.exp(logp - logp.max())
    p /= p.sum()
    # 8 independent groups of walkers (own seeds) give the spread of the estimate
    est = []
    for grp in range(8):
        spins, E = oracle.muca_start(L, W, 100 + grp)
        oracle.muca_sweeps(L, spins, E, lnW, 100 + grp, 0, 50, False)
        H = oracle.muca_sweeps(L, spins, E, lnW, 100 + grp, 50, 200, True)
        est.append(H / H.sum())
    est = np.array(est)
    mean, sig = est.mean(axis=0), est.std(axis=0, ddof=1) / np.sqrt(len(est))
    big = p > 0.005
    assert np.all(np.abs(mean[big] - p[big]) < 5 * sig[big] + 1e-3), np.max(np.abs(mean[big] - p[big]) / sig[big])


def test_plain_recursion_converges_to_exact_lng():
    # the histogram of one iteration must be big enough for its own noise to
    # pass the 0.8 flatness test: 1024 walkers x 40 recorded sweeps at L = 8
    L, W = 8, 1024
    res = oracle.muca_run(L, W, 19 + L, eq_sweeps=2, rec_sweeps=40, max_iter=80, prod_sweeps=400)
    assert res["converged"]
    lng = _exact_window_lng(L)
    reach = oracle.muca_flat_levels(L)
    est = res["lng"][reach]
    ex = lng[reach]
    # fix the additive constant by matching log-sum-exp over the window
    c = np.logaddexp.reduce(ex) - np.logaddexp.reduce(est)
    err = np.max(np.abs(est + c - ex))
    assert err < 0.03, err


@pytest.mark.parametrize("W", [1, 7, 100, 4096])
def test_stratified_level_is_rounded_closed_form(W):
    # integer definition against 128 (1 - sqrt(1 - (w + 1/2)/W)) rounded
    got = [oracle.muca_strat_level(w, W) for w in range(W)]
    ref = [math.floor(128.0 * (1.0 - math.sqrt(1.0 - (w + 0.5) / W)) + 0.5) for w in range(W)]
    assert got == ref
    assert all(a <= b for a, b in zip(got, got[1:]))


def test_stratified_start_spreads_energies():
    # walker w flips each ground-state spin with probability c_w / 256, so its
    # energy is -2N (1 - c_w/128)^2 on average (independent flips, nearest
    # neighbours both flipped or not with probability p^2 + (1-p)^2)
    L, W = 32, 64
    N = L * L
    spins, E = oracle.muca_start(L, W, 9, oracle.MUCA_STRATIFIED)
    assert np.all(E <= 0)
    c = np.array([oracle.muca_strat_level(w, W) for w in range(W)])
    p = c / 256.0
    expect = -2.0 * N * (1.0 - 2.0 * p) ** 2
    sigma = np.sqrt(2.0 * N * 4.0 * (1.0 - (1.0 - 2.0 * p) ** 4) + 1.0)  # per-bond variance bound
    z = (E - expect) / sigma
    assert np.all(np.abs(z) < 6.0)
    assert c[0] == 1 and oracle.muca_strat_level(0, 4096) == 0  # 4096 walkers: walker 0 is a ground state
    # start 0 equals the hot start of each walker's replica id
    hs, hE = oracle.muca_start(L, 5, 9, oracle.MUCA_HOT)
    for w in range(5):
        s = oracle.init(2, L, oracle.HOT, 9, w).reshape(-1)
        e, m = oracle.measure(2, L, s)
        if e > 0:
            s = s.reshape(L, L).copy()
            s[(np.add.outer(np.arange(L), np.arange(L)) % 2) == 1] *= -1
            s = s.reshape(-1)
        assert np.array_equal(hs[w * N:(w + 1) * N], s)


def _levels_E(L):
    N = L * L
    return np.array([4.0 * k - 2.0 * N for k in range(oracle.muca_levels(L))])


def _target_levels(L, G):
    # round-half-up of (g + 1/2) K / G, clamped to 2 .. K - 1, in exact integers
    K = oracle.muca_levels(L) - 1
    out = []
    for g in range(G):
        num, den = (2 * g + 1) * K, 2 * G
        k = (2 * num + den) // (2 * den)
        out.append(min(max(k, 2), K - 1))
    return out


@pytest.mark.parametrize("L,walkers", [(8, 100), (16, 4096), (12, 5)])
def test_prep_betas_of_canonical_weights(L, walkers):
    # ln W = -beta0 E: every group's slope is beta0
    beta0 = 0.37
    lnW = -beta0 * _levels_E(L)
    b = oracle.muca_prep_betas(L, walkers, lnW)
    assert len(b) == min(oracle.MUCA_PREP_GROUPS, walkers)
    assert np.allclose(b, beta0, rtol=0, atol=1e-12)


def test_prep_betas_of_quadratic_weights():
    # ln W = a E^2: the central difference is exact, -d lnW/dE = -2 a E at the
    # group's level (E <= 0 in the window, so positive)
    L, a = 16, 3e-4
    E = _levels_E(L)
    b = oracle.muca_prep_betas(L, 4096, a * E * E)
    want = [-2.0 * a * E[k] for k in _target_levels(L, 16)]
    assert np.allclose(b, want, rtol=1e-12, atol=1e-12)


def test_prep_betas_flat_and_rising_weights_are_zero():
    L = 8
    assert oracle.muca_prep_betas(L, 64, np.zeros(oracle.muca_levels(L))) == [0.0] * 16
    # weights rising with E (negative slope temperature) are clamped to 0
    assert oracle.muca_prep_betas(L, 64, 0.5 * _levels_E(L)) == [0.0] * 16


def test_prepare_gives_canonical_walkers():
    # canonical weights at beta0 = 0.3: prepared walkers sample P_beta0, so the
    # mean energy per site approaches Kaufman's exact u(beta0) at L = 16, and
    # each recorded energy equals the walker's measured energy
    L, W, beta0 = 16, 256, 0.3
    N = L * L
    spins, E = oracle.muca_start(L, W, 91)
    lnW = -beta0 * _levels_E(L)
    oracle.muca_prepare(L, spins, E, 91, lnW, 120)
    for w in range(0, W, 17):
        em = oracle.measure(2, L, spins[w * N:(w + 1) * N])
        assert E[w] == em[0]
    assert np.all(E <= 0)
    u, _ = exact.kaufman_u_cv(L, beta0)
    assert abs(E.mean() / N - u) < 0.04, (E.mean() / N, u)


def test_settle_folds_walkers_into_the_window():
    """Every bond joins the two sub-lattices, so flipping the odd one maps E to
    -E: a walker above the window is folded into it (the antiferromagnet,
    E = +2N, becomes the ground state, E = -2N), a walker inside is left
    alone, and the stored energies are those of the returned lattices."""
    L, W = 6, 6
    N = L * L
    x, y = np.meshgrid(np.arange(L), np.arange(L))
    af = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8).reshape(-1)
    rows = [np.ones(N, dtype=np.int8), af, -af] + [oracle.init(2, L, oracle.HOT, 5, r) for r in range(3)]
    spins = np.concatenate(rows).astype(np.int8)
    before = spins.reshape(W, N).copy()
    E = np.zeros(W, dtype=np.int64)
    assert oracle.lib().orc_muca_settle(L, W, oracle._p(spins), oracle._p(E)) == 0
    odd = ((x + y) % 2 == 1).reshape(-1)
    for w in range(W):
        e0 = oracle.measure(2, L, before[w])[0]
        s = spins.reshape(W, N)[w]
        assert E[w] == oracle.measure(2, L, s)[0] == -abs(e0)
        want = before[w].copy()
        if e0 > 0:
            want[odd] = -want[odd]
        assert np.array_equal(s, want)
    assert E[1] == E[2] == -2 * N and np.all(spins.reshape(W, N)[1] == 1) and np.all(spins.reshape(W, N)[2] == -1)


def test_sweeps_resume_from_a_checkpoint():
    """The state of a run is (spins, E, sweep number): n1 + n2 sweeps equal n1
    sweeps, then n2 more from sweep n1, with the histograms adding up."""
    L, W, seed = 8, 20, 41
    K = oracle.muca_levels(L)
    lnW = -0.3 * np.sqrt(np.arange(K, dtype=np.float64))[::-1]
    s1, E1 = oracle.muca_start(L, W, seed, oracle.MUCA_STRATIFIED)
    s2, E2 = s1.copy(), E1.copy()
    H = oracle.muca_sweeps(L, s1, E1, lnW, seed, (1 << 32) - 3, 7, True)
    Ha = oracle.muca_sweeps(L, s2, E2, lnW, seed, (1 << 32) - 3, 3, True)
    Hb = oracle.muca_sweeps(L, s2, E2, lnW, seed, (1 << 32), 4, True)
    assert np.array_equal(s1, s2) and np.array_equal(E1, E2) and np.array_equal(H, Ha + Hb)
