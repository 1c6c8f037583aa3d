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
"""
import math

import numpy as np

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
