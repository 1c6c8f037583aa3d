"""Pins of the oracle's parallel tempering (Sec. "Parallel Tempering", Eq. pt).

* Equal inverse temperatures: the exponent is 0, so every proposed exchange
  is accepted and each round swaps exactly the proposed pairs.
* At fixed energies the acceptance frequency of an exchange is
  min(1, exp((beta_i - beta_j)(E_a - E_b))) within binomial errors, and the
  two maps stay inverse permutations.
* A full run on the 4 x 4 torus: in equilibrium the replicas held at
  different temperatures are independent and Boltzmann distributed, so the
  mean energy at each temperature and the acceptance rate of each pair,
  sum_{E, E'} P_i(E) P_{i+1}(E') min(1, exp((beta_i - beta_{i+1})(E - E'))),
  follow from the exact density of states; the run must agree within the
  spread of batch means.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact


def _boltzmann_4x4(beta):
    g = [int(v) for v in exact.exact_g(4)]
    N = 16
    E = np.array([4 * k - 2 * N for k in range(N + 1)], dtype=np.float64)
    w = np.array([float(c) for c in g]) * np.exp(-beta * (E + 2 * N))
    return E, w / w.sum()


def test_equal_temperatures_always_exchange():
    nT = 5
    beta = [0.3] * nT
    E = np.array([-32, 0, 8, -16, 4], dtype=np.int64)
    temp_of, replica_at, acc = list(range(nT)), list(range(nT)), [0] * (nT - 1)
    oracle.pt_exchange(beta, E, temp_of, replica_at, 1, 0, acc)  # pairs (0,1), (2,3)
    assert replica_at == [1, 0, 3, 2, 4] and acc == [1, 0, 1, 0]
    oracle.pt_exchange(beta, E, temp_of, replica_at, 1, 1, acc)  # pairs (1,2), (3,4)
    assert replica_at == [1, 3, 0, 4, 2] and acc == [1, 1, 1, 1]
    assert all(replica_at[temp_of[a]] == a for a in range(nT))


@pytest.mark.parametrize("dE,dbeta", [(8, 0.05), (24, 0.1), (-12, 0.2)])
def test_acceptance_frequency_at_fixed_energies(dE, dbeta):
    beta = [0.4, 0.4 + dbeta]
    E = np.array([dE, 0], dtype=np.int64)  # replica 0 at temperature 0, 1 at 1
    p = min(1.0, math.exp(-dbeta * dE))
    n, hits = 20000, 0
    for rnd in range(0, 2 * n, 2):  # even rounds propose the pair (0, 1)
        temp_of, replica_at, acc = [0, 1], [0, 1], [0]
        oracle.pt_exchange(beta, E, temp_of, replica_at, 7, rnd, acc)
        hits += acc[0]
        assert replica_at == ([1, 0] if acc[0] else [0, 1]) and temp_of == replica_at
    assert abs(hits / n - p) <= 5 * math.sqrt(p * (1 - p) / n) + 1e-12, (hits / n, p)


def test_full_run_on_4x4_against_exact_distributions():
    beta = [0.15, 0.3, 0.45, 0.6]
    rounds, nb = 24000, 24
    r = oracle.pt_run(2, 4, beta, 2024, rounds, 1)
    Eat = r["E_at"][1000:].astype(np.float64)  # first 1000 rounds: equilibration
    batches = np.array_split(np.arange(len(Eat)), nb)
    for i, b in enumerate(beta):
        Ev, P = _boltzmann_4x4(b)
        u = float((Ev * P).sum())
        means = np.array([Eat[idx, i].mean() for idx in batches])
        sig = means.std(ddof=1) / math.sqrt(nb)
        assert abs(means.mean() - u) < 5 * sig + 0.02, (b, means.mean(), u, sig)
    # acceptance rate of each pair against the product of exact distributions
    for i in range(len(beta) - 1):
        Ea, Pa = _boltzmann_4x4(beta[i])
        Eb, Pb = _boltzmann_4x4(beta[i + 1])
        x = (beta[i] - beta[i + 1]) * (Ea[:, None] - Eb[None, :])
        want = float((Pa[:, None] * Pb[None, :] * np.minimum(1.0, np.exp(x))).sum())
        proposals = len([rnd for rnd in range(rounds) if rnd % 2 == i % 2])
        rate = r["accepted"][i] / proposals
        # 0.03 is several times the run's own spread (about 0.005); halving the
        # exponent moves the rates by 0.06 to 0.14, flipping its sign by 0.3+
        assert abs(rate - want) < 0.03, (i, rate, want)
    assert sorted(r["replica_at"]) == list(range(len(beta)))
    assert all(r["replica_at"][r["temp_of"][a]] == a for a in range(len(beta)))


def test_exchange_draw_of_a_set_is_keyed_by_the_set_index():
    # two temperatures, E_a - E_b = 8 at beta 0.3, 0.5: x = -1.6, accepted iff
    # word 0 of Philox(EXCHANGE, 0, set, round) < ceil(exp(-1.6) 2^32)
    T = math.ceil(math.ldexp(math.exp((0.3 - 0.5) * 8.0), 32))
    for pt_set in (0, 1, 7):
        for rnd in range(0, 40, 2):  # even rounds propose pair 0
            t, r, acc = [0, 1], [0, 1], [0]
            oracle.pt_exchange([0.3, 0.5], [8, 0], t, r, 99, rnd, acc, pt_set)
            want = oracle.draw_word(99, oracle.TAG_EXCHANGE, 0, pt_set, rnd) < T
            assert acc[0] == int(want) and (r == [1, 0]) == want


def test_sets_start_from_their_own_replica_ids():
    # set 2 of three-temperature sets: replica r is replica id 6 + r, so before
    # the first exchange (identity maps) temperature r shows that replica's
    # energy after theta sweeps of its own stream
    beta, seed, theta = [0.2, 0.4, 0.6], 5, 2
    b = oracle.pt_run(2, 4, beta, seed, 3, theta, pt_set=2)
    for r in range(3):
        s = oracle.init(2, 4, oracle.HOT, seed, 6 + r)
        em = oracle.sweep(2, 4, s, beta[r], seed, 6 + r, 0, theta)
        assert b["E_at"][0][r] == em[-1, 0]
