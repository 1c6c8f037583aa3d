"""Pins of the acceptance tables (Eq. metropolis-canonical, Eq. heatbath).

An entry is ceil(p * 2^32), so that r32 < T is the same event as r < p with
r = r32 / 2^32 uniform on the 2^32-point grid of [0, 1).
"""
import math

import numpy as np

import oracle
from oracle import exact


def test_beta_zero():
    assert np.all(oracle.metropolis_table(0.0) == 2 ** 32)
    for z in (4, 6):
        assert np.all(oracle.heatbath_table(0.0, z) == 2 ** 31)


def test_metropolis_closed_form():
    for beta in (0.1, 0.2216546, 0.4, exact.BETA_C, 0.5, 1.0):
        T = oracle.metropolis_table(beta)
        assert T[0] == 2 ** 32
        for k in range(1, 4):
            p = math.exp(-beta * 4 * k)
            assert T[k] - 1 < p * 2 ** 32 <= T[k]
        assert np.all(np.diff(T.astype(np.int64)) < 0)


def test_heatbath_symmetry_and_closed_form():
    for beta in (0.1, 0.2216546, 0.25, 1.0):
        for z in (4, 6):
            T = oracle.heatbath_table(beta, z).astype(np.int64)
            assert T[z] == 2 ** 31  # h = 0: probability exactly 1/2
            for h in range(-z, z + 1):
                p = 1.0 / (1.0 + math.exp(-2.0 * beta * h))
                assert T[h + z] - 1 < p * 2 ** 32 <= T[h + z]
                # P(+|h) + P(+|-h) = 1 up to the two ceilings
                assert 2 ** 32 <= T[h + z] + T[z - h] <= 2 ** 32 + 1
            assert np.all(np.diff(T) >= 0)


def test_large_beta_saturates():
    T = oracle.heatbath_table(40.0, 6)
    assert T[-1] == 2 ** 32 and T[0] == 1
    Tm = oracle.metropolis_table(40.0)
    assert Tm[1] == 1 and Tm[3] == 1
