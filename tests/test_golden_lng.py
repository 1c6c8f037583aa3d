"""The stored exact ln g(E) files (tests/golden/lng_L*.txt, written by
tests/golden/make_exact_lng.py from oracle.exact) against facts that do not
come from that code path:

* L = 16: equal to a fresh exact computation, level by level;
* every L: ln g(-2N) = ln 2 (the two ground states), level 1 empty (no state
  has E = -2N + 4), ln g(-2N + 8) = ln 2N (one flipped spin), ln g(-2N + 12)
  = ln 4N (two flipped neighbours: N sites times 2 bond directions, times
  2 ground states);
* the window holds half of all 2^N states plus half of the E = 0 states:
  sum_{k <= N/2} g = (2^N + g(0)) / 2, checked in logarithms;
* ln g(0) / N approaches ln 2 from below as L grows.
"""
import math
import os

import numpy as np
import pytest

from oracle import exact

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(L):
    return np.loadtxt(os.path.join(HERE, "lng_L%d.txt" % L))


def test_L16_matches_fresh_computation():
    g = exact.exact_g(16)
    ref = np.array([exact.big_log(v) if v else -np.inf for v in g[:16 * 16 // 2 + 1]])
    got = _load(16)
    assert np.array_equal(np.isinf(got), np.isinf(ref))
    fin = np.isfinite(ref)
    assert np.max(np.abs(got[fin] - ref[fin])) <= 1e-12 * np.max(np.abs(ref[fin]))


@pytest.mark.parametrize("L", [16, 24, 32, 48, 64, 96, 128])
def test_closed_form_levels_and_window_sum(L):
    N = L * L
    lng = _load(L)
    assert lng.shape == (N // 2 + 1,)
    assert lng[0] == pytest.approx(math.log(2.0), abs=1e-14)
    assert np.isneginf(lng[1])
    assert lng[2] == pytest.approx(math.log(2.0 * N), rel=1e-14)
    assert lng[3] == pytest.approx(math.log(4.0 * N), rel=1e-14)
    fin = lng[np.isfinite(lng)]
    m = fin.max()
    log_window = m + math.log(np.sum(np.exp(fin - m)))
    log_expect = N * math.log(2.0) - math.log(2.0) + math.log1p(math.exp(lng[-1] - N * math.log(2.0)))
    assert log_window == pytest.approx(log_expect, abs=1e-9)


def test_entropy_density_at_zero_energy_grows_to_ln2():
    s = [_load(L)[-1] / (L * L) for L in (16, 24, 32, 48, 64, 96, 128)]
    assert all(a < b for a, b in zip(s, s[1:]))
    assert math.log(2.0) - s[-1] < 1e-3


@pytest.mark.parametrize("L,want", [(24, 0.687841305184), (48, 0.691519512433), (64, 0.692161353360)])
def test_entropy_density_at_zero_energy_independent_values(L, want):
    # ln g(0) / N as computed independently (arbitrary-precision evaluation of
    # the same exact count, 12 significant digits)
    assert abs(_load(L)[-1] / (L * L) - want) < 2e-12
