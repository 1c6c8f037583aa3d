"""Pins of the oracle's Wang-Landau sampling in energy windows (Sec.
"Wang-Landau update"; windows and the count-again rule of Sec.
"Multicanonical simulations").

* The acceptance threshold ceil(exp(-x 2^-32) 2^32), built from a product of
  tabulated exponentials, is within one unit of the exact value (mpmath, 50
  digits), and is 1 once the probability is below 2^-32.
* Walkers driven into their windows are inside them, their recorded energies
  equal their measured ones, and they differ from each other.
* With fixed exact weights (estimate = ln g_exact, no modification) the visit
  histogram of a window is flat within statistics, the count-again rule at the
  window's edges included: dropping it under-counts the edge levels.
* The whole method converges at L = 8: two overlapping windows, 64 walkers
  each, ln f down to 1e-4, matched ln g within 0.1 of the exact one.
* Matching: pieces of the exact ln g shifted by arbitrary constants are put
  back together exactly.
* The multicanonical recursion in windows (flat start, ln W -= ln H per
  window, count-again, matching) converges to the exact g(E) at L = 8 and 16.
* Stream contract: a tiny case rebuilt site by site from the pinned Philox
  draws and the threshold (typewriter order, draw index, count-again, visit
  and estimate updates after every attempt, the estimate shifted to a
  minimum of 0 at the end of the call).
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import exact


def _exact_levels(L):
    K = L * L // 2
    return exact.exact_lng(L)[:K + 1]


@pytest.mark.parametrize("x", [1, 255, 1 << 20, (1 << 32) - 1, 1 << 32, 3 * (1 << 32) + 123456789,
                               (22 << 32) + (1 << 31), (23 << 32) - 1, 23 << 32, 40 << 32])
def test_threshold_within_one_of_the_exact_exponential(x):
    mpmath.mp.dps = 50
    exact_T = int(mpmath.ceil(mpmath.exp(-mpmath.mpf(x) / 2 ** 32) * 2 ** 32))
    T = oracle.wl_threshold(x)
    assert abs(T - max(1, exact_T)) <= 1, (x, T, exact_T)
    if x >= (23 << 32):
        assert T == 1


def test_threshold_random_differences():
    mpmath.mp.dps = 40
    rng = np.random.default_rng(5)
    xs = rng.integers(1, 24 << 32, size=300, dtype=np.int64)
    off = 0
    for x in xs:
        e = int(mpmath.ceil(mpmath.exp(-mpmath.mpf(int(x)) / 2 ** 32) * 2 ** 32))
        d = oracle.wl_threshold(int(x)) - max(1, e)
        assert abs(d) <= 1
        off += d != 0
    assert off <= 3  # a product of five rounded factors is off by one only near an integer


def test_drive_puts_walkers_inside_their_windows():
    L, M = 8, 5
    lo, hi = [0, 10, 25], [12, 27, 32]
    spins, E = oracle.win_drive(L, lo, hi, M, 3)
    for w in range(len(lo) * M):
        k = (E[w] + 2 * L * L) // 4
        assert lo[w // M] <= k <= hi[w // M]
        assert oracle.measure(2, L, spins[w].copy())[0] == E[w]
    # distinct walkers of one window
    assert len({spins[w].tobytes() for w in range(M, 2 * M)}) == M
    s2, E2 = oracle.win_drive(L, lo, hi, M, 3)
    assert np.array_equal(s2, spins) and np.array_equal(E2, E)


def test_drive_rejects_bad_windows():
    with pytest.raises(ValueError):
        oracle.win_drive(8, [0], [0], 2, 1)       # one level
    with pytest.raises(ValueError):
        oracle.win_drive(8, [0], [33], 2, 1)      # above E = 0


def _fixed_weight_histogram(L, lo, hi, M, nsw, seed):
    ex = _exact_levels(L)
    G = np.zeros((M, hi - lo + 1), dtype=np.int64)
    for k in range(lo, hi + 1):
        G[:, k - lo] = int(round(ex[k] * oracle.WL_ONE)) if np.isfinite(ex[k]) else 0
    H = np.zeros_like(G, dtype=np.uint32)
    spins, E = oracle.win_drive(L, [lo], [hi], M, seed)
    # unrecorded equilibration, then the recorded sweeps
    oracle.wl_sweeps(L, [lo], [hi], M, [0], [1], seed, 0, 50, spins, E, G, H)
    H[:] = 0
    oracle.wl_sweeps(L, [lo], [hi], M, [0], [1], seed, 50, nsw, spins, E, G, H)
    return H


def test_fixed_exact_weights_give_a_flat_window():
    L, lo, hi, M = 8, 12, 22, 64
    H = _fixed_weight_histogram(L, lo, hi, M, 400, 17)
    tot = H.sum(axis=0).astype(np.float64)
    frac = tot / tot.sum()
    # per-walker shares give the error of the mean over independent walkers
    per = H.astype(np.float64) / H.sum(axis=1, keepdims=True)
    err = per.std(axis=0, ddof=1) / math.sqrt(M)
    n = hi - lo + 1
    assert np.all(np.abs(frac - 1.0 / n) < 5 * err + 1e-4), (frac, err)
    # the edge levels in particular (the count-again rule)
    for j in (0, n - 1):
        assert abs(frac[j] - 1.0 / n) < 5 * err[j] + 1e-4


def test_wang_landau_converges_at_L8():
    L = 8
    ex = _exact_levels(L)
    r = oracle.wl_run(L, [0, 14], [20, 32], 64, 11, 1e-4)
    assert all(r["converged"])
    assert r["stages"] == [14, 14]  # 2^-14 < 1e-4 <= 2^-13
    m = np.isfinite(ex)
    assert not np.isfinite(r["lng"][1])
    assert abs(r["lng"][0] - math.log(2.0)) < 1e-12
    err = np.max(np.abs(r["lng"][m] - ex[m]))
    assert err < 0.1, err
    # after the last stage every walker of a window holds the averaged
    # estimate, shifted to a minimum of 0 over the levels with states
    G = r["G"]
    for i, (a, b) in enumerate(((0, 20), (14, 32))):
        rows = G[64 * i:64 * (i + 1), :b - a + 1]
        assert np.all(rows == rows[0])
        assert min(int(rows[0][k - a]) for k in range(a, b + 1) if k != 1) == 0


def test_match_recovers_shifted_exact_pieces():
    L = 16
    K = L * L // 2
    ex = _exact_levels(L)
    lo, hi = [0, 30, 70, 100], [40, 80, 110, K]
    rng = np.random.default_rng(2)
    pieces = []
    for a, b in zip(lo, hi):
        p = ex[a:b + 1].copy()
        p[~np.isfinite(p)] = 0.0
        pieces.append(p + rng.normal() * 100)
    out = oracle.wl_match(lo, hi, pieces, K)
    m = np.isfinite(ex)
    assert np.max(np.abs(out[m] - ex[m])) < 1e-9
    assert out[1] == -np.inf


def test_stream_contract_rebuilt_site_by_site():
    L, M, seed, sweep0, nsw = 4, 2, 9, 7, 3
    lo, hi = [2], [8]
    N = L * L
    spins, E = oracle.win_drive(L, lo, hi, M, seed)
    rng = np.random.default_rng(1)
    G = rng.integers(0, 3 << 32, size=(M, hi[0] - lo[0] + 1)).astype(np.int64)
    H = np.zeros(G.shape, dtype=np.uint32)
    inc = 1 << 29
    s_ref, E_ref, G_ref, H_ref = spins.copy(), E.copy(), G.copy(), H.copy()
    oracle.wl_sweeps(L, lo, hi, M, [inc], [1], seed, sweep0, nsw, spins, E, G, H)
    for w in range(M):
        s = s_ref[w]
        k = (E_ref[w] + 2 * N) // 4
        for t in range(nsw):
            for y in range(L):
                for x in range(L):
                    i = x + L * y
                    h = s[(x + 1) % L + L * y] + s[(x - 1) % L + L * y] + s[x + L * ((y + 1) % L)] + \
                        s[x + L * ((y - 1) % L)]
                    dl = int(s[i]) * int(h) // 2
                    k2 = k + dl
                    if dl == 0:
                        acc = True
                    elif k2 < lo[0] or k2 > hi[0]:
                        acc = False
                    else:
                        d = int(G_ref[w, k2 - lo[0]]) - int(G_ref[w, k - lo[0]])
                        acc = d <= 0 or oracle.draw_word(seed, oracle.TAG_MUCA, i, w, sweep0 + t) < \
                            oracle.wl_threshold(d)
                    if acc:
                        s[i] = -s[i]
                        k = k2
                    G_ref[w, k - lo[0]] += inc
                    H_ref[w, k - lo[0]] += 1
        assert np.array_equal(s, spins[w])
        assert 4 * k - 2 * N == E[w]
        G_ref[w] -= G_ref[w].min()  # the call ends with the estimate's minimum at 0
    assert np.array_equal(G_ref, G) and np.array_equal(H_ref, H)


@pytest.mark.parametrize("L,lo,hi,rec,tol", [(8, [0, 14], [20, 32], 200, 0.15), (16, [0, 40, 90], [60, 110, 128], 1000, 0.15)])
def test_windowed_multicanonical_converges(L, lo, hi, rec, tol):
    ex = _exact_levels(L)
    r = oracle.muca_windows_run(L, lo, hi, 64, 5, rec, 100)
    assert all(r["converged"])
    m = np.isfinite(ex)
    err = np.max(np.abs(r["lng"][m] - ex[m]))
    assert err < tol, err
