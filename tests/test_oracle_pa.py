"""Pins of the oracle's population annealing (Sec. "Population annealing",
Eq. Q) and of its fixed-order prefix sum.

* The fixed-order scan is an inclusive prefix sum: exact on integer-valued
  weights (every partial sum representable), within a few ulp of an exactly
  rounded sum (math.fsum) on random weights, over one, two and three levels
  with ragged tails.
* dbeta = 0: every weight is exactly 1, so C_tot = R, Q = 1 and ln Q = 0
  exactly, and the parents are floor(u_k R) (uniform multinomial).
* Copy numbers add up to R; energies agree with the spins; the beta_0 = 0
  population is a set of independent hot starts (binomial magnetisation).
* ln Z(beta_i) = N ln 2 + sum ln Q agrees with Kaufman's exact ln Z, and the
  population energy histogram with the exact g(E) e^{-beta E}/Z, within the
  spread over independent seeds (statistical, fixed seeds).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact


@pytest.mark.parametrize("R", [1, 5, 64, 100, 4096, 4096 + 64 * 3 + 7, 64 * 64 * 2 + 5])
def test_scan_integer_weights_exact(R):
    rng = np.random.default_rng(R)
    w = rng.integers(0, 1 << 20, size=R).astype(np.float64)
    C = oracle.canonical_scan(w)
    assert np.array_equal(C, np.cumsum(w))


@pytest.mark.parametrize("R", [63, 4097, 64 * 64 * 3 + 11])
def test_scan_float_weights_close_to_exact(R):
    rng = np.random.default_rng(7 + R)
    w = np.exp(-rng.random(R) * 30.0)
    C = oracle.canonical_scan(w)
    for i in list(range(0, R, max(1, R // 97))) + [R - 1]:
        ex = math.fsum(w[:i + 1])
        assert abs(C[i] - ex) <= 16 * np.spacing(ex)


def test_zero_dbeta_step_is_exact():
    L, R = 8, 300
    pop = oracle.PAPopulation(L, R, 0, 5)
    beta = np.array([0.0, 0.0])
    E0 = pop.E.copy()
    pop.advance(beta, 0, 1)
    assert pop.Ctot[0] == float(R) and pop.lnQ[0] == 0.0
    # with C_j = j + 1 the parent of slot k is floor(u_k R)
    parents = sorted(int(math.floor(oracle.resample_u(5, k, 0, 1) * R)) for k in range(R))
    counts = np.bincount(parents, minlength=R)
    assert np.array_equal(pop.last_counts, counts)
    # contiguous placement: slots hold parents in increasing order
    assert np.array_equal(pop.E, E0[np.repeat(np.arange(R), counts)])


def test_population_invariants():
    L, R = 8, 500
    pop = oracle.PAPopulation(L, R, 1, 9)
    N = L * L
    # beta_0 = 0: independent hot starts; M per replica ~ Binomial
    M = pop.spins.reshape(R, N).sum(axis=1)
    assert abs(M.mean()) < 5 * math.sqrt(N / R)
    assert abs(M.var() / N - 1.0) < 0.25
    beta = oracle.pa_schedule(10, 0.5)
    pop.advance(beta, 3, 10)
    assert pop.last_counts.sum() == R
    for k in range(0, R, 37):
        e, _ = oracle.measure(2, L, pop.spins[k * N:(k + 1) * N])
        assert e == pop.E[k]
    for h in pop.hist:
        assert h.sum() == R


def test_lnZ_vs_kaufman_and_histogram_vs_exact():
    L, R, nsteps, theta = 8, 2000, 40, 5
    N = L * L
    beta = oracle.pa_schedule(nsteps, 1.0)
    runs = [oracle.PAPopulation(L, R, 0, 100 + s).advance(beta, theta, nsteps) for s in range(4)]
    g = exact.exact_g(L)
    for i in (10, 20, 40):
        est = np.array([p.lnZ[i] for p in runs]) / N
        ex = float(exact.kaufman_lnZ(L, beta[i])) / N
        sig = est.std(ddof=1) / math.sqrt(len(runs))
        assert abs(est.mean() - ex) < max(5 * sig, 2e-3), (i, est.mean(), ex, sig)
    # final population: energy distribution against g(E) e^{-beta E} / Z
    b = beta[-1]
    w = np.array([float(c) * math.exp(-b * (4 * k - 2 * N) - 2 * N * b) if c else 0.0 for k, c in enumerate(g)])
    pex = w / w.sum()
    uex = float((pex * (4 * np.arange(N + 1) - 2 * N)).sum()) / N
    u = np.array([(p.hist[-1] * (4 * np.arange(N + 1) - 2 * N)).sum() / R / N for p in runs])
    assert abs(u.mean() - uex) < max(5 * u.std(ddof=1) / 2, 2e-3), (u.mean(), uex)


@pytest.mark.parametrize("dbeta", [0.05, 0.3])
def test_resampling_step_against_unshifted_weights(dbeta):
    """One step without sweeps from a population of varied energies: the copy
    numbers equal those of multinomial resampling written directly from the
    reweighting factors exp(-dbeta E_j) (no shift, numpy's cumulative sum and
    binary search), with the same uniform draws u_k; C_tot relates to the
    unshifted sum by the factor exp(-2N dbeta), and ln Q to the mean factor."""
    L, R, seed = 8, 400, 31
    N = L * L
    pop = oracle.PAPopulation(L, R, 0, seed)
    E0 = pop.E.copy()
    assert len(set(E0.tolist())) > 5  # hot starts: many energy levels
    pop.advance(np.array([0.0, dbeta]), 0, 1)
    w = np.exp(-dbeta * E0.astype(np.float64))
    c = np.cumsum(w)
    u = np.array([oracle.resample_u(seed, k, 0, 1) for k in range(R)])
    parents = np.searchsorted(c, u * c[-1], side="right")
    assert np.array_equal(pop.last_counts, np.bincount(parents, minlength=R))
    assert abs(pop.Ctot[0] - c[-1] * math.exp(-2 * N * dbeta)) <= 1e-12 * c[-1] * math.exp(-2 * N * dbeta)
    assert abs(pop.lnQ[0] - math.log(w.mean())) <= 1e-12
    # the new population holds the copies in parent order
    assert np.array_equal(pop.E, E0[np.sort(parents)])


def test_anneal_resumes_from_a_checkpoint():
    """The state of an anneal is (population, energies, step number, ln Z so
    far): 6 steps in one call equal 2 + 4 steps in two calls."""
    L, R, seed, theta = 8, 150, 12, 2
    beta = oracle.pa_schedule(6, 0.6)
    a = oracle.PAPopulation(L, R, 1, seed).advance(beta, theta, 6)
    b = oracle.PAPopulation(L, R, 1, seed).advance(beta, theta, 2).advance(beta, theta, 4)
    assert np.array_equal(a.spins, b.spins) and np.array_equal(a.E, b.E)
    assert a.Ctot == b.Ctot and a.lnQ == b.lnQ and a.lnZ == b.lnZ
    assert all(np.array_equal(x, y) for x, y in zip(a.hist, b.hist))
