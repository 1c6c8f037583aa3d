"""Pins of the oracle's checkerboard sweeps (Sec. "Checkerboard scheme",
Eq. metropolis-canonical, Eq. heatbath, Eq. ising_model, Eqs. balance / DB).

Deterministic special cases:
* Metropolis at beta = 0 accepts every move, so a full sweep maps s -> -s;
* heat-bath at beta = 0 sets s_i = +1 with probability exactly 1/2, i.e. iff
  the site's random byte is below 128;
* the +-J model is covariant under a gauge transformation (s_i -> e_i s_i,
  J_ij -> e_i e_j J_ij): Metropolis acceptances depend on dE only, so the two
  trajectories agree bit for bit after undoing the gauge;
* an explicit all-ferromagnetic J equals the J = 1 path; E = 2N (mod 4) and
  M = N (mod 2) on the 2D torus.
Exact enumeration:
* every half-sweep satisfies detailed balance and the full sweep satisfies
  global balance but not detailed balance (4x4, all 65,536 states), to the
  2^-32 quantisation of the acceptance probabilities;
* long runs sample the Boltzmann energy distribution g(E) e^{-beta E} / Z on
  4x4, 2x2x4 (3D) and 3x3 (three colours), Metropolis and heat-bath.
Statistical physics (the paper's Ising application test):
* Kaufman's exact finite-lattice energy and specific heat at L = 16, 32;
* Yang's spontaneous magnetisation at beta = 0.5 from a cold start.
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


# ---------------------------------------------------------------- deterministic
@pytest.mark.parametrize("dims,L", [(2, 8), (2, 16), (3, 6)])
def test_metropolis_beta0_flips_everything(dims, L):
    s = oracle.init(dims, L, oracle.HOT, 3)
    s0 = s.copy()
    oracle.sweep(dims, L, s, 0.0, 3, 0, 0, 1)
    assert np.array_equal(s, -s0)
    J = oracle.couplings(dims, L, 5)
    oracle.sweep(dims, L, s, 0.0, 3, 0, 1, 1, J=J)
    assert np.array_equal(s, s0)


@pytest.mark.parametrize("dims,L", [(2, 8), (3, 4)])
def test_heatbath_beta0_is_coin_flip(dims, L):
    seed, rep, t = 21, 7, 5
    s = oracle.init(dims, L, oracle.COLD, 0)
    oracle.sweep(dims, L, s, 0.0, seed, rep, t, 1, rule=oracle.HEATBATH)
    Lz = L if dims == 3 else 1
    for z in range(Lz):
        for y in range(L):
            for x in range(L):
                i = x + L * (y + L * z)
                c = (x + y + z) & 1
                b = oracle.draw_byte(seed, oracle.TAG_SWEEP, i >> 1, rep, t, c)
                assert s[i] == (1 if b < 128 else -1)


def _gauge(dims, L, s, J, eps):
    """s_i -> e_i s_i, J(i, i+e_d) -> e_i e_{i+e_d} J."""
    Lz = L if dims == 3 else 1
    N = L * L * Lz
    coords = np.stack(np.meshgrid(np.arange(L), np.arange(L), np.arange(Lz), indexing="ij"), -1).reshape(-1, 3)
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    i = x + L * (y + L * z)
    Jg = J.copy().reshape(dims, N)
    nbrs = [(x + 1) % L + L * (y + L * z), x + L * ((y + 1) % L + L * z)]
    if dims == 3:
        nbrs.append(x + L * (y + L * ((z + 1) % Lz)))
    for d in range(dims):
        Jg[d, i] = J.reshape(dims, N)[d, i] * eps[i] * eps[nbrs[d]]
    return (s * eps).astype(np.int8), Jg.reshape(-1).astype(np.int8)


@pytest.mark.parametrize("dims,L", [(2, 8), (3, 6)])
def test_ea_gauge_covariance(dims, L):
    N = L ** dims
    J = oracle.couplings(dims, L, 13)
    s = oracle.init(dims, L, oracle.HOT, 13, 0)
    eps = np.where(np.random.default_rng(1).random(N) < 0.5, 1, -1).astype(np.int8)
    sg, Jg = _gauge(dims, L, s, J, eps)
    EM = oracle.sweep(dims, L, s, 1.0, 13, 0, 0, 50, J=J)
    EMg = oracle.sweep(dims, L, sg, 1.0, 13, 0, 0, 50, J=Jg)
    assert np.array_equal(EM[:, 0], EMg[:, 0])
    assert np.array_equal(s * eps, sg)


def test_ferromagnet_explicit_couplings_and_invariants():
    L = 12
    s1 = oracle.init(2, L, oracle.HOT, 4)
    s2 = s1.copy()
    EM1 = oracle.sweep(2, L, s1, 0.44, 4, 2, 10, 20)
    EM2 = oracle.sweep(2, L, s2, 0.44, 4, 2, 10, 20, J=np.ones(2 * L * L, dtype=np.int8))
    assert np.array_equal(s1, s2) and np.array_equal(EM1, EM2)
    N = L * L
    assert np.all((EM1[:, 0] - 2 * N) % 4 == 0) and np.all((EM1[:, 1] - N) % 2 == 0)
    # recorded (E, M) is the measurement of the lattice after that sweep
    assert oracle.measure(2, L, s1) == tuple(EM1[-1])


def test_sweeps_compose():
    # n sweeps from sweep0 = a then m sweeps from a + n equal n + m sweeps: the
    # stream depends on the global sweep number only (resume from a checkpoint)
    L = 10
    s1 = oracle.init(2, L, oracle.HOT, 8)
    s2 = s1.copy()
    oracle.sweep(2, L, s1, 0.3, 8, 1, 100, 7)
    oracle.sweep(2, L, s1, 0.3, 8, 1, 107, 5)
    oracle.sweep(2, L, s2, 0.3, 8, 1, 100, 12)
    assert np.array_equal(s1, s2)


# ------------------------------------------------------------------ enumeration
def _half_step_probs(L, beta, state_spins, colour_mask):
    """Per-state, per-site flip probability of a Metropolis half-sweep."""
    T = oracle.metropolis_table(beta).astype(np.float64) / 2.0 ** 32
    N = L * L
    idx = np.arange(N)
    x, y = idx % L, idx // L
    nb = np.stack([(x + 1) % L + L * y, (x - 1) % L + L * y, x + L * ((y + 1) % L), x + L * ((y - 1) % L)], 1)
    h = state_spins[:, nb].sum(axis=2)
    dE = 2 * state_spins * h
    p = np.where(dE <= 0, 1.0, T[np.clip(dE // 4, 0, 3)])
    return np.where(colour_mask[None, :], p, 0.0)


def test_balance_and_detailed_balance_4x4():
    L, N, beta = 4, 16, 0.35
    E, _ = exact.enumerate_states(2, (L, L))
    idx = np.arange(1 << N)
    spins = 1 - 2 * ((idx[:, None] >> np.arange(N)) & 1)
    w = np.exp(-beta * (E - E.min()))
    pi = w / w.sum()
    sites = np.arange(N)
    colour = ((sites % L) + (sites // L)) & 1
    dist = pi.copy()
    for c in (0, 1):
        mask = colour == c
        p = _half_step_probs(L, beta, spins, mask)
        csites = sites[mask]
        # all subsets F of the colour-c sites: successor s ^ F
        sub = np.arange(1 << csites.size)
        flipbits = ((sub[:, None] >> np.arange(csites.size)) & 1).astype(bool)
        Fmask = (flipbits.astype(np.int64) << csites).sum(axis=1)
        pc = p[:, csites]
        P = np.ones((1 << N, sub.size))
        for k in range(csites.size):
            P *= np.where(flipbits[None, :, k], pc[:, k:k + 1], 1.0 - pc[:, k:k + 1])
        succ = idx[:, None] ^ Fmask[None, :]
        # detailed balance of the half step: pi(s) P(s->s') = pi(s') P(s'->s);
        # the reverse move of F from s' is the same subset F
        fwd = pi[:, None] * P
        rev = pi[succ] * P[succ, np.arange(sub.size)[None, :]]
        rel = np.abs(fwd - rev) / np.maximum(fwd, 1e-300)
        assert np.max(np.where(fwd > 1e-30, rel, 0.0)) < 1e-7
        dist = np.bincount(succ.ravel(), weights=(dist[:, None] * P).ravel(), minlength=1 << N)
        if c == 0:
            P0, succ0 = P, succ
        else:
            P1, succ1 = P, succ
    # global balance of the full sweep
    assert np.max(np.abs(dist - pi) / pi) < 1e-7
    # ... but the full sweep (even then odd) violates detailed balance
    s = 0
    row = np.zeros(1 << N)
    for a in range(P0.shape[1]):
        m = succ0[s, a]
        np.add.at(row, succ1[m], P0[s, a] * P1[m])
    target = int(np.argmax(row * (np.arange(1 << N) != s)))
    back = 0.0
    for a in range(P0.shape[1]):
        m = succ0[target, a]
        back += P0[target, a] * P1[m][succ1[m] == s].sum()
    lhs, rhs = pi[s] * row[target], pi[target] * back
    assert abs(lhs - rhs) / lhs > 1e-3


def _energy_histogram_test(E_series, gdict, beta, label):
    levels = np.array(sorted(gdict))
    with np.errstate(over="ignore"):
        w = np.array([gdict[e] * math.exp(-beta * (e - levels.min())) for e in levels])
    p = w / w.sum()
    E_series = np.asarray(E_series)
    for e, pe in zip(levels, p):
        ind = (E_series == e).astype(np.float64)
        sig = _batch_sigma(ind)
        if pe < 1e-3:
            continue
        assert abs(ind.mean() - pe) < 5 * sig + 1e-4, (label, e, ind.mean(), pe, sig)


@pytest.mark.parametrize("rule", [oracle.METROPOLIS, oracle.HEATBATH])
def test_boltzmann_4x4(rule):
    beta = 0.3
    s = oracle.init(2, 4, oracle.HOT, 31)
    EM = oracle.sweep(2, 4, s, beta, 31, 0, 0, 200000, rule=rule)
    _energy_histogram_test(EM[1000:, 0], exact.enumerate_torus(2, (4, 4)), beta, ("4x4", rule))


@pytest.mark.parametrize("rule", [oracle.METROPOLIS, oracle.HEATBATH])
def test_boltzmann_2x2x4(rule):
    beta = 0.2
    s = oracle.init(3, (2, 2, 4), oracle.HOT, 32)
    EM = oracle.sweep(3, (2, 2, 4), s, beta, 32, 0, 0, 150000, rule=rule)
    _energy_histogram_test(EM[1000:, 0], exact.enumerate_torus(3, (2, 2, 4)), beta, ("2x2x4", rule))


def test_boltzmann_3x3_three_colours():
    beta = 0.4
    s = oracle.init(2, 3, oracle.HOT, 33)
    EM = oracle.sweep_q3(3, s, beta, 33, 0, 0, 200000)
    _energy_histogram_test(EM[1000:, 0], exact.enumerate_torus(2, (3, 3)), beta, "3x3")


# ------------------------------------------------------------ statistical physics
@pytest.mark.parametrize("L,beta,nsw", [(16, 0.4, 60000), (16, exact.BETA_C, 60000), (16, 0.5, 40000),
                                        (32, 0.4, 20000)])
def test_kaufman_energy_and_specific_heat(L, beta, nsw):
    N = L * L
    s = oracle.init(2, L, oracle.HOT, 41)
    EM = oracle.sweep(2, L, s, beta, 41, 0, 0, nsw)
    e = EM[2000:, 0].astype(np.float64) / N
    u_ex, cv_ex = exact.kaufman_u_cv(L, beta, dps=30)
    assert abs(e.mean() - u_ex) < 5 * _batch_sigma(e), (e.mean(), u_ex)
    cv = beta ** 2 * N * e.var()
    # specific heat from fluctuations: batch the variance estimator
    nb = 20
    n = (e.size // nb) * nb
    cvb = beta ** 2 * N * e[:n].reshape(nb, -1).var(axis=1)
    assert abs(cv - cv_ex) < 5 * cvb.std(ddof=1) / math.sqrt(nb) + 0.02 * cv_ex, (cv, cv_ex)


def test_yang_magnetisation_cold_start():
    L, beta = 64, 0.5
    s = oracle.init(2, L, oracle.COLD, 0)
    EM = oracle.sweep(2, L, s, beta, 43, 0, 0, 3000)
    m = np.abs(EM[200:, 1]).astype(np.float64) / (L * L)
    assert abs(m.mean() - exact.yang_m(beta)) < 5 * _batch_sigma(m) + 1e-3, (m.mean(), exact.yang_m(beta))
