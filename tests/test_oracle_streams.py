"""The oracle's use of its random streams, against the contract stated with
each call: which item, replica id, sweep number and colour every decision
draws, and in which order the sub-lattices are updated.

Distribution-level pins (balance, Boltzmann, Kaufman, flat histograms) cannot
see any of this: every assignment of independent uniforms to decisions gives
a correct Markov chain.  Each test rebuilds the decisions of a tiny case from
the pinned draw primitives and the pinned tables, walking the lattice
differently from the oracle (by same-colour index rather than by site), and
compares the result bit for bit.
"""
import numpy as np
import pytest

import oracle

SW, SW_LO, MUCA = oracle.TAG_SWEEP, oracle.TAG_SWEEP_LO, oracle.TAG_MUCA


def _coords(i, Lx, Ly):
    return i % Lx, (i // Lx) % Ly, i // (Lx * Ly)


def _field(s, J, i, shape, dims):
    """h_i = sum over bonds of J s_j; J[d N + i] belongs to the bond (i, i + e_d)."""
    Lx, Ly, Lz = shape
    N = Lx * Ly * Lz
    x, y, z = _coords(i, Lx, Ly)
    steps = [(1, 0, 0), (0, 1, 0), (0, 0, 1)][:dims]
    h = 0
    for d, (dx, dy, dz) in enumerate(steps):
        up = (x + dx) % Lx + Lx * ((y + dy) % Ly + Ly * ((z + dz) % Lz))
        dn = (x - dx) % Lx + Lx * ((y - dy) % Ly + Ly * ((z - dz) % Lz))
        h += (1 if J is None else int(J[d * N + i])) * int(s[up])
        h += (1 if J is None else int(J[d * N + dn])) * int(s[dn])
    return h


def _sweeps_by_colour_index(dims, shape, s, J, rule, beta, seed, replica, sweep0, nsweeps):
    Lx, Ly, Lz = shape
    N = Lx * Ly * Lz
    s = s.copy()
    Tm = [int(v) for v in oracle.metropolis_table(beta)]
    Thb = [int(v) for v in oracle.heatbath_table(beta, 2 * dims)]
    EM = []
    for t in range(nsweeps):
        sweep = sweep0 + t
        for c in (0, 1):  # the even sub-lattice (x + y + z even) first
            for j in range(N // 2):
                # sites 2j and 2j + 1 share the same-colour index j; exactly one
                # of them (x even, then x + 1) has colour c
                x0, y0, z0 = _coords(2 * j, Lx, Ly)
                i = 2 * j + (((x0 + y0 + z0) & 1) ^ c)
                h = _field(s, J, i, shape, dims)
                r = oracle.draw32(seed, SW, SW_LO, j, replica, sweep, c)
                if rule == oracle.METROPOLIS:
                    dE = 2 * int(s[i]) * h
                    if dE <= 0 or r < Tm[dE // 4]:
                        s[i] = -s[i]
                else:
                    s[i] = 1 if r < Thb[h + 2 * dims] else -1
        EM.append(oracle.measure(dims, (Lx, Ly, Lz), s, J))
    return s, np.array(EM, dtype=np.int64)


@pytest.mark.parametrize("dims,shape,rule,beta,withJ", [
    (2, (4, 6, 1), oracle.METROPOLIS, 0.44, False),
    (2, (6, 4, 1), oracle.HEATBATH, 0.7, True),
    (3, (4, 4, 6), oracle.HEATBATH, 0.3, True),
    (3, (6, 4, 4), oracle.METROPOLIS, 0.25, False),
])
def test_sweep_draws_follow_the_stream_contract(dims, shape, rule, beta, withJ):
    seed, replica = 0x1234_5678_9ABC, 5
    sweep0 = (1 << 32) - 2  # the sweep number crosses into the counter's high bits
    L = shape[:dims]
    s0 = oracle.init(dims, L, oracle.HOT, seed, replica)
    J = oracle.couplings(dims, L, 17) if withJ else None
    want, want_em = _sweeps_by_colour_index(dims, shape, s0, J, rule, beta, seed, replica, sweep0, 4)
    got = s0.copy()
    em = oracle.sweep(dims, L, got, beta, seed, replica, sweep0, 4, rule=rule, J=J)
    assert np.array_equal(got, want)
    assert np.array_equal(em, want_em)


def test_pa_steps_compose_resampling_and_documented_sweeps():
    """With dbeta = 0 the parents are floor(u_k R) (u_k of step i, population
    p); the copies then run theta sweeps as replica id p R + slot with sweep
    numbers (i - 1) theta .. i theta - 1."""
    L, R, pop, seed, theta, b = 4, 40, 1, 77, 2, 0.35
    N = L * L
    popn = oracle.PAPopulation(L, R, pop, seed)
    spins = popn.spins.reshape(R, N).copy()
    popn.advance(np.array([b, b, b]), theta, 2)
    for i in (1, 2):
        parents = sorted(int(oracle.resample_u(seed, k, pop, i) * R) for k in range(R))
        spins = spins[parents].copy()
        for k in range(R):
            row = spins[k].copy()
            oracle.sweep(2, L, row, b, seed, pop * R + k, (i - 1) * theta, theta, record=False)
            spins[k] = row
    assert np.array_equal(popn.spins.reshape(R, N), spins)
    assert np.array_equal(popn.E, [oracle.measure(2, L, spins[k])[0] for k in range(R)])


def test_muca_draws_follow_the_stream_contract():
    """Walker w visits the sites in typewriter order; the move at site i of
    sweep t draws word (i mod 4) of Philox(MUCA, i div 4, w, t); the histogram
    counts the level after every attempt."""
    L, W, seed, sweep0, nsw = 4, 3, 99, (1 << 32) - 1, 3
    N, K = L * L, L * L // 2
    lnW = -0.4 * np.sqrt(np.arange(K + 1, dtype=np.float64))[::-1]  # favours low energies
    lnW -= lnW[-1]
    T = oracle.muca_table(L, lnW).reshape(K + 1, 4)
    spins, E = oracle.muca_start(L, W, seed)
    want_s, want_E = spins.reshape(W, N).copy(), E.copy()
    H = np.zeros(K + 1, dtype=np.int64)
    for w in range(W):
        s, e = want_s[w], int(want_E[w])
        for t in range(nsw):
            for i in range(N):
                dE = 2 * int(s[i]) * _field(s, None, i, (L, L, 1), 2)
                if e + dE <= 0:  # moves out of the window [-2N, 0] are rejected
                    r = oracle.draw_word(seed, MUCA, i, w, sweep0 + t)
                    k = (e + 2 * N) // 4
                    col = {-8: 0, -4: 1, 4: 2, 8: 3}.get(dE)
                    if dE == 0 or r < int(T[k, col]):
                        s[i] = -s[i]
                        e += dE
                H[(e + 2 * N) // 4] += 1
        want_E[w] = e
    Hg = oracle.muca_sweeps(L, spins, E, lnW, seed, sweep0, nsw, True)
    assert np.array_equal(spins.reshape(W, N), want_s)
    assert np.array_equal(E, want_E)
    assert np.array_equal(Hg, H)
