"""CPU oracle for the Monte Carlo hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

The arithmetic lives in ``mcoracle.c`` (plain C, built with gcc, OpenMP over
independent sites / replicas / walkers); this module only builds it, marshals
numpy arrays and strings the steps of the population-annealing and
multicanonical loops together in the order the paper gives them (M. Weigel,
arXiv:1709.04394, Sec. "Population annealing" and Sec. "Multicanonical
simulations").  Exact references (enumeration, Kaufman, Onsager, Yang, exact
density of states) are in ``oracle.exact``; the FP64 MLP is ``oracle.mlp``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcoracle.c")
_LIB = os.path.join(_HERE, "libmcoracle.so")

TAG_INIT, TAG_SWEEP, TAG_COUPLING, TAG_RESAMPLE = 1, 2, 3, 4
TAG_MUCA, TAG_MLP_INIT, TAG_SWEEP_LO, TAG_MUCA_LO = 5, 6, 7, 8
TAG_EXCHANGE = 9
TAG_WINDOW = 10
METROPOLIS, HEATBATH = 0, 1
COLD, HOT = 0, 1


def build(force: bool = False) -> str:
    """Compile mcoracle.c with gcc (plain IEEE double, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
               "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [u8p, u8p, u8p]
        L.orc_draw_byte.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_uint32]
        L.orc_draw_byte.restype = ctypes.c_uint32
        L.orc_draw32.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_draw32.restype = ctypes.c_uint32
        L.orc_draw_word.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint64]
        L.orc_draw_word.restype = ctypes.c_uint32
        L.orc_resample_u.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_resample_u.restype = ctypes.c_double
        L.orc_metropolis_table.argtypes = [ctypes.c_double, ctypes.c_int, u8p]
        L.orc_heatbath_table.argtypes = [ctypes.c_double, ctypes.c_int, u8p]
        L.orc_init.argtypes = [ctypes.c_int] * 4 + [u8p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_couplings.argtypes = [ctypes.c_int] * 4 + [u8p, ctypes.c_uint64]
        L.orc_couplings_of.argtypes = [ctypes.c_int] * 4 + [u8p, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_measure.argtypes = [ctypes.c_int] * 4 + [u8p, u8p, u8p, u8p]
        L.orc_measure.restype = None
        L.orc_sweep.argtypes = [ctypes.c_int] * 4 + [u8p, u8p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                                     ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, u8p]
        L.orc_sweep_q3.argtypes = [ctypes.c_int, u8p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_int, u8p]
        L.orc_sweep_dcb.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_double, ctypes.c_uint64,
                                    ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, u8p]
        L.orc_canonical_scan.argtypes = [u8p, u8p, ctypes.c_int64]
        L.orc_canonical_scan.restype = None
        L.orc_pa_init.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, u8p, u8p]
        L.orc_pa_steps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p,
                                   ctypes.c_int, ctypes.c_uint64, u8p, u8p, u8p, u8p, u8p, u8p]
        L.orc_muca_table.argtypes = [ctypes.c_int, u8p, u8p]
        L.orc_muca_table.restype = None
        L.orc_muca_start.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u8p, u8p]
        L.orc_muca_strat_level.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_muca_settle.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p]
        L.orc_muca_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, u8p, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_int, ctypes.c_int, u8p]
        L.orc_wl_threshold.argtypes = [ctypes.c_uint64]
        L.orc_wl_threshold.restype = ctypes.c_uint64
        L.orc_win_drive.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, u8p, ctypes.c_uint64,
                                    ctypes.c_int, u8p, u8p]
        L.orc_wl_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p, u8p, ctypes.c_int, u8p, u8p,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, u8p, u8p, u8p, u8p]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments (rc=%d)" % (what, rc))


# --------------------------------------------------------------------------- RNG
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw_byte(seed, tag, j, replica, sweep, phase):
    return int(lib().orc_draw_byte(seed, tag, j, replica, sweep, phase))


def draw32(seed, tag, tag_lo, j, replica, sweep, phase):
    return int(lib().orc_draw32(seed, tag, tag_lo, j, replica, sweep, phase))


def draw_word(seed, tag, j, replica, sweep):
    return int(lib().orc_draw_word(seed, tag, j, replica, sweep))


def resample_u(seed, k, pop, step):
    return float(lib().orc_resample_u(seed, k, pop, step))


# ------------------------------------------------------------------------ tables
def metropolis_table(beta, kmax=3):
    T = np.zeros(kmax + 1, dtype=np.uint64)
    lib().orc_metropolis_table(float(beta), kmax, _p(T))
    return T


def heatbath_table(beta, z):
    T = np.zeros(2 * z + 1, dtype=np.uint64)
    lib().orc_heatbath_table(float(beta), z, _p(T))
    return T


# ---------------------------------------------------------------------- lattices
def _shape(dims, L):
    if isinstance(L, int):
        L = (L,) * dims
    Lx, Ly = L[0], L[1]
    Lz = L[2] if dims == 3 else 1
    return Lx, Ly, Lz


def init(dims, L, start, seed, replica=0):
    Lx, Ly, Lz = _shape(dims, L)
    s = np.zeros(Lx * Ly * Lz, dtype=np.int8)
    _check(lib().orc_init(dims, Lx, Ly, Lz, _p(s), start, seed, replica), "init")
    return s


def couplings(dims, L, seed, realisation=0):
    """Bimodal couplings of disorder realisation `realisation` (int8
    [dims][N], +1 / -1 with p = 1/2)."""
    Lx, Ly, Lz = _shape(dims, L)
    J = np.zeros(dims * Lx * Ly * Lz, dtype=np.int8)
    if realisation == 0:
        _check(lib().orc_couplings(dims, Lx, Ly, Lz, _p(J), seed), "couplings")
    else:
        _check(lib().orc_couplings_of(dims, Lx, Ly, Lz, _p(J), seed, realisation), "couplings")
    return J


def measure(dims, L, s, J=None):
    Lx, Ly, Lz = _shape(dims, L)
    E = np.zeros(1, dtype=np.int64)
    M = np.zeros(1, dtype=np.int64)
    s = np.ascontiguousarray(s, dtype=np.int8)
    Jc = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
    lib().orc_measure(dims, Lx, Ly, Lz, _p(s), _p(Jc), _p(E), _p(M))
    return int(E[0]), int(M[0])


def sweep(dims, L, s, beta, seed, replica, sweep0, nsweeps, rule=METROPOLIS, J=None, record=True):
    """Run nsweeps checkerboard sweeps in place on int8 lattice s; returns EM [n,2] or None."""
    Lx, Ly, Lz = _shape(dims, L)
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.size == Lx * Ly * Lz
    EM = np.zeros((nsweeps, 2), dtype=np.int64) if record else None
    Jc = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
    _check(lib().orc_sweep(dims, Lx, Ly, Lz, _p(s), _p(Jc), rule, float(beta), seed, replica, sweep0,
                           nsweeps, _p(EM)), "sweep")
    return EM


def sweep_q3(L, s, beta, seed, replica, sweep0, nsweeps, record=True):
    EM = np.zeros((nsweeps, 2), dtype=np.int64) if record else None
    _check(lib().orc_sweep_q3(L, _p(s), float(beta), seed, replica, sweep0, nsweeps, _p(EM)), "sweep_q3")
    return EM


def sweep_dcb(L, s, beta, seed, replica, sweep0, nsweeps, T, k, record=True):
    """Double-checkerboard Metropolis sweeps of the L x L ferromagnet with
    T x T tiles and k hits per tile (orc_sweep_dcb), in place on int8 s;
    returns EM [n, 2] or None."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.size == L * L
    EM = np.zeros((nsweeps, 2), dtype=np.int64) if record else None
    _check(lib().orc_sweep_dcb(L, T, k, _p(s), float(beta), seed, replica, sweep0, nsweeps, _p(EM)), "sweep_dcb")
    return EM


# ----------------------------------------------------------- population annealing
def canonical_scan(w):
    w = np.ascontiguousarray(w, dtype=np.float64)
    C = np.zeros_like(w)
    lib().orc_canonical_scan(_p(w), _p(C), w.size)
    return C


def pa_schedule(nsteps, beta_final=1.0):
    """beta_i = i * beta_final / nsteps (linear annealing from beta_0 = 0)."""
    return np.array([i * beta_final / nsteps for i in range(nsteps + 1)], dtype=np.float64)


class PAPopulation:
    """One annealing population of R replicas of the L x L ferromagnet."""

    def __init__(self, L, R, pop, seed):
        self.L, self.R, self.pop, self.seed = L, R, pop, seed
        self.N = L * L
        self.spins = np.zeros(R * self.N, dtype=np.int8)
        self.E = np.zeros(R, dtype=np.int64)
        _check(lib().orc_pa_init(L, R, pop, seed, _p(self.spins), _p(self.E)), "pa_init")
        self.step = 0
        self.lnZ = [self.N * math.log(2.0)]
        self.lnQ, self.Ctot = [], []
        h0 = np.zeros(self.N + 1, dtype=np.int64)
        np.add.at(h0, (self.E + 2 * self.N) // 4, 1)
        self.hist = [h0]
        self.last_counts = None

    def advance(self, beta, theta, nsteps):
        Ct = np.zeros(nsteps, dtype=np.float64)
        lq = np.zeros(nsteps, dtype=np.float64)
        hist = np.zeros((nsteps, self.N + 1), dtype=np.int64)
        counts = np.zeros(self.R, dtype=np.int32)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        _check(lib().orc_pa_steps(self.L, self.R, self.pop, self.step + 1, nsteps, _p(beta), theta, self.seed,
                                  _p(self.spins), _p(self.E), _p(Ct), _p(lq), _p(hist), _p(counts)), "pa_steps")
        for s in range(nsteps):
            self.Ctot.append(float(Ct[s]))
            self.lnQ.append(float(lq[s]))
            # ln Z(beta_i) = ln Z(beta_{i-1}) + ln Q_i, ln Z(0) = N ln 2
            self.lnZ.append(self.lnZ[-1] + float(lq[s]))
            self.hist.append(hist[s])
        self.step += nsteps
        self.last_counts = counts
        return self


def pa_anneal(Ls, R, beta, theta, seed, nsteps=None):
    """All populations (one per L) from beta_0 = 0 through the whole schedule."""
    nsteps = len(beta) - 1 if nsteps is None else nsteps
    pops = []
    for p, L in enumerate(Ls):
        pops.append(PAPopulation(L, R, p, seed).advance(beta, theta, nsteps))
    return pops


# -------------------------------------------------------------------- multicanonical
def muca_levels(L):
    """Number of levels in the window [-2N, 0]: k = (E + 2N)/4 = 0..N/2."""
    return L * L // 2 + 1


def muca_table(L, lnW):
    lnW = np.ascontiguousarray(lnW, dtype=np.float64)
    T = np.zeros((muca_levels(L), 4), dtype=np.uint64)
    lib().orc_muca_table(L, _p(lnW), _p(T))
    return T


MUCA_HOT, MUCA_STRATIFIED = 0, 1


def muca_strat_level(w, walkers):
    return lib().orc_muca_strat_level(w, walkers)


def muca_start(L, walkers, seed, start=MUCA_HOT):
    N = L * L
    spins = np.zeros(walkers * N, dtype=np.int8)
    E = np.zeros(walkers, dtype=np.int64)
    _check(lib().orc_muca_start(L, walkers, seed, start, _p(spins), _p(E)), "muca_start")
    return spins, E


def muca_sweeps(L, spins, E, lnW, seed, sweep0, nsweeps, record):
    walkers = E.size
    H = np.zeros(muca_levels(L), dtype=np.int64)
    lnW = np.ascontiguousarray(lnW, dtype=np.float64)
    _check(lib().orc_muca_sweeps(L, walkers, _p(spins), _p(E), _p(lnW), seed, sweep0, nsweeps,
                                 1 if record else 0, _p(H)), "muca_sweeps")
    return H


def muca_flat_levels(L):
    """Levels of the window that any state can reach: all but k = 1."""
    K = muca_levels(L)
    mask = np.ones(K, dtype=bool)
    mask[1] = False
    return mask


def muca_flatness(L, H):
    m = muca_flat_levels(L)
    h = H[m]
    return float(h.min()) / float(h.max()) if h.max() > 0 else 0.0


def muca_update(L, lnW, H):
    """W^(n+1) = W^(n) / H^(n) (Eq. weight_modification) in logs, where H > 0;
    then renormalised so that ln W at E = 0 (level N/2) is zero."""
    out = np.array(lnW, dtype=np.float64)
    for k in range(out.size):
        if H[k] > 0:
            out[k] = out[k] - math.log(float(H[k]))
    ref = out[-1]
    for k in range(out.size):
        out[k] = out[k] - ref
    return out


MUCA_PREP_GROUPS = 16


def muca_prep_betas(L, walkers, lnW):
    """Inverse temperature of each preparation group: the slope -d ln W / dE
    of the initial weights (central difference, dE = 8 between levels k - 1
    and k + 1) at the group's target level k_g = round((g + 1/2) K / G),
    clamped to 2 .. K - 1, and at least 0.  Flat weights give 0 everywhere."""
    K = muca_levels(L) - 1
    G = min(MUCA_PREP_GROUPS, walkers)
    out = []
    for g in range(G):
        k = ((2 * g + 1) * K + G) // (2 * G)
        k = min(max(k, 2), K - 1)
        out.append(max(0.0, -(float(lnW[k + 1]) - float(lnW[k - 1])) / 8.0))
    return out


def muca_prepare(L, spins, E, seed, lnW, prep_sweeps):
    """Walkers thermalised to the initial weights: walker group g (walkers
    g W / G .. (g + 1) W / G - 1) runs prep_sweeps canonical Metropolis sweeps
    at muca_prep_betas()[g] (replica id = walker, sweeps 0 ..), then every
    walker's energy is recomputed and a walker above the window has its odd
    sub-lattice flipped."""
    walkers = E.size
    N = L * L
    G = min(MUCA_PREP_GROUPS, walkers)
    betas = muca_prep_betas(L, walkers, lnW)
    for g in range(G):
        for w in range(g * walkers // G, (g + 1) * walkers // G):
            s = spins[w * N:(w + 1) * N]
            sweep(2, L, s, betas[g], seed, w, 0, prep_sweeps, record=False)
    _check(lib().orc_muca_settle(L, walkers, _p(spins), _p(E)), "muca_settle")


def muca_run(L, walkers, seed, eq_sweeps, rec_sweeps, max_iter, prod_sweeps, flat=0.8, lnW_init=None,
             start=MUCA_HOT, rec_max=0, eq_scale=0, prep_sweeps=0, rec_rule=0):
    """Parallel-walker multicanonical iteration: every walker shares W; the
    histograms of all walkers are added; the weights follow the plain recursion
    until the histogram is flat (min/max over reachable levels >= flat); then a
    production run at fixed weights gives ln g = ln H - ln W.  Iteration
    length: rec_sweeps recorded sweeps, doubled (up to rec_max) after every
    iteration whose histogram reached every level of the window (rec_rule 0)
    or after every such iteration whose flatness did not improve on the
    previous one (rec_rule 1); each iteration first runs eq_sweeps + eq_scale * R
    unrecorded sweeps.  prep_sweeps > 0 thermalises the walkers to the initial
    weights first (muca_prepare)."""
    K = muca_levels(L)
    lnW = np.zeros(K) if lnW_init is None else np.array(lnW_init, dtype=np.float64)
    spins, E = muca_start(L, walkers, seed, start)
    if prep_sweeps > 0:
        muca_prepare(L, spins, E, seed, lnW, prep_sweeps)
    reach = muca_flat_levels(L)
    sweep = 0
    it, converged, ratio, prev = 0, False, 0.0, 0.0
    R = rec_sweeps
    history = []
    while it < max_iter:
        neq = eq_sweeps + eq_scale * R
        muca_sweeps(L, spins, E, lnW, seed, sweep, neq, False)
        sweep += neq
        H = muca_sweeps(L, spins, E, lnW, seed, sweep, R, True)
        sweep += R
        it += 1
        ratio = muca_flatness(L, H)
        history.append(ratio)
        if ratio >= flat:
            converged = True
            break
        covered = bool(np.all(H[reach] > 0))
        if covered and (rec_rule == 0 or ratio <= prev):
            R = min(2 * R, max(rec_max, rec_sweeps))
        prev = ratio if covered else 0.0
        lnW = muca_update(L, lnW, H)
    Hp = muca_sweeps(L, spins, E, lnW, seed, sweep, prod_sweeps, True) if prod_sweeps > 0 else None
    lng = None
    if Hp is not None:
        lng = np.full(K, -np.inf)
        for k in range(K):
            if Hp[k] > 0:
                lng[k] = math.log(float(Hp[k])) - lnW[k]
    return dict(lnW=lnW, iterations=it, converged=converged, min_over_max=ratio, sweeps_per_walker=sweep,
                H_prod=Hp, lng=lng, spins=spins, E=E, history=history)


# ---------------------------------------------------------- parallel tempering
def pt_exchange(beta, E, temp_of, replica_at, seed, rnd, accepted, pt_set=0):
    """One round of replica-exchange moves (Sec. "Parallel Tempering", Eq. pt).
    Temperatures are indexed in order of increasing beta; replica_at[i] is the
    replica held at temperature i and temp_of[a] its inverse.  Round rnd
    proposes the pairs (i, i + 1) with i = rnd mod 2, rnd mod 2 + 2, ...  With
    a, b the replicas at i and i + 1 the exchange is accepted with probability
    min(1, exp((beta_i - beta_{i+1}) (E_a - E_b))): always when the exponent is
    >= 0, else iff r32 < ceil(exp(exponent) 2^32), r32 = word (i mod 4) of
    Philox(EXCHANGE, i div 4, pt_set, rnd), pt_set the index of this set of
    replicas among independent sets run side by side (0 for a single set).
    An accepted exchange swaps the two replicas' temperatures in both maps and
    counts in accepted[i].  The maps and accepted are updated in place."""
    nT = len(beta)
    for i in range(rnd % 2, nT - 1, 2):
        a, b = replica_at[i], replica_at[i + 1]
        x = (beta[i] - beta[i + 1]) * float(E[a] - E[b])
        if x >= 0.0:
            acc = True
        else:
            acc = draw_word(seed, TAG_EXCHANGE, i, pt_set, rnd) < math.ceil(math.ldexp(math.exp(x), 32))
        if acc:
            replica_at[i], replica_at[i + 1] = b, a
            temp_of[a], temp_of[b] = i + 1, i
            accepted[i] += 1


def pt_run(dims, L, beta, seed, rounds, theta, rule=METROPOLIS, start=HOT, pt_set=0):
    """Parallel tempering of len(beta) = nT replicas of one lattice shape, the
    set pt_set of independent sets: replica r has replica id pt_set nT + r and
    starts from init(start, seed, that id); per round every replica runs theta
    sweeps at the inverse temperature it holds (its replica id, sweep numbers
    round theta + t), then pt_exchange acts on the energies after those
    sweeps.  Returns the energies seen at each temperature per round ([rounds]
    [nT], before the exchange), the final maps and the acceptance counts."""
    nT = len(beta)
    rid = [pt_set * nT + r for r in range(nT)]
    spins = [init(dims, L, start, seed, rid[r]) for r in range(nT)]
    temp_of, replica_at = list(range(nT)), list(range(nT))
    accepted = [0] * (nT - 1)
    E = np.zeros(nT, dtype=np.int64)
    E_at = np.zeros((rounds, nT), dtype=np.int64)
    for rnd in range(rounds):
        for r in range(nT):
            EM = sweep(dims, L, spins[r], beta[temp_of[r]], seed, rid[r], rnd * theta, theta, rule=rule)
            E[r] = EM[-1, 0] if theta > 0 else measure(dims, L, spins[r])[0]
        E_at[rnd] = [E[replica_at[i]] for i in range(nT)]
        pt_exchange(beta, E, temp_of, replica_at, seed, rnd, accepted, pt_set)
    return dict(E_at=E_at, temp_of=temp_of, replica_at=replica_at, accepted=accepted, spins=spins)


# ------------------------------------------------------ Wang-Landau in windows
# Sec. "Wang-Landau update": g(E) starts at 1 and is multiplied by f at every
# visit, moves are accepted with min[1, g(E)/g(E')], f -> sqrt(f) once the
# histogram is flat (minimum >= 80 % of the mean), until ln f is below a
# threshold.  Parallel form (same section, and the windows of Sec.
# "Multicanonical simulations"): the level range is split into overlapping
# windows, each sampled by M walkers with their own estimates; a move out of
# the window is rejected and the current level counted again; the walkers'
# estimates are averaged when all of a window's walkers have flat histograms,
# before f is reduced; the windows' pieces are matched on their overlaps.
WL_ONE = 1 << 32  # ln g unit: estimates are integers in units of 2^-32


def wl_threshold(x):
    """ceil(exp(-x 2^-32) 2^32), at least 1, for an estimate difference x > 0
    (the table product of orc_wl_threshold)."""
    return int(lib().orc_wl_threshold(int(x)))


def _windows(lo, hi):
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    hi = np.ascontiguousarray(hi, dtype=np.int32)
    return lo, hi, int((hi - lo).max()) + 1


def win_drive(L, lo, hi, M, seed, max_pass=1000):
    """Walkers of every window driven from the ground state into their window
    (orc_win_drive); returns (spins [nwin M][N], E [nwin M])."""
    lo, hi, _ = _windows(lo, hi)
    W = lo.size * M
    spins = np.zeros((W, L * L), dtype=np.int8)
    E = np.zeros(W, dtype=np.int64)
    _check(lib().orc_win_drive(L, lo.size, M, _p(lo), _p(hi), seed, max_pass, _p(spins), _p(E)), "win_drive")
    return spins, E


def wl_sweeps(L, lo, hi, M, inc, active, seed, sweep0, nsweeps, spins, E, G, H):
    """nsweeps Wang-Landau sweeps of the walkers of the active windows
    (orc_wl_sweeps), in place on spins, E, G [nwin M][wmax], H [nwin M][wmax]."""
    lo, hi, wmax = _windows(lo, hi)
    assert G.shape == (lo.size * M, wmax) and H.shape == G.shape
    inc = np.ascontiguousarray(inc, dtype=np.int64)
    act = np.ascontiguousarray(active, dtype=np.uint8)
    _check(lib().orc_wl_sweeps(L, lo.size, M, _p(lo), _p(hi), wmax, _p(inc), _p(act), seed, sweep0, nsweeps,
                               _p(spins), _p(E), _p(G), _p(H)), "wl_sweeps")


def wl_levels_with_states(lo, hi):
    """Window levels that have states on the 2D L x L torus (L >= 4): all of
    [lo, hi] but level 1 (E = -2N + 4)."""
    return [k for k in range(lo, hi + 1) if k != 1]


def wl_flat(Hw, lo, hi, flat):
    """min H >= flat * mean H over the window levels with states."""
    ks = [k - lo for k in wl_levels_with_states(lo, hi)]
    h = [int(Hw[j]) for j in ks]
    return float(min(h)) * float(len(h)) >= flat * float(sum(h))


def wl_average(G, lo, hi, M, i):
    """Average of window i's walker estimates (floor of the integer mean per
    level), shifted so that its minimum over the levels with states is 0, then
    given to every walker of the window."""
    n = hi[i] - lo[i] + 1
    rows = G[i * M:(i + 1) * M, :n]
    avg = np.array([sum(int(v) for v in rows[:, j]) // M for j in range(n)], dtype=np.int64)
    ks = [k - lo[i] for k in wl_levels_with_states(lo[i], hi[i])]
    avg -= min(int(avg[j]) for j in ks)
    G[i * M:(i + 1) * M, :n] = avg
    return avg


def wl_match(lo, hi, pieces, K):
    """One ln g over [0, K] from the windows' pieces (pieces[i][k - lo_i]):
    window i + 1 is shifted by the mean of (previous, shifted) - (own) over the
    overlap levels with states; level k takes window i's value up to the middle
    of each overlap, mid = (lo_{i+1} + hi_i) div 2; then ln g(0) = ln 2 (the two
    ground states) and ln g(1) = -inf (no states)."""
    out = np.full(K + 1, np.nan)
    prev = np.asarray(pieces[0], dtype=np.float64)
    out[lo[0]:hi[0] + 1] = prev
    for i in range(1, len(lo)):
        cur = np.asarray(pieces[i], dtype=np.float64)
        ov = [k for k in wl_levels_with_states(lo[i], hi[i - 1])]
        if not ov:
            raise ValueError("windows %d and %d share no level with states" % (i - 1, i))
        s = 0.0
        for k in ov:
            s = s + (prev[k - lo[i - 1]] - cur[k - lo[i]])
        cur = cur + s / len(ov)
        mid = (lo[i] + hi[i - 1]) // 2
        out[mid + 1:hi[i] + 1] = cur[mid + 1 - lo[i]:]
        prev = cur
    out = out - out[0] + math.log(2.0)
    if K >= 1:
        out[1] = -np.inf
    return out


def wl_run(L, lo, hi, M, seed, lnf_final, flat=0.8, check=1, max_sweeps=1 << 30, max_pass=1000):
    """Wang-Landau sampling in windows: walkers driven into their windows;
    stage s of window i has ln f = 2^-s (f = e at s = 0); after every `check`
    sweeps of the active windows, a window whose walkers all have flat
    histograms averages their estimates (wl_average), clears the histograms
    and halves ln f, and stops once ln f < lnf_final.  Returns the windows'
    final pieces (averaged estimates in units of 1), the matched ln g, and per
    window the stages completed and the sweeps run."""
    lo, hi, wmax = _windows(lo, hi)
    nwin = lo.size
    N = L * L
    K = N // 2
    spins, E = win_drive(L, lo, hi, M, seed, max_pass)
    G = np.zeros((nwin * M, wmax), dtype=np.int64)
    H = np.zeros((nwin * M, wmax), dtype=np.uint32)
    stage = [0] * nwin
    active = [1] * nwin
    sweeps = [0] * nwin
    sweep = 0
    while any(active) and sweep < max_sweeps:
        inc = [WL_ONE >> stage[i] for i in range(nwin)]
        wl_sweeps(L, lo, hi, M, inc, active, seed, sweep, check, spins, E, G, H)
        sweep += check
        for i in range(nwin):
            if not active[i]:
                continue
            sweeps[i] += check
            if all(wl_flat(H[w], lo[i], hi[i], flat) for w in range(i * M, (i + 1) * M)):
                wl_average(G, lo, hi, M, i)
                H[i * M:(i + 1) * M] = 0
                stage[i] += 1
                if math.ldexp(1.0, -stage[i]) < lnf_final:
                    active[i] = 0
    pieces = []
    for i in range(nwin):
        if active[i]:
            wl_average(G, lo, hi, M, i)  # unfinished window: its current average
        n = hi[i] - lo[i] + 1
        pieces.append(G[i * M, :n].astype(np.float64) / float(WL_ONE))
    return dict(pieces=pieces, lng=wl_match(lo, hi, pieces, K), stages=stage, sweeps=sweeps,
                converged=[not a for a in active], spins=spins, E=E, G=G, H=H, sweep=sweep)


# ------------------------------------------------ multicanonical in windows
def muca_windows_run(L, lo, hi, M, seed, rec_sweeps, max_iter, flat=0.8, eq_sweeps=2, max_pass=1000):
    """The multicanonical recursion in windows (Sec. "Multicanonical
    simulations": the range split into windows simulated separately, a move
    out of the window rejected and the current state counted again, flat
    weights to start, the weight recursion, neighbouring pieces matched on
    their overlaps).  Walkers are driven into their windows; each window's
    weights are ln W = -G 2^-32 with G integer (start 0), held by all its
    walkers.  An iteration of a window still running: eq_sweeps unrecorded
    and rec_sweeps recorded multicanonical sweeps (wl_sweeps with ln f = 0),
    the walkers' counts added into H; the window stops once min H >= flat *
    max H over its levels with states, its piece being ln g = ln H + G 2^-32
    of that iteration; otherwise G += floor(ln H 2^32 + 1/2) where H > 0
    (ln W <- ln W - ln H), shifted to a minimum of 0.  Windows not flat after
    max_iter iterations give their last weights' -ln W = G 2^-32.  Returns the
    pieces, the matched ln g (wl_match), and per window the iterations run
    and whether it became flat."""
    lo, hi, wmax = _windows(lo, hi)
    nwin = lo.size
    K = L * L // 2
    spins, E = win_drive(L, lo, hi, M, seed, max_pass)
    G = np.zeros((nwin * M, wmax), dtype=np.int64)
    H = np.zeros((nwin * M, wmax), dtype=np.uint32)
    active = [1] * nwin
    iters = [0] * nwin
    pieces = [None] * nwin
    zero = [0] * nwin
    sweep = 0
    for _ in range(max_iter):
        if not any(active):
            break
        wl_sweeps(L, lo, hi, M, zero, active, seed, sweep, eq_sweeps, spins, E, G, H)
        sweep += eq_sweeps
        H[:] = 0
        wl_sweeps(L, lo, hi, M, zero, active, seed, sweep, rec_sweeps, spins, E, G, H)
        sweep += rec_sweeps
        for i in range(nwin):
            if not active[i]:
                continue
            iters[i] += 1
            n = hi[i] - lo[i] + 1
            Hw = [sum(int(v) for v in H[i * M:(i + 1) * M, j]) for j in range(n)]
            ks = [k - lo[i] for k in wl_levels_with_states(lo[i], hi[i])]
            g = G[i * M, :n]
            if float(min(Hw[j] for j in ks)) >= flat * float(max(Hw[j] for j in ks)):
                pieces[i] = np.array([math.log(float(Hw[j])) + float(g[j]) / float(WL_ONE) if Hw[j] > 0 else 0.0
                                      for j in range(n)])
                active[i] = 0
                continue
            new = g.copy()
            for j in range(n):
                if Hw[j] > 0:
                    new[j] += math.floor(math.log(float(Hw[j])) * float(WL_ONE) + 0.5)
            new -= min(int(new[j]) for j in ks)
            G[i * M:(i + 1) * M, :n] = new
    for i in range(nwin):
        if pieces[i] is None:
            # not flat: the last recursion's weights, -ln W = G 2^-32
            n = hi[i] - lo[i] + 1
            pieces[i] = G[i * M, :n].astype(np.float64) / float(WL_ONE)
    return dict(pieces=pieces, lng=wl_match(lo, hi, pieces, K), iterations=iters,
                converged=[not a for a in active], spins=spins, E=E, G=G, sweep=sweep)
