"""Exact reference values for the 2D/3D Ising model -- TEST INFRASTRUCTURE ONLY.

* ``enumerate_torus``: density of states g(E) (and the full energy / magnetisation
  table) by listing every state of a small periodic lattice.
* ``kaufman_lnZ`` / ``kaufman_u_cv``: Kaufman's exact partition function of the
  finite L x L torus (the "exact finite-lattice" values the paper's Ising
  application test compares against, Sec. "Random number generation").
* ``onsager_u`` / ``onsager_minus_beta_f`` / ``yang_m`` / ``BETA_C``: the
  infinite-lattice energy, free energy and spontaneous magnetisation.
* ``exact_g``: the exact integer density of states of the L x L torus from
  Kaufman's formula written as a polynomial in w = e^{4K}, evaluated modulo
  primes and interpolated (Chinese remainders join the residues).

Everything here uses Python integers, numpy integer arithmetic or mpmath at
high precision; nothing is shared with the product library.
"""
from __future__ import annotations

import functools
import math
import os

import mpmath as mp
import numpy as np

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0


# --------------------------------------------------------------------- enumeration
def _bonds(dims, shape):
    Lx, Ly = shape[0], shape[1]
    Lz = shape[2] if dims == 3 else 1
    out = []
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = x + Lx * (y + Ly * z)
                out.append((i, (x + 1) % Lx + Lx * (y + Ly * z)))
                out.append((i, x + Lx * ((y + 1) % Ly + Ly * z)))
                if dims == 3:
                    out.append((i, x + Lx * (y + Ly * ((z + 1) % Lz))))
    return out


def enumerate_states(dims, shape):
    """E and M for every state s (bit i of the state index set <=> s_i = -1)."""
    N = int(np.prod(shape))
    assert N <= 24
    idx = np.arange(1 << N, dtype=np.int64)
    spins = 1 - 2 * ((idx[:, None] >> np.arange(N)) & 1)
    E = np.zeros(1 << N, dtype=np.int64)
    for i, j in _bonds(dims, shape):
        E -= spins[:, i] * spins[:, j]
    M = spins.sum(axis=1)
    return E, M


def enumerate_torus(dims, shape):
    """g(E) as a dict {E: count}."""
    E, _ = enumerate_states(dims, shape)
    vals, counts = np.unique(E, return_counts=True)
    return {int(v): int(c) for v, c in zip(vals, counts)}


# ----------------------------------------------------------------------- Kaufman
def kaufman_lnZ(L, beta, dps=50):
    """ln Z of the L x L periodic ferromagnet (J = 1), L even, at inverse
    temperature beta (mpmath number at `dps` digits, or more if the caller's
    working precision is higher, as during numerical differentiation)."""
    with mp.workdps(max(dps, mp.mp.dps)):
        K = mp.mpf(beta)
        n = m = L
        c2, s2 = mp.cosh(2 * K), mp.sinh(2 * K)
        a = c2 * c2 / s2  # cosh 2K coth 2K

        def gamma(l):
            if l == 0:
                return 2 * K + mp.log(mp.tanh(K))
            return mp.acosh(a - mp.cos(mp.pi * l / n))

        Z1 = Z2 = Z3 = Z4 = mp.mpf(1)
        for r in range(n):
            g1, g0 = gamma(2 * r + 1), gamma(2 * r)
            Z1 *= 2 * mp.cosh(m * g1 / 2)
            Z2 *= 2 * mp.sinh(m * g1 / 2)
            Z3 *= 2 * mp.cosh(m * g0 / 2)
            Z4 *= 2 * mp.sinh(m * g0 / 2)
        N = L * L
        return mp.log(mp.mpf(1) / 2) + (mp.mpf(N) / 2) * mp.log(2 * s2) + mp.log(Z1 + Z2 + Z3 + Z4)


def kaufman_u_cv(L, beta, dps=50):
    """Energy per spin u = -d lnZ/d beta / N and specific heat per spin
    c_v = beta^2 d^2 lnZ / d beta^2 / N (exact derivatives by mpmath)."""
    with mp.workdps(dps):
        f = lambda b: kaufman_lnZ(L, b, dps=dps)
        N = L * L
        d1 = mp.diff(f, mp.mpf(beta), 1)
        d2 = mp.diff(f, mp.mpf(beta), 2)
        return float(-d1 / N), float(mp.mpf(beta) ** 2 * d2 / N)


# ---------------------------------------------------------------- infinite lattice
def onsager_u(beta):
    """Energy per spin of the infinite square lattice."""
    with mp.workdps(30):
        K = mp.mpf(beta)
        t = mp.tanh(2 * K)
        kappa = 2 * mp.sinh(2 * K) / mp.cosh(2 * K) ** 2
        K1 = mp.ellipk(kappa ** 2)  # mpmath takes the parameter m = kappa^2
        return float(-mp.coth(2 * K) * (1 + (2 / mp.pi) * (2 * t * t - 1) * K1))


def onsager_minus_beta_f(beta):
    """-beta f = ln 2 + (1/(8 pi^2)) double integral of
    ln[cosh^2 2K - sinh 2K (cos t1 + cos t2)] over [0, 2pi]^2."""
    with mp.workdps(25):
        K = mp.mpf(beta)
        c, s = mp.cosh(2 * K), mp.sinh(2 * K)
        f = lambda t1, t2: mp.log(c * c - s * (mp.cos(t1) + mp.cos(t2)))
        I = mp.quad(f, [0, mp.pi, 2 * mp.pi], [0, mp.pi, 2 * mp.pi])
        return float(mp.log(2) + I / (8 * mp.pi ** 2))


def yang_m(beta):
    """Spontaneous magnetisation (1 - sinh(2K)^-4)^(1/8) above beta_c, else 0."""
    if beta <= BETA_C:
        return 0.0
    return (1.0 - math.sinh(2.0 * beta) ** -4) ** 0.125


# ----------------------------------------------------------- exact density of states
def _is_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _primes_1_mod(m, count, start=(1 << 31) - 1):
    out = []
    p = start - (start % m) + 1
    if p > start:
        p -= m
    while len(out) < count:
        if _is_prime(p):
            out.append(p)
        p -= m
    return out


def _prime_factors(n):
    f, d = set(), 2
    while d * d <= n:
        while n % d == 0:
            f.add(d)
            n //= d
        d += 1
    if n > 1:
        f.add(n)
    return f


def _root_of_unity(order, p):
    qs = _prime_factors(order)
    for a in range(2, 1000):
        z = pow(a, (p - 1) // order, p)
        if all(pow(z, order // q, p) != 1 for q in qs):
            return z
    raise RuntimeError("no root of unity found")


def _vpow(base, e, p):
    """Elementwise base**e mod p (numpy int64, p < 2^31)."""
    base = np.asarray(base, dtype=np.int64) % p
    r = np.ones_like(base)
    while e:
        if e & 1:
            r = r * base % p
        base = base * base % p
        e >>= 1
    return r


def _vinv(x, p):
    return _vpow(x, p - 2, p)


def _cheb_T(n, c, p):
    """T_n(c) mod p elementwise via the pair (T_k, T_{k+1}) and doubling."""
    c = np.asarray(c, dtype=np.int64) % p
    t0, t1 = np.ones_like(c), c.copy()  # (T_0, T_1)
    for bit in bin(n)[2:]:
        if bit == "0":
            # (T_{2k}, T_{2k+1}) = (2 T_k^2 - 1, 2 T_k T_{k+1} - c)
            t0, t1 = (2 * t0 % p * t0 - 1) % p, (2 * t0 % p * t1 - c) % p
        else:
            # (T_{2k+1}, T_{2k+2}) = (2 T_k T_{k+1} - c, 2 T_{k+1}^2 - 1)
            t0, t1 = (2 * t0 % p * t1 - c) % p, (2 * t1 % p * t1 - 1) % p
    return t0


def _poly_values_mod(L, p):
    """P(w_i) = y_i^N Z(y_i) mod p at y_i = 2..N+2, where y = e^{2K}, w = y^2 and
    Z is Kaufman's partition function written rationally in y."""
    N = L * L
    zeta = _root_of_unity(2 * L, p)
    inv2 = (p + 1) // 2
    cosv = [(pow(zeta, l, p) + pow(zeta, 2 * L - l, p)) * inv2 % p for l in range(L + 1)]
    y = np.arange(2, N + 3, dtype=np.int64)
    yi = _vinv(y, p)
    ym = (y - yi) % p                         # y - 1/y = 2 sinh 2K
    yp = (y + yi) % p                         # y + 1/y = 2 cosh 2K
    a = yp * yp % p * _vinv(2 * ym % p, p) % p  # cosh 2K coth 2K
    Zodd_c = np.ones_like(y)
    Zodd_s = np.ones_like(y)
    Zev_c = np.ones_like(y)
    Zev_s = np.ones_like(y)
    for l in range(1, L):
        TL = _cheb_T(L, (a - cosv[l]) % p, p)
        plus, minus = (2 + 2 * TL) % p, (2 * TL - 2) % p
        if l % 2:
            Zodd_c = Zodd_c * plus % p
            Zodd_s = Zodd_s * minus % p
        else:
            Zev_c = Zev_c * plus % p
            Zev_s = Zev_s * minus % p
    e0 = y * (y - 1) % p * _vinv(y + 1, p) % p
    eL = y * (y + 1) % p * _vinv(y - 1, p) % p
    h = L // 2
    e0h, eLh = _vpow(e0, h, p), _vpow(eL, h, p)
    e0hi, eLhi = _vinv(e0h, p), _vinv(eLh, p)
    Z3 = (e0h + e0hi) % p * ((eLh + eLhi) % p) % p * Zev_c % p
    Z4 = (e0h - e0hi) % p * ((eLh - eLhi) % p) % p * Zev_s % p
    Zs = (Zodd_c + Zodd_s + Z3 + Z4) % p
    Z = inv2 * _vpow(ym, N // 2, p) % p * Zs % p
    return _vpow(y, N, p) * Z % p


def _interpolate_mod(L, vals, p):
    """Monomial coefficients of the degree-N polynomial through (w_i, vals_i),
    w_i = (i+2)^2, by Newton divided differences mod p."""
    N = L * L
    n = N + 1
    a = vals.astype(np.int64).copy()
    # w_i - w_{i-k} = k * (i + (i-k) + 4)
    invk = _vinv(np.arange(1, n, dtype=np.int64), p)
    invs = _vinv(np.arange(0, 2 * n + 4, dtype=np.int64), p)  # index 0 unused
    idx = np.arange(n, dtype=np.int64)
    for k in range(1, n):
        i = idx[k:]
        den = invk[k - 1] * invs[2 * i - k + 4] % p
        a[k:] = (a[k:] - a[k - 1:-1]) % p * den % p
    w = (idx + 2) ** 2 % p
    coef = np.zeros(n, dtype=np.int64)
    coef[0] = a[N]
    deg = 0
    for k in range(N - 1, -1, -1):
        # coef <- coef * (x - w_k) + a_k
        new = np.zeros(n, dtype=np.int64)
        new[1:deg + 2] = coef[:deg + 1]
        new[:deg + 1] = (new[:deg + 1] - coef[:deg + 1] * w[k]) % p
        new[0] = (new[0] + a[k]) % p
        coef = new % p
        deg += 1
    return coef


def _residue(Lp):
    L, p = Lp
    return _interpolate_mod(L, _poly_values_mod(L, p), p)


@functools.lru_cache(maxsize=None)
def exact_g(L, workers=1):
    """Exact integer g(E) of the L x L periodic ferromagnet, L even >= 4, as a
    list indexed by level k = (E + 2N)/4 = 0..N (Python ints).  The primes are
    independent: workers > 1 spreads them over that many processes."""
    assert L % 2 == 0 and L >= 4
    N = L * L
    nprimes = (N + 2) // 30 + 2
    primes = _primes_1_mod(2 * L, nprimes)
    if workers > 1:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(workers) as pool:
            residues = pool.map(_residue, [(L, p) for p in primes], chunksize=1)
    else:
        residues = [_residue((L, p)) for p in primes]
    # Garner's mixed-radix reconstruction, vectorised over the coefficients
    digits = []
    for i, p in enumerate(primes):
        x = residues[i] % p
        for jdx in range(i):
            q = primes[jdx]
            x = (x - digits[jdx]) % p * pow(q, p - 2, p) % p
        digits.append(x)
    g = []
    for c in range(N + 1):
        v = 0
        for i in range(len(primes) - 1, -1, -1):
            v = v * primes[i] + int(digits[i][c])
        g.append(v)
    # coefficient of w^j is g(E = 2N - 4j); reorder to level k = (E + 2N)/4 = N - j
    return g[::-1]


def big_log(v):
    """Natural log of a positive Python integer to double precision."""
    b = v.bit_length()
    if b <= 60:
        return math.log(v)
    s = b - 60
    return math.log(v >> s) + s * math.log(2.0)


def exact_lng(L, cache_dir=None):
    """ln g by level k = 0..N (-inf where g = 0), cached as a text file."""
    if cache_dir is not None:
        path = os.path.join(cache_dir, "lng_L%d.txt" % L)
        if os.path.exists(path):
            return np.loadtxt(path)
    g = exact_g(L)
    out = np.array([big_log(v) if v > 0 else -np.inf for v in g])
    if cache_dir is not None:
        np.savetxt(path, out, fmt="%.17g")
    return out
