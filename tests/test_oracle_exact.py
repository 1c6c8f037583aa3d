"""Pins of the exact references, each against an independent method.

* brute-force enumeration of every state of 3x3, 4x4 and 2x2x4 lattices;
* exact g(E) from Kaufman's formula (modular evaluation + interpolation)
  against enumeration (L = 4) and an integer row-transfer-matrix count (L = 6),
  plus the invariants sum g = 2^N, g(E) = g(-E), g(-2N) = 2, g(-2N+8) = 2N and
  the only empty levels k = 1 and k = N-1;
* Kaufman ln Z against the enumeration sum and against exact g(E);
* Onsager u(beta_c) = -sqrt(2), Onsager u against Kaufman at L = 64 off
  criticality, -beta f against Kaufman ln Z / N, Yang's m limits.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import exact


def test_enumeration_small_tori():
    g3 = exact.enumerate_torus(2, (3, 3))
    assert sum(g3.values()) == 512
    g4 = exact.enumerate_torus(2, (4, 4))
    assert sum(g4.values()) == 65536
    assert all(g4[e] == g4[-e] for e in g4)
    assert g4[-32] == 2 and g4[-24] == 32  # ground states; one flipped spin: 2N
    g3d = exact.enumerate_torus(3, (2, 2, 4))
    assert sum(g3d.values()) == 65536
    # 2x2x4: every site has 6 bonds counted with multiplicity (doubled bonds
    # in the size-2 directions), 3N bonds in total
    assert min(g3d) == -3 * 16 and g3d[-48] == 2


def _transfer_matrix_g(L):
    """g(E) of the L x L torus by a row-to-row transfer count (all partial
    counts stay below 2^53, so float64 BLAS arithmetic is exact here)."""
    n = 1 << L
    rows = 1 - 2 * ((np.arange(n)[:, None] >> np.arange(L)) & 1)
    e_row = -(rows * np.roll(rows, -1, axis=1)).sum(axis=1)
    e_int = -(rows @ rows.T)
    dE = e_row[None, :] + e_int  # entering row b after row a: bonds inside b and between a and b
    N = L * L
    off, nE = 2 * N, 4 * N + 1
    vals = np.unique(dE)
    masks = {v: (dE == v).astype(np.float64) for v in vals}
    # cnt[b, a0, e]: paths that started at row a0, now at row b, energy e - off
    cnt = np.zeros((n, n, nE))
    cnt[np.arange(n), np.arange(n), off] = 1.0
    for _ in range(L - 1):
        new = np.zeros_like(cnt)
        for v in vals:
            moved = (masks[v].T @ cnt.reshape(n, -1)).reshape(cnt.shape)
            new += np.roll(moved, v, axis=2)
        cnt = new
    total = np.zeros(nE)
    for v in vals:
        # close the torus: the last row is followed by the start row a0
        w = masks[v]  # w[b, a0]
        contrib = np.einsum("ba,bae->e", w, cnt)
        total += np.roll(contrib, v)
    assert total.max() < 2.0 ** 53
    return {e - off: int(round(c)) for e, c in enumerate(total) if c}


def _as_levels(gdict, N):
    out = [0] * (N + 1)
    for e, c in gdict.items():
        out[(e + 2 * N) // 4] = c
    return out


def test_exact_g_vs_enumeration_L4():
    assert exact.exact_g(4) == _as_levels(exact.enumerate_torus(2, (4, 4)), 16)


def test_exact_g_vs_transfer_matrix_L6():
    assert exact.exact_g(6) == _as_levels(_transfer_matrix_g(6), 36)


@pytest.mark.parametrize("L", [8, 12, 16])
def test_exact_g_invariants(L):
    N = L * L
    g = exact.exact_g(L)
    assert sum(g) == 2 ** N
    assert g == g[::-1]
    assert g[0] == 2 and g[2] == 2 * N
    empty = [k for k, v in enumerate(g) if v == 0]
    assert empty == [1, N - 1]


def test_kaufman_vs_enumeration_and_exact_g():
    g4 = exact.enumerate_torus(2, (4, 4))
    for beta in (0.1, 0.3, exact.BETA_C, 0.7):
        lnZ = float(mp.log(mp.fsum(c * mp.exp(-beta * e) for e, c in g4.items())))
        assert abs(float(exact.kaufman_lnZ(4, beta)) - lnZ) < 1e-12
    g16 = exact.exact_g(16)
    for beta in (0.2, exact.BETA_C, 0.6):
        with mp.workdps(60):
            Z = mp.fsum(mp.mpf(c) * mp.exp(-mp.mpf(beta) * (4 * k - 512)) for k, c in enumerate(g16) if c)
            assert abs(mp.log(Z) - exact.kaufman_lnZ(16, beta, dps=60)) < mp.mpf(10) ** -40


def test_onsager_and_yang():
    assert abs(exact.onsager_u(exact.BETA_C + 1e-12) + math.sqrt(2.0)) < 1e-6
    for beta in (0.3, 0.4, 0.55):
        u64, _ = exact.kaufman_u_cv(64, beta, dps=30)
        assert abs(u64 - exact.onsager_u(beta)) < 1e-5  # finite-size shift ~4e-6 at beta = 0.4
    lnZ64 = float(exact.kaufman_lnZ(64, 0.3)) / 4096
    assert abs(lnZ64 - exact.onsager_minus_beta_f(0.3)) < 1e-6
    assert exact.yang_m(exact.BETA_C * 0.999) == 0.0
    assert 0.0 < exact.yang_m(exact.BETA_C * 1.0001) < 0.5
    assert abs(exact.yang_m(5.0) - 1.0) < 1e-12
