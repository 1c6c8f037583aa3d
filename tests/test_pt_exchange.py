"""Parallel tempering's exchange step in libmcspin (mc_pt_exchange, host only,
no GPU needed) against the oracle, bit for bit: the two maps and the
acceptance counts after every round of long random trajectories (several
numbers of temperatures, round numbers crossing 2^32, 64-bit seeds), and the
documented errors, which leave every argument unchanged."""
import ctypes

import numpy as np
import pytest

import oracle

mcs = pytest.importorskip("paper_1709_04394_amd")


@pytest.fixture(scope="module")
def ctx():
    return mcs.Context(0)  # host state only


@pytest.mark.parametrize("nT,round0,seed,N", [(2, 0, 5, 256), (3, (1 << 32) - 7, (9 << 40) | 3, 1024),
                                              (17, 12345, 77, 4096), (64, 1 << 40, 1, 16384)])
def test_matches_oracle_round_by_round(ctx, nT, round0, seed, N):
    rng = np.random.default_rng(nT)
    beta = np.sort(rng.uniform(0.1, 0.8, size=nT))
    assert np.all(np.diff(beta) > 0)
    t_lib, r_lib = np.arange(nT, dtype=np.int32), np.arange(nT, dtype=np.int32)
    a_lib = np.zeros(nT - 1, dtype=np.int64)
    t_orc, r_orc, a_orc = list(range(nT)), list(range(nT)), [0] * (nT - 1)
    for rnd in range(round0, round0 + 1500):
        # energies of a lattice of N sites, multiples of 4, spread so that both
        # outcomes occur often
        E = (4 * rng.integers(-N // 8, 1, size=nT)).astype(np.int64)
        ctx.pt_exchange(beta, E, t_lib, r_lib, seed, rnd, a_lib)
        oracle.pt_exchange(list(beta), E, t_orc, r_orc, seed, rnd, a_orc)
        assert list(r_lib) == r_orc and list(t_lib) == t_orc and list(a_lib) == a_orc, rnd
    assert 0 < a_lib.sum() < 1500 * (nT // 2 + 1)  # both outcomes happened


def _call(ctx, n, beta, E, t, r, rnd=0, acc=None):
    acc = np.zeros(max(n - 1, 1), dtype=np.int64) if acc is None else acc
    p = lambda a, ty: None if a is None else a.ctypes.data_as(ctypes.POINTER(ty))
    return mcs._lib.mc_pt_exchange(ctx._h, n, p(beta, ctypes.c_double), p(E, ctypes.c_int64),
                                   p(t, ctypes.c_int32), p(r, ctypes.c_int32), 1, rnd, p(acc, ctypes.c_int64))


def test_errors_change_nothing(ctx):
    beta = np.array([0.1, 0.2, 0.3])
    E = np.array([-8, 0, 4], dtype=np.int64)
    ident = lambda: np.arange(3, dtype=np.int32)
    cases = [
        (1, beta, E, ident(), ident(), 0, mcs.MC_E_RANGE),                           # one temperature
        (3, np.array([0.1, 0.1, 0.3]), E, ident(), ident(), 0, mcs.MC_E_RANGE),     # not strictly increasing
        (3, np.array([0.1, np.nan, 0.3]), E, ident(), ident(), 0, mcs.MC_E_RANGE),
        (3, np.array([-0.1, 0.2, 0.3]), E, ident(), ident(), 0, mcs.MC_E_RANGE),
        (3, beta, np.array([0, 1 << 53, 0], dtype=np.int64), ident(), ident(), 0, mcs.MC_E_RANGE),
        (3, beta, E, ident(), ident(), 1 << 55, mcs.MC_E_RANGE),
        (3, beta, E, np.array([0, 2, 1], dtype=np.int32), ident(), 0, mcs.MC_E_INVAL),  # not inverse
        (3, beta, E, np.array([0, 0, 1], dtype=np.int32), np.array([0, 0, 1], dtype=np.int32), 0, mcs.MC_E_INVAL),
        (3, beta, E, ident(), np.array([0, 1, 3], dtype=np.int32), 0, mcs.MC_E_INVAL),
        (3, beta, None, ident(), ident(), 0, mcs.MC_E_INVAL),
    ]
    for n, b, e, t, r, rnd, code in cases:
        t0, r0 = t.copy(), r.copy()
        acc = np.zeros(2, dtype=np.int64)
        assert _call(ctx, n, b, e, t, r, rnd, acc) == code, (n, b, e, t, r, rnd)
        assert np.array_equal(t, t0) and np.array_equal(r, r0) and not acc.any()
    assert mcs._lib.mc_pt_exchange(None, 3, None, None, None, None, 0, 0, None) == mcs.MC_E_INVAL


def test_binding_checks_types(ctx):
    with pytest.raises(TypeError):
        ctx.pt_exchange([0.1, 0.2], [0, 0], [0, 1], np.arange(2, dtype=np.int32), 1, 0, np.zeros(1, np.int64))
    with pytest.raises(ValueError):
        ctx.pt_exchange([0.1, 0.2], [0, 0], np.arange(2, dtype=np.int32), np.arange(2, dtype=np.int32), 1, 0,
                        np.zeros(2, np.int64))


def _pt_args(L=16, beta=(0.3, 0.4, 0.5), n_sets=2, theta=2, rounds=5, round0=0):
    b = np.ascontiguousarray(beta, dtype=np.float64)
    a = mcs.PTArgs(L, b.size, n_sets, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), theta, 7, round0, rounds)
    return a, b


def test_pt_run_workspace_and_argument_errors(ctx):
    """mc_pt_run checks everything before any device work (no GPU needed):
    the workspace formula, extents, counts, temperatures and maps."""
    a, keep = _pt_args()
    nb = mcs._lib.mc_pt_workspace_bytes(ctypes.byref(a))
    # thresholds, exchange table (2 pairs x (N + 1) entries), maps, energies,
    # counts and the recorded energies, each rounded up to 256 B
    up = lambda b: (b + 255) // 256 * 256
    count, N = 6, 256
    assert nb == up(3 * 2 * 8) + up(2 * (N + 1) * 8) + 3 * up(count * 4) + up(2 * 2 * 8) + up(5 * count * 8)
    t = np.tile(np.arange(3, dtype=np.int32), (2, 1))
    r, acc = t.copy(), np.zeros((2, 2), dtype=np.int64)
    p = lambda x, ty: x.ctypes.data_as(ctypes.POINTER(ty))
    fake = ctypes.c_void_p(1)

    def call(args, tt=t, rr=r, ws=fake, wsb=nb):
        return mcs._lib.mc_pt_run(ctx._h, ctypes.byref(args), fake, p(tt, ctypes.c_int32), p(rr, ctypes.c_int32),
                                  p(acc, ctypes.c_int64), None, ws, wsb, None)

    assert call(_pt_args(L=12)[0]) == mcs.MC_E_SHAPE
    assert call(_pt_args(beta=(0.3,))[0]) == mcs.MC_E_RANGE
    assert call(_pt_args(beta=(0.3, 0.3, 0.5))[0]) == mcs.MC_E_RANGE
    assert call(_pt_args(beta=(0.3, float("nan"), 0.5))[0]) == mcs.MC_E_RANGE
    assert call(_pt_args(theta=0)[0]) == mcs.MC_E_RANGE
    assert call(_pt_args(n_sets=0)[0]) == mcs.MC_E_RANGE
    assert call(_pt_args(n_sets=30000)[0]) == mcs.MC_E_RANGE
    bad = t.copy()
    bad[1] = [0, 2, 1]  # temp_of of set 1 no longer inverse to replica_at
    assert call(a, tt=bad) == mcs.MC_E_INVAL
    assert call(a, wsb=nb - 1) == mcs.MC_E_WORKSPACE
    assert call(a, ws=None) == mcs.MC_E_WORKSPACE
    assert np.array_equal(t, np.tile(np.arange(3), (2, 1))) and not acc.any()  # nothing changed
