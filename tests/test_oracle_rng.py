"""Pins of the oracle's random streams (Philox4x32-10, Sec. "Random number
generation", counter-based generators).

* Known answers: the oracle's Philox block equals rocRAND's host-side
  Philox4x32-10 engine (an independent implementation shipped with ROCm, built
  here from its header) for edge and random (key, counter) values.
* The draws follow the documented counter layout (key = seed words; counter =
  index, replica, sweep low word, tag << 24 | colour << 23 | sweep >> 32) and
  the documented bit-plane gather of a block's byte.
* The 32-bit draws assembled from two blocks are uniform (chi-square on the top
  byte and on the low bits), distinct streams are uncorrelated, and the 53-bit
  resampling variate lies in [0, 1).
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_blocks(cases):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "kat")
        subprocess.run([hipcc, "-O1", "-I/opt/rocm/include", os.path.join(HERE, "philox_rocrand_kat.cpp"),
                        "-o", exe], check=True, capture_output=True)
        inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [list(map(int, line.split())) for line in out.strip().splitlines()]


def test_philox_matches_rocrand():
    rng = np.random.default_rng(2024)
    # rocRAND reaches counter word x1 through a 64-bit offset of 4 (x0 + 2^32 x1)
    # numbers, so its mapping covers x1 < 2^30; x1 stays in that range here.
    top = 0xFFFFFFFF
    cases = [(0, 0, 0, 0, 0, 0), (top, top, top, 0x3FFFFFFF, top, top), (1, 0, 0, 0, 0, 0),
             (0, 0, 1, 0, 0, 0), (0, 0, 0, 0, 0, 0x80000000), (7, 0, 123456, 3, 9999, (2 << 24) | (1 << 23))]
    for _ in range(24):
        v = [int(x) for x in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)]
        v[3] >>= 2
        cases.append(tuple(v))
    ref = _rocrand_blocks(cases)
    for c, r in zip(cases, ref):
        got = oracle.philox([c[2], c[3], c[4], c[5]], [c[0], c[1]])
        assert [int(v) for v in got] == r, c


def test_philox_counter_sensitivity():
    # every counter word and key word changes every output word (avalanche)
    base = oracle.philox([1, 2, 3, 4], [5, 6])
    for pos in range(6):
        ctr, key = [1, 2, 3, 4], [5, 6]
        if pos < 4:
            ctr[pos] ^= 1
        else:
            key[pos - 4] ^= 1
        other = oracle.philox(ctr, key)
        assert np.all(other != base)


def _chi2(counts, expected):
    return float(((counts - expected) ** 2 / expected).sum())


def test_draw32_uniform_bytes_and_bits():
    n = 40000
    r = np.array([oracle.draw32(99, oracle.TAG_SWEEP, oracle.TAG_SWEEP_LO, j, 3, 17, 1) for j in range(n)],
                 dtype=np.uint64)
    top = np.bincount((r >> 24).astype(np.int64), minlength=256)
    # 255 dof: mean 255, sd ~22.6; 6 sd bound
    assert _chi2(top, n / 256) < 255 + 6 * 22.6
    low = np.bincount((r & 0xFF).astype(np.int64), minlength=256)
    assert _chi2(low, n / 256) < 255 + 6 * 22.6
    bits = np.array([((r >> b) & 1).mean() for b in range(32)])
    assert np.all(np.abs(bits - 0.5) < 6 * 0.5 / np.sqrt(n))


def test_draw_streams_distinct():
    # neighbouring replicas / sweeps / phases / tags give unrelated streams
    ref = np.array([oracle.draw32(5, 2, 7, j, 0, 0, 0) for j in range(2000)], dtype=np.float64)
    for args in [(5, 2, 7, None, 1, 0, 0), (5, 2, 7, None, 0, 1, 0), (5, 2, 7, None, 0, 0, 1),
                 (6, 2, 7, None, 0, 0, 0), (5, 5, 8, None, 0, 0, 0), (5, 2, 7, None, 0, 1 << 32, 0)]:
        other = np.array([oracle.draw32(args[0], args[1], args[2], j, args[4], args[5], args[6])
                          for j in range(2000)], dtype=np.float64)
        assert np.mean(ref == other) < 0.01
        c = np.corrcoef(ref, other)[0, 1]
        assert abs(c) < 6 / np.sqrt(2000)


def test_draw_byte_is_top_byte_of_draw32():
    for j in range(300):
        b = oracle.draw_byte(11, oracle.TAG_SWEEP, j, 4, 8, 1)
        r = oracle.draw32(11, oracle.TAG_SWEEP, oracle.TAG_SWEEP_LO, j, 4, 8, 1)
        assert r >> 24 == b


def test_resample_u_range_and_mean():
    u = np.array([oracle.resample_u(17, k, 2, 33) for k in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 6 * np.sqrt(1 / 12 / u.size)
    # 53-bit grid
    assert np.all(u * 2.0 ** 53 == np.floor(u * 2.0 ** 53))


def _gather_byte(block, p):
    # the documented "byte p of a block": bit k is bit p of 16-bit half-word k,
    # half-word k being bits 16 (k mod 2) .. +15 of word k / 2
    return sum(((int(block[k >> 1]) >> (16 * (k & 1) + p)) & 1) << k for k in range(8))


@pytest.mark.parametrize("seed,tag,replica,sweep,phase", [(11, oracle.TAG_SWEEP, 4, 8, 1),
                                                          ((7 << 40) | 123, oracle.TAG_SWEEP, 65, (1 << 33) + 5, 0),
                                                          (3, oracle.TAG_INIT, 9, 0, 0)])
def test_draws_follow_the_documented_counter_layout(seed, tag, replica, sweep, phase):
    # key = (seed low word, seed high word); counter = (index, replica, sweep low
    # word, tag << 24 | phase << 23 | sweep >> 32); the top byte is the gathered
    # byte of block j / 16, the low 24 bits word 0 of block j under TAG_SWEEP_LO
    key = [seed & 0xFFFFFFFF, seed >> 32]
    w3 = lambda t: (t << 24) | (phase << 23) | ((sweep >> 32) & 0x7FFFFF)
    for j in list(range(40)) + [1000, 65535, 1 << 20]:
        blk = oracle.philox([j >> 4, replica, sweep & 0xFFFFFFFF, w3(tag)], key)
        assert oracle.draw_byte(seed, tag, j, replica, sweep, phase) == _gather_byte(blk, j & 15)
        if tag == oracle.TAG_SWEEP:
            lo = oracle.philox([j, replica, sweep & 0xFFFFFFFF, w3(oracle.TAG_SWEEP_LO)], key)
            r = oracle.draw32(seed, tag, oracle.TAG_SWEEP_LO, j, replica, sweep, phase)
            assert r == (_gather_byte(blk, j & 15) << 24) | (int(lo[0]) & 0xFFFFFF)


@pytest.mark.parametrize("seed,pop,step", [(17, 2, 33), ((5 << 36) | 9, 0, 1), (1, 7, 200)])
def test_resample_u_follows_the_documented_construction(seed, pop, step):
    # u_k = ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53, w = Philox(ctr = (k, pop, step,
    # TAG_RESAMPLE << 24)) under key (seed low word, seed high word)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in list(range(50)) + [4095, 65535]:
        w = oracle.philox([k, pop, step, oracle.TAG_RESAMPLE << 24], key)
        want = ((int(w[0]) >> 5) * 2 ** 26 + (int(w[1]) >> 6)) / 2.0 ** 53
        assert oracle.resample_u(seed, k, pop, step) == want


@pytest.mark.parametrize("seed,replica,sweep", [(99, 2, 7), ((3 << 33) | 1, 4095, (1 << 32) + 3)])
def test_draw_word_follows_the_documented_construction(seed, replica, sweep):
    # item j of a sequential chain: word (j mod 4) of Philox(ctr = (j div 4,
    # replica, sweep low word, tag << 24 | sweep >> 32))
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for j in list(range(20)) + [16383]:
        w = oracle.philox([j >> 2, replica, sweep & 0xFFFFFFFF, (oracle.TAG_MUCA << 24) | (sweep >> 32)], key)
        assert oracle.draw_word(seed, oracle.TAG_MUCA, j, replica, sweep) == int(w[j & 3])


def test_weyl_increments_follow_their_definition_in_both_sources():
    """Philox's key increments are the leading 32 fraction bits of the golden
    ratio and of sqrt(3): floor(2^32 (phi - 1)) and floor(2^32 (sqrt 3 - 1)),
    computed here with exact integer square roots.  The oracle and the GPU
    library each write them down independently; both must match."""
    import math
    import re

    w0 = (math.isqrt(5 << 64) - (1 << 32)) // 2  # 2^32 (sqrt 5 - 1) / 2, floored
    w1 = math.isqrt(3 << 64) - (1 << 32)
    root = os.path.dirname(HERE)
    orc = open(os.path.join(root, "oracle", "mcoracle.c")).read()
    lib = open(os.path.join(root, "paper_1709_04394_amd", "csrc", "common.hpp")).read()
    got_orc = [int(re.search(r"#define ORC_PHILOX_%s (0x[0-9A-Fa-f]+)u" % n, orc).group(1), 16) for n in ("W0", "W1")]
    got_lib = [int(re.search(r"kPhilox%s = (0x[0-9A-Fa-f]+)u" % n, lib).group(1), 16) for n in ("W0", "W1")]
    assert got_orc == [w0, w1] and got_lib == [w0, w1]


@pytest.mark.parametrize("realisation", [0, 1, 63, 4095])
def test_couplings_of_a_realisation_follow_the_documented_counter_layout(realisation):
    # bond b = d N + i of realisation k is +1 iff the gathered byte (b mod 16)
    # of Philox(ctr = (b / 16, k, 0, TAG_COUPLING << 24)) is below 128
    dims, L, seed = 3, 4, (1 << 35) | 13
    J = oracle.couplings(dims, L, seed, realisation)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for b in range(J.size):
        blk = oracle.philox([b >> 4, realisation, 0, oracle.TAG_COUPLING << 24], key)
        assert J[b] == (1 if _gather_byte(blk, b & 15) < 128 else -1), b


def test_couplings_of_different_realisations_are_independent_fair_coins():
    # 64 realisations of a 16^3 lattice: +1 with p = 1/2, and two realisations
    # agree on a bond with p = 1/2 (binomial 5 sigma bounds)
    Js = np.stack([oracle.couplings(3, 16, 13, k) for k in range(64)]).astype(np.float64)
    n = Js.size
    assert abs((Js > 0).mean() - 0.5) < 5 * 0.5 / np.sqrt(n)
    agree = (Js[1:] == Js[:-1]).mean()
    assert abs(agree - 0.5) < 5 * 0.5 / np.sqrt(Js[1:].size)
    assert np.array_equal(Js[0], oracle.couplings(3, 16, 13).astype(np.float64))
