"""Mutation check of the oracle's pins -- TEST INFRASTRUCTURE, run by hand
(pytest does not collect it):

    python tests/mutate_oracle.py [--jobs N] [--only NAME ...]

Each mutant plants one plausible mistake in a temporary copy of the oracle
(oracle/mcoracle.c, oracle/mlp.py or oracle/__init__.py): a dropped term, a
wrong sign, index, constant or bit order, a changed update order or stream
number.  The copy is built and the CPU pin tests (tests/test_oracle_*.py but
the sanitizer run, and tests/test_golden_lng.py) run against it; the mutant
is caught when any of them fails.  The working tree is never modified.  One
line per mutant is printed, then the count caught.
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text (must occur once), replacement[, file; default oracle/mcoracle.c])
MUTANTS = [
    # Philox4x32-10 (Sec. "Random number generation")
    ("philox: key dropped from a round", "uint32_t y0 = hi1 ^ x1 ^ k0;", "uint32_t y0 = hi1 ^ x1;"),
    ("philox: wrong key word in a round", "uint32_t y2 = hi0 ^ x3 ^ k1;", "uint32_t y2 = hi0 ^ x3 ^ k0;"),
    ("philox: wrong Weyl increment", "k1 += ORC_PHILOX_W1;", "k1 += ORC_PHILOX_W0;"),
    ("philox: nine rounds", "for (int round = 0; round < 10; ++round)", "for (int round = 0; round < 9; ++round)"),
    # stream layout
    ("stream: colour bit moved", "((phase & 1u) << 23)", "((phase & 1u) << 22)"),
    ("stream: byte bit order reversed", "byte |= ((halfword >> pos) & 1u) << k;",
     "byte |= ((halfword >> pos) & 1u) << (7u - k);"),
    ("stream: low bits from word 1", "return (top << 24) | (out[0] & 0xFFFFFFu);",
     "return (top << 24) | (out[1] & 0xFFFFFFu);"),
    ("stream: resample u takes 27 + 27 bits", "uint64_t a = out[0] >> 5, b = out[1] >> 6;",
     "uint64_t a = out[0] >> 5, b = out[1] >> 5;"),
    # acceptance tables (Eq. metropolis-canonical, Eq. heatbath)
    ("tables: Metropolis dE = 2k", "double p = exp(-beta * (double)(4 * k));",
     "double p = exp(-beta * (double)(2 * k));"),
    ("tables: Metropolis floor", "        T[k] = (uint64_t)ceil(ldexp(p, 32));",
     "        T[k] = (uint64_t)floor(ldexp(p, 32));"),
    ("tables: heat-bath field not doubled", "double e = exp(-2.0 * beta * (double)h);",
     "double e = exp(-beta * (double)h);"),
    # geometry, couplings, measurement (Eq. ising_model)
    ("field: left bond takes the site's coupling", "b[1] = 0 * g->N + n[1];", "b[1] = 0 * g->N + i;"),
    ("field: down-z bond takes the site's coupling", "b[5] = 2 * g->N + n[5];", "b[5] = 2 * g->N + i;"),
    ("field: y wrap to 1", "int yp = y + 1 == g->Ly ? 0 : y + 1", "int yp = y + 1 == g->Ly ? 1 : y + 1"),
    ("measure: energy sign", "e -= (int64_t)(J ? J[d * g.N + i] : 1) * s[i] * s[nb[d]];",
     "e += (int64_t)(J ? J[d * g.N + i] : 1) * s[i] * s[nb[d]];"),
    ("measure: z bond to the wrong neighbour", "site(&g, x, y, z + 1 == g.Lz ? 0 : z + 1)",
     "site(&g, x, y + 1 == g.Ly ? 0 : y + 1, z)"),
    ("init: hot start threshold 64", "(uint32_t)i, replica, 0, 0) < 128u ? 1 : -1;",
     "(uint32_t)i, replica, 0, 0) < 64u ? 1 : -1;"),
    # checkerboard sweep (Sec. "Checkerboard scheme")
    ("sweep: heat-bath sign swapped", "s[i] = (uint64_t)r < Thb[h + z_coord] ? 1 : -1;",
     "s[i] = (uint64_t)r < Thb[h + z_coord] ? -1 : 1;"),
    ("sweep: Metropolis index dE/2", "if (dE <= 0 || (uint64_t)r < Tm[dE / 4]) s[i] = (int8_t)-s[i];\n                        } else",
     "if (dE <= 0 || (uint64_t)r < Tm[dE / 8]) s[i] = (int8_t)-s[i];\n                        } else"),
    ("sweep: draw index i instead of i >> 1", "(uint32_t)(i >> 1), replica, sweep, (uint32_t)c);",
     "(uint32_t)i, replica, sweep, (uint32_t)c);"),
    ("sweep: odd sub-lattice first", "if (((x + y + z) & 1) != c) continue;", "if (((x + y + z + 1) & 1) != c) continue;"),
    ("sweep: colour bit not passed", "(uint32_t)(i >> 1), replica, sweep, (uint32_t)c);",
     "(uint32_t)(i >> 1), replica, sweep, 0u);"),
    # population annealing (Sec. "Population annealing", Eq. Q)
    ("pa: ln Q shift sign", "lnQ[s] = log(ct / (double)R) + dbeta * (double)(2 * N);",
     "lnQ[s] = log(ct / (double)R) - dbeta * (double)(2 * N);"),
    ("pa: weight level off by one", "w[j] = wtab[(E[j] + 2 * N) / 4];", "w[j] = wtab[(E[j] + 2 * N) / 4 + 1];"),
    ("pa: weights of the new beta only", "double dbeta = beta[i] - beta[i - 1];", "double dbeta = beta[i];"),
    ("pa: placement offset", "P[j] = P[j - 1] + n[j - 1];", "P[j] = P[j - 1] + n[j];"),
    ("pa: sweep numbers from i theta", "(uint64_t)(i - 1) * (uint64_t)theta, theta, NULL);",
     "(uint64_t)i * (uint64_t)theta, theta, NULL);"),
    ("pa: replica id without the population", "(uint32_t)((int64_t)pop * R + k), (uint64_t)(i - 1)",
     "(uint32_t)k, (uint64_t)(i - 1)"),
    ("pa: sweeps at the previous beta", "orc_sweep(2, L, L, 1, spins + k * N, NULL, 0, beta[i], seed,",
     "orc_sweep(2, L, L, 1, spins + k * N, NULL, 0, beta[i - 1], seed,"),
    ("scan: group prefix from the wrong element", "G[q] = G[q - 1] + t[64 * (q - 1) + 63];",
     "G[q] = G[q - 1] + t[64 * (q - 1) + 62];"),
    ("scan: in-place doubling", "for (int i = d; i < 64; ++i) v[i] = tmp[i] + tmp[i - d];",
     "for (int i = d; i < 64; ++i) v[i] = tmp[i] + v[i - d];"),
    # multicanonical walkers (Sec. "Multicanonical simulations", Eq. muca)
    ("muca: ratio inverted", "double x = lnW[k2] - lnW[k];", "double x = lnW[k] - lnW[k2];"),
    ("muca: window excludes E = 0", "if (e2 <= 0) {", "if (e2 < 0) {"),
    ("muca: wrong table column", "int col = d < 0 ? d + 2 : d + 1;", "int col = d < 0 ? d + 2 : d;"),
    ("muca: rejected moves not counted", "if (record) hw[(e + 2 * N) / 4] += 1;",
     "if (record && e == e2) hw[(e + 2 * N) / 4] += 1;"),
    ("muca: walkers share one stream",
     "if (e2 <= 0) {\n                        uint32_t r = orc_draw_word(seed, ORC_TAG_MUCA, (uint32_t)i, (uint32_t)w, sweep);",
     "if (e2 <= 0) {\n                        uint32_t r = orc_draw_word(seed, ORC_TAG_MUCA, (uint32_t)i, 0u, sweep);"),
    ("wl: walkers share one stream",
     "                            uint32_t r = orc_draw_word(seed, ORC_TAG_MUCA, (uint32_t)i, (uint32_t)w, sweep);",
     "                            uint32_t r = orc_draw_word(seed, ORC_TAG_MUCA, (uint32_t)i, 0u, sweep);"),
    ("muca: stratified rounding", "int64_t b = (int64_t)65536 * (2 * (int64_t)W - 2 * (int64_t)w - 1);",
     "int64_t b = (int64_t)65536 * (2 * (int64_t)W - 2 * (int64_t)w + 1);"),
    ("muca: start threshold off by one", "(uint32_t)w, 0, 0) >= 256u - c ? -1 : 1;",
     "(uint32_t)w, 0, 0) > 256u - c ? -1 : 1;"),
    ("muca: settle keeps E above the window", "            e = -e;\n", "            e = e;\n"),
    # the FP64 network (oracle/mlp.py)
    ("mlp: second layer linear (forward and backward)",
     "    h2 = np.tanh(z2)\n", "    h2 = z2\n", "oracle/mlp.py"),
    ("mlp: first-layer gradient without tanh'", 'dz1 = (dz2 @ q["W2"]) * (1.0 - h1 * h1)',
     'dz1 = (dz2 @ q["W2"])', "oracle/mlp.py"),
    ("mlp: Adam without bias correction", "mh = m / (1.0 - beta1 ** t)", "mh = m", "oracle/mlp.py"),
    ("mlp: Xavier bound sqrt(3 / fan)", "a = math.sqrt(6.0 / (fan_in + fan_out))",
     "a = math.sqrt(3.0 / (fan_in + fan_out))", "oracle/mlp.py"),
    # parallel tempering (oracle/__init__.py, Sec. "Parallel Tempering", Eq. pt)
    ("pt: exponent sign", "x = (beta[i] - beta[i + 1]) * float(E[a] - E[b])",
     "x = (beta[i + 1] - beta[i]) * float(E[a] - E[b])", "oracle/__init__.py"),
    ("pt: every pair every round", "for i in range(rnd % 2, nT - 1, 2):", "for i in range(0, nT - 1):",
     "oracle/__init__.py"),
    ("pt: one map not updated", "            temp_of[a], temp_of[b] = i + 1, i\n", "", "oracle/__init__.py"),
    ("pt: sets share the exchange stream", "draw_word(seed, TAG_EXCHANGE, i, pt_set, rnd)",
     "draw_word(seed, TAG_EXCHANGE, i, 0, rnd)", "oracle/__init__.py"),
    ("pt: sets share replica ids", "rid = [pt_set * nT + r for r in range(nT)]", "rid = list(range(nT))",
     "oracle/__init__.py"),
    # double checkerboard with k hits (Sec. "Checkerboard scheme")
    ("dcb: second coarse colour first", "if (((x / T + y / T) & 1) != P || ((x + y) & 1) != c) continue;",
     "if (((x / T + y / T + 1) & 1) != P || ((x + y) & 1) != c) continue;"),
    ("dcb: one hit fewer", "for (int h = 0; h < k; ++h) {\n                uint64_t draw_sweep",
     "for (int h = 1; h < k; ++h) {\n                uint64_t draw_sweep"),
    ("dcb: hits share one draw", "uint64_t draw_sweep = sweep * (uint64_t)k + (uint64_t)h;",
     "uint64_t draw_sweep = sweep * (uint64_t)k;"),
    ("dcb: tiles by row bands", "if (((x / T + y / T) & 1) != P || ((x + y) & 1) != c) continue;",
     "if (((y / T) & 1) != P || ((x + y) & 1) != c) continue;"),
    ("dcb: odd sites first", "if (((x / T + y / T) & 1) != P || ((x + y) & 1) != c) continue;",
     "if (((x / T + y / T) & 1) != P || ((x + y + 1) & 1) != c) continue;"),
    # Wang-Landau in windows (Sec. "Wang-Landau update", windows of Sec.
    # "Multicanonical simulations")
    ("wl: rejected out-of-window move not counted", "else if (k2 < klo || k2 > khi) accept = 0;       /* counted again */",
     "else if (k2 < klo || k2 > khi) continue;"),
    ("wl: acceptance ratio inverted", "int64_t d = Gw[k2 - klo] - Gw[k - klo];",
     "int64_t d = Gw[k - klo] - Gw[k2 - klo];"),
    ("wl: estimate raised before the move", "                    if (accept) { s[i] = (int8_t)-s[i]; k = k2; }\n"
     "                    Gw[k - klo] += inc[win];",
     "                    Gw[k - klo] += inc[win];\n                    if (accept) { s[i] = (int8_t)-s[i]; k = k2; }"),
    ("wl: table factor for the wrong byte", "p = p * t16[(lo >> 16) & 255u];", "p = p * t16[(lo >> 8) & 255u];"),
    ("wl: threshold floor", "    uint64_t T = (uint64_t)ceil(ldexp(p, 32));\n    return T < 1 ? 1 : T;",
     "    uint64_t T = (uint64_t)floor(ldexp(p, 32));\n    return T < 1 ? 1 : T;"),
    ("wl: drive ignores the draw", "if (r >> 31) { s[i] = (int8_t)-s[i]; k += dl; }",
     "{ s[i] = (int8_t)-s[i]; k += dl; }"),
    ("wl: match shift sign", "s = s + (prev[k - lo[i - 1]] - cur[k - lo[i]])",
     "s = s + (cur[k - lo[i]] - prev[k - lo[i - 1]])", "oracle/__init__.py"),
    ("wl: ln f not halved", "inc = [WL_ONE >> stage[i] for i in range(nwin)]", "inc = [WL_ONE for i in range(nwin)]",
     "oracle/__init__.py"),
    ("muca windows: recursion sign", "new[j] += math.floor(math.log(float(Hw[j])) * float(WL_ONE) + 0.5)",
     "new[j] -= math.floor(math.log(float(Hw[j])) * float(WL_ONE) + 0.5)", "oracle/__init__.py"),
    ("muca windows: piece without the weights", "pieces[i] = np.array([math.log(float(Hw[j])) + float(g[j]) / float(WL_ONE) if Hw[j] > 0 else 0.0\n                                      for j in range(n)])",
     "pieces[i] = np.array([math.log(float(Hw[j])) if Hw[j] > 0 else 0.0\n                                      for j in range(n)])", "oracle/__init__.py"),
]

PIN_TESTS = ["tests/test_golden_lng.py", "tests/test_oracle_dcb.py", "tests/test_oracle_exact.py",
             "tests/test_oracle_mlp.py",
             "tests/test_oracle_muca.py", "tests/test_oracle_pa.py", "tests/test_oracle_pt.py",
             "tests/test_oracle_rng.py", "tests/test_oracle_streams.py", "tests/test_oracle_sweep.py",
             "tests/test_oracle_tables.py", "tests/test_oracle_wl.py"]


def _copy_tree(dst):
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "*.tmp*", "__pycache__"))
    os.makedirs(os.path.join(dst, "tests"))
    for name in os.listdir(os.path.join(ROOT, "tests")):
        src = os.path.join(ROOT, "tests", name)
        if name == "golden":
            shutil.copytree(src, os.path.join(dst, "tests", "golden"))
        elif name in ("conftest.py", "philox_rocrand_kat.cpp") or "tests/" + name in PIN_TESTS:
            shutil.copy(src, os.path.join(dst, "tests", name))
    # the Weyl-increment pin reads the library's constants header as text
    os.makedirs(os.path.join(dst, "paper_1709_04394_amd", "csrc"))
    shutil.copy(os.path.join(ROOT, "paper_1709_04394_amd", "csrc", "common.hpp"),
                os.path.join(dst, "paper_1709_04394_amd", "csrc", "common.hpp"))


def run_mutant(m):
    name, old, new = m[:3]
    rel = m[3] if len(m) > 3 else "oracle/mcoracle.c"
    with tempfile.TemporaryDirectory(prefix="mut_") as d:
        _copy_tree(d)
        path = os.path.join(d, rel)
        text = open(path).read()
        if text.count(old) != 1:
            return name, "not applicable (pattern found %d times)" % text.count(old), 0.0
        open(path, "w").write(text.replace(old, new))
        env = dict(os.environ, PYTHONPATH=d, OMP_NUM_THREADS="2")
        b = subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=d, env=env,
                           capture_output=True, text=True)
        if b.returncode:
            return name, "does not compile", 0.0
        t0 = time.time()
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PIN_TESTS,
                           cwd=d, env=env, capture_output=True, text=True)
        el = time.time() - t0
        if r.returncode == 0:
            return name, "SURVIVED", el
        failed = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED ")]
        return name, "caught by " + (failed[0] if failed else "a failing run (exit %d)" % r.returncode), el


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=3)
    ap.add_argument("--only", nargs="*", default=None, help="substrings of mutant names to run")
    a = ap.parse_args()
    todo = [m for m in MUTANTS if not a.only or any(s in m[0] for s in a.only)]
    caught = 0
    with cf.ThreadPoolExecutor(a.jobs) as ex:
        for name, verdict, el in ex.map(run_mutant, todo):
            caught += verdict.startswith("caught")
            print("%-48s %s (%.0f s)" % (name, verdict, el), flush=True)
    print("caught %d of %d" % (caught, len(todo)))


if __name__ == "__main__":
    main()
