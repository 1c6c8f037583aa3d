"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a small C driver calls every exported oracle routine on small
inputs -- odd and three-colour lattices, 2D and 3D, couplings, both update
rules, a ragged multi-level scan, a population-annealing run, a
multicanonical start, settle and sweeps -- and the run must end cleanly with
no sanitizer report.  The driver also checks a few results against each
other (sweeps compose, energies agree with a fresh measurement)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mcoracle.c")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t orc_draw_byte(uint64_t, uint32_t, uint32_t, uint32_t, uint64_t, uint32_t);
uint32_t orc_draw32(uint64_t, uint32_t, uint32_t, uint32_t, uint32_t, uint64_t, uint32_t);
uint32_t orc_draw_word(uint64_t, uint32_t, uint32_t, uint32_t, uint64_t);
double orc_resample_u(uint64_t, uint32_t, uint32_t, uint32_t);
void orc_metropolis_table(double, int, uint64_t *);
void orc_heatbath_table(double, int, uint64_t *);
int orc_init(int, int, int, int, int8_t *, int, uint64_t, uint32_t);
int orc_couplings(int, int, int, int, int8_t *, uint64_t);
int orc_couplings_of(int, int, int, int, int8_t *, uint64_t, uint32_t);
int orc_sweep_dcb(int, int, int, int8_t *, double, uint64_t, uint32_t, uint64_t, int, int64_t *);
void orc_measure(int, int, int, int, const int8_t *, const int8_t *, int64_t *, int64_t *);
int orc_sweep(int, int, int, int, int8_t *, const int8_t *, int, double, uint64_t, uint32_t, uint64_t, int,
              int64_t *);
int orc_sweep_q3(int, int8_t *, double, uint64_t, uint32_t, uint64_t, int, int64_t *);
void orc_canonical_scan(const double *, double *, int64_t);
int orc_pa_init(int, int, int, uint64_t, int8_t *, int64_t *);
int orc_pa_steps(int, int, int, int, int, const double *, int, uint64_t, int8_t *, int64_t *, double *, double *,
                 int64_t *, int32_t *);
void orc_muca_table(int, const double *, uint64_t *);
int orc_muca_strat_level(int, int);
int orc_muca_start(int, int, uint64_t, int, int8_t *, int64_t *);
int orc_muca_settle(int, int, int8_t *, int64_t *);
int orc_muca_sweeps(int, int, int8_t *, int64_t *, const double *, uint64_t, uint64_t, int, int, int64_t *);

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); return 1; } } while (0)

static int lattice_case(int dims, int Lx, int Ly, int Lz, int rule, int withJ)
{
    const int64_t N = (int64_t)Lx * Ly * Lz;
    int8_t *s = malloc((size_t)N), *t = malloc((size_t)N), *J = withJ ? malloc((size_t)(dims * N)) : NULL;
    int64_t *EM = malloc(sizeof(int64_t) * 2 * 12), E, M;
    CHECK(orc_init(dims, Lx, Ly, Lz, s, 1, 7, 3) == 0);
    if (J) CHECK(orc_couplings(dims, Lx, Ly, Lz, J, 11) == 0);
    if (J) CHECK(orc_couplings_of(dims, Lx, Ly, Lz, J, 11, 5) == 0);
    memcpy(t, s, (size_t)N);
    CHECK(orc_sweep(dims, Lx, Ly, Lz, s, J, rule, 0.4, 5, 3, 0, 12, EM) == 0);
    CHECK(orc_sweep(dims, Lx, Ly, Lz, t, J, rule, 0.4, 5, 3, 0, 5, NULL) == 0);
    CHECK(orc_sweep(dims, Lx, Ly, Lz, t, J, rule, 0.4, 5, 3, 5, 7, NULL) == 0);
    CHECK(memcmp(s, t, (size_t)N) == 0);
    orc_measure(dims, Lx, Ly, Lz, s, J, &E, &M);
    CHECK(E == EM[2 * 11] && M == EM[2 * 11 + 1]);
    free(s); free(t); free(J); free(EM);
    return 0;
}

int main(void)
{
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    uint64_t T[16];
    orc_philox4x32_10(ctr, key, out);
    CHECK(orc_draw_byte(1, 2, 100, 3, 4, 1) < 256);
    (void)orc_draw32(1, 2, 7, 100, 3, 4, 0);
    (void)orc_draw_word(1, 5, 100, 3, 4);
    double u = orc_resample_u(1, 2, 3, 4);
    CHECK(u >= 0.0 && u < 1.0);
    orc_metropolis_table(0.44, 3, T);
    orc_heatbath_table(0.22, 6, T);

    if (lattice_case(2, 8, 6, 1, 0, 0)) return 1;
    if (lattice_case(2, 4, 4, 1, 1, 1)) return 1;
    if (lattice_case(3, 4, 6, 4, 1, 0)) return 1;
    if (lattice_case(3, 6, 4, 4, 0, 1)) return 1;
    {
        int8_t s[9] = {0};
        int64_t EM[8];
        CHECK(orc_init(2, 3, 3, 1, s, 1, 3, 0) == 0);
        CHECK(orc_sweep_q3(3, s, 0.3, 3, 0, 0, 4, EM) == 0);
        CHECK(orc_sweep(2, 5, 4, 1, s, NULL, 0, 0.3, 1, 0, 0, 1, NULL) == -1);  /* odd extent rejected */
    }
    {
        int8_t s[144];
        int64_t EM[6];
        CHECK(orc_init(2, 12, 12, 1, s, 1, 3, 0) == 0);
        CHECK(orc_sweep_dcb(12, 2, 3, s, 0.4, 3, 0, 5, 3, EM) == 0);
        CHECK(orc_sweep_dcb(12, 4, 1, s, 0.4, 3, 0, 5, 3, EM) == -1);  /* 3 tiles per side: not a checkerboard */
    }
    {
        const int64_t R = 64 * 64 + 64 * 3 + 7;
        double *w = malloc(sizeof(double) * R), *C = malloc(sizeof(double) * R);
        for (int64_t i = 0; i < R; ++i) w[i] = (double)((i * 37) % 101);
        orc_canonical_scan(w, C, R);
        double acc = 0;
        for (int64_t i = 0; i < R; ++i) { acc += w[i]; CHECK(C[i] == acc); }
        free(w); free(C);
    }
    {
        const int L = 8, R = 70, ns = 4;
        const int64_t N = L * L;
        int8_t *sp = malloc((size_t)(R * N));
        int64_t *E = malloc(sizeof(int64_t) * R), *h = calloc((size_t)(ns + 1) * (N + 1), sizeof(int64_t));
        double beta[5] = {0, 0.1, 0.2, 0.3, 0.4}, Ct[4], lq[4];
        int32_t *cnt = malloc(sizeof(int32_t) * R);
        CHECK(orc_pa_init(L, R, 1, 9, sp, E) == 0);
        CHECK(orc_pa_steps(L, R, 1, 1, ns, beta, 2, 9, sp, E, Ct, lq, h, cnt) == 0);
        int64_t tot = 0;
        for (int k = 0; k < R; ++k) tot += cnt[k];
        CHECK(tot == R);
        free(sp); free(E); free(h); free(cnt);
    }
    {
        const int L = 8, W = 10;
        const int64_t N = L * L, K = N / 2;
        double *lnW = calloc((size_t)(K + 1), sizeof(double));
        uint64_t *Tm = malloc(sizeof(uint64_t) * 4 * (K + 1));
        int8_t *sp = malloc((size_t)(W * N));
        int64_t *E = malloc(sizeof(int64_t) * W), *H = calloc((size_t)(K + 1), sizeof(int64_t));
        for (int64_t k = 0; k <= K; ++k) lnW[k] = -0.05 * (double)((K - k) * (K - k)) / (double)K;
        orc_muca_table(L, lnW, Tm);
        CHECK(orc_muca_strat_level(0, W) >= 0);
        CHECK(orc_muca_start(L, W, 3, 1, sp, E) == 0);
        CHECK(orc_muca_settle(L, W, sp, E) == 0);
        CHECK(orc_muca_sweeps(L, W, sp, E, lnW, 3, 0, 5, 1, H) == 0);
        int64_t tot = 0;
        for (int64_t k = 0; k <= K; ++k) tot += H[k];
        CHECK(tot == 5 * W * N);
        free(lnW); free(Tm); free(sp); free(E); free(H);
    }
    puts("oracle sanitized ok");
    return 0;
}
"""


def _run(tmp_path, sanitize):
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / ("drv_" + sanitize.replace(",", "_"))
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=" + sanitize, "-fno-sanitize-recover=all", str(drv), SRC, "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2")
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_oracle_under_ubsan(tmp_path):
    r = _run(tmp_path, "undefined")
    assert r.returncode == 0 and "oracle sanitized ok" in r.stdout and "runtime error" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_oracle_under_asan(tmp_path):
    r = _run(tmp_path, "address")
    if "does not come first in initial library list" in r.stderr:
        pytest.skip("AddressSanitizer cannot start in this environment (another library is preloaded)")
    assert r.returncode == 0 and "oracle sanitized ok" in r.stdout, r.stderr
