"""The C ABI from plain C (no GPU needed, no compute call made): the header
compiles as strict C99 with every warning an error, and a C program linked
against libmcspin.so reads the ABI version, names error codes, and gets the
documented validation errors from calls whose arguments are invalid."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1709_04394_amd")
LIB = os.path.join(PKG, "libmcspin.so")

SRC = r"""
#include <stdio.h>
#include <string.h>
#include "mcspin.h"

int main(void)
{
    mc_ctx *ctx = NULL;
    mc_geom bad = {2, 5, 8, 1, MC_INT8, 1};   /* odd extent */
    mc_geom ok = {2, 64, 64, 1, MC_INT8, 1};
    mc_sweep_args sa;
    int32_t L[1] = {12};                       /* not a population annealing extent */
    double beta[2] = {0.0, 0.1};
    mc_pa_args pa;
    int32_t G = 0;
    int rc;

    if (mc_abi_version() != MC_ABI_VERSION) return 10;
    if (strlen(mc_strerror(MC_E_SHAPE)) == 0) return 11;
    if (mc_ctx_create(&ctx, 0) != MC_OK || ctx == NULL) return 12;
    memset(&sa, 0, sizeof sa);
    sa.rule = MC_METROPOLIS;
    sa.beta = 0.4;
    sa.nsweeps = 1;
    rc = mc_sweep(ctx, &bad, (void *)0x1000, NULL, &sa, NULL, NULL, 0, NULL);
    if (rc != MC_E_SHAPE) return 13;
    if (strlen(mc_ctx_last_error(ctx)) == 0) return 14;
    sa.beta = -1.0;
    if (mc_sweep(ctx, &ok, (void *)0x1000, NULL, &sa, NULL, NULL, 0, NULL) != MC_E_RANGE) return 15;
    if (mc_sweep_workspace_bytes(&ok) != 2 * 64 * 64 / 8 + 2 * 8 * 16 * 16) return 16;
    memset(&pa, 0, sizeof pa);
    pa.npop = 1;
    pa.L = L;
    pa.R = 10;
    pa.theta = 1;
    pa.step_first = 1;
    pa.nsteps = 1;
    pa.beta = beta;
    if (mc_pa_workspace_bytes(&pa) != 0) return 17;
    if (mc_get_pa_group(ctx, 16, &G) != MC_OK || G != 16) return 18;
    mc_ctx_destroy(ctx);
    printf("c abi ok %d\n", mc_abi_version());
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_and_library_from_c99(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("libmcspin.so is not built")
    src = tmp_path / "abi.c"
    src.write_text(SRC)
    exe = tmp_path / "abi"
    cmd = ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           str(src), "-o", str(exe), "-L", PKG, "-lmcspin", "-Wl,-rpath," + PKG]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "c abi ok 1" in r.stdout, (r.returncode, r.stdout, r.stderr)
