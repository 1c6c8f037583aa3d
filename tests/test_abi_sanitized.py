"""libmcspin's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU needed, no device work).  The host-side translation units (argument
checks, tables, launch-shape settings, the launch-shape file parser, the
training-set builder, the replica-exchange step) are rebuilt with the sanitizers on the host pass only
and linked with the kernel objects of the normal build; a C driver built
with the same compiler family then calls every host-only entry point --
valid and invalid arguments, a cache round trip and malformed cache files --
and must finish with no sanitizer report."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1709_04394_amd", "csrc")
OBJS = os.path.join(ROOT, "paper_1709_04394_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_UNITS = ["abi", "tuning", "tempering", "sweep_driver", "pa_driver", "muca_driver", "mlp_driver", "wl_driver"]

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include "mcspin.h"

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); return 1; } } while (0)
static void *const FAKE = (void *)0x1000;  /* never dereferenced: every call using it fails validation */

int main(int argc, char **argv)
{
    mc_ctx *ctx = NULL, *c2 = NULL;
    int32_t H, K, T, G, n;
    CHECK(argc == 4);
    CHECK(mc_ctx_create(&ctx, 0) == MC_OK && mc_ctx_create(&c2, 0) == MC_OK);
    for (int code = 1; code >= -9; --code) CHECK(strlen(mc_strerror(code)) > 0);

    /* geometry and argument checks */
    mc_sweep_args sa = {MC_METROPOLIS, 0.4, 1, 0, 0, 1};
    mc_geom bad[] = {{1, 8, 8, 1, MC_INT8, 1}, {2, 5, 8, 1, MC_INT8, 1}, {2, 8, 8, 3, MC_INT8, 1},
                     {3, 8, 8, 7, MC_INT8, 1}, {2, 8, 8, 1, 9, 1}, {2, 8, 8, 1, MC_INT8, 0},
                     {2, 8, 8, 1, MC_INT8, 65536}, {2, 1 << 21, 8, 1, MC_INT8, 1}};
    for (size_t i = 0; i < sizeof bad / sizeof bad[0]; ++i) {
        CHECK(mc_sweep(ctx, &bad[i], FAKE, NULL, &sa, NULL, NULL, 0, NULL) < 0);
        CHECK(strlen(mc_ctx_last_error(ctx)) > 0);
        CHECK(mc_sweep_workspace_bytes(&bad[i]) == 0);
    }
    mc_geom g2 = {2, 4096, 4096, 1, MC_INT8, 3}, g3 = {3, 256, 256, 256, MC_INT8, 1};
    sa.beta = -1.0;
    CHECK(mc_sweep(ctx, &g2, FAKE, NULL, &sa, NULL, NULL, 0, NULL) == MC_E_RANGE);
    double betas[3] = {0.4, -0.1, 0.5};
    sa.beta = 0.4;
    CHECK(mc_sweep_betas(ctx, &g2, FAKE, NULL, &sa, betas, NULL, NULL, 0, NULL) == MC_E_RANGE);
    CHECK(mc_sweep_workspace_bytes(&g2) == 2ull * 3 * 4096 * 4096 / 8 + 2ull * 8 * 3 * 1024 * 16);

    /* kernel family and launch shapes */
    int32_t path = 0;
    CHECK(mc_sweep_path(ctx, &g2, MC_METROPOLIS, 0, 0, mc_sweep_workspace_bytes(&g2), &path) == MC_OK &&
          path == MC_PATH_FUSED_2D);
    CHECK(mc_sweep_path(ctx, &g2, MC_HEATBATH, 1, 0, 0, &path) == MC_OK && path == MC_PATH_GENERIC);
    CHECK(mc_get_tile_plan(ctx, &g2, &H, &K, &T) == MC_OK);
    CHECK(mc_set_tile_plan(ctx, &g2, 16, 4, 512) == MC_OK);
    CHECK(mc_set_tile_plan(ctx, &g2, 16, 4, 96) == MC_E_RANGE);
    CHECK(mc_set_tile_plan(ctx, &g3, 8, 4, 256) == MC_OK);
    CHECK(mc_set_pa_group(ctx, 32, 16) == MC_OK && mc_set_pa_group(ctx, 512, 2) == MC_E_RANGE);
    CHECK(mc_get_pa_group(ctx, 128, &G) == MC_OK && G == 1);

    /* population annealing argument checks */
    int32_t Ls[2] = {16, 16};
    double beta[3] = {0.0, 0.1, 0.2};
    mc_pa_args pa = {2, Ls, 64, 1, 1, 1, 2, beta};
    void *pops[2] = {FAKE, FAKE};
    CHECK(mc_tune_pa(ctx, &pa, pops, FAKE, (size_t)1 << 30, NULL, NULL) == MC_E_INVAL);  /* same L twice */
    Ls[1] = 32;
    CHECK(mc_pa_workspace_bytes(&pa) > 0);
    CHECK(mc_tune_pa(ctx, &pa, pops, FAKE, 16, NULL, NULL) == MC_E_WORKSPACE);
    CHECK(mc_pa_anneal(ctx, &pa, pops, NULL, NULL, NULL, NULL, FAKE, 16, NULL) == MC_E_INVAL);

    /* multicanonical and MLP host calls */
    CHECK(mc_muca_workspace_bytes(128, 4096) > 0 && mc_muca_workspace_bytes(10, 4096) == 0);
    CHECK(mc_muca_start(ctx, 10, 16, 1, MC_MUCA_HOT, FAKE, FAKE, NULL) == MC_E_SHAPE);
    double lw4[9], lw8[33];
    for (int k = 0; k < 9; ++k) lw4[k] = -0.5 * (8 - k);
    for (int k = 0; k < 33; ++k) lw8[k] = -0.25 * (32 - k);
    int32_t tl[2] = {4, 8};
    const double *tw[2] = {lw4, lw8};
    float X[2 * 64], Y[64];
    CHECK(mc_mlp_training_set(ctx, 2, tl, tw, X, Y, 64, &n) == MC_OK && n == 8 + 32);
    CHECK(mc_mlp_training_set(ctx, 2, tl, tw, X, Y, 10, &n) == MC_E_RANGE);
    CHECK(mc_mlp_param_count() == 4417 && mc_mlp_workspace_bytes(100) > 0);
    {
        double uw[33], flat;
        int64_t uh[33];
        for (int k = 0; k < 33; ++k) { uw[k] = -0.1 * k; uh[k] = k == 1 ? 0 : 100 + k; }
        CHECK(mc_muca_update(ctx, 8, uw, uh, uw, &flat) == MC_OK && uw[32] == 0.0 && flat > 0.0);
        uh[4] = -1;
        CHECK(mc_muca_update(ctx, 8, uw, uh, uw, NULL) == MC_E_RANGE);
    }

    /* parallel tempering exchange (host only) */
    double tb[3] = {0.1, 0.2, 0.3};
    int64_t tE[3] = {-8, 0, 4}, tacc[2] = {0, 0};
    int32_t tof[3] = {0, 1, 2}, rat[3] = {0, 1, 2};
    for (uint64_t t = 0; t < 100; ++t) CHECK(mc_pt_exchange(ctx, 3, tb, tE, tof, rat, 1, t, tacc) == MC_OK);
    CHECK(rat[tof[0]] == 0 && rat[tof[1]] == 1 && rat[tof[2]] == 2);
    CHECK(mc_pt_exchange(ctx, 3, tb, tE, tof, rat, 1, (uint64_t)1 << 55, tacc) == MC_E_RANGE);
    tof[0] = tof[1];
    CHECK(mc_pt_exchange(ctx, 3, tb, tE, tof, rat, 1, 0, tacc) == MC_E_INVAL);

    /* windows (host-side checks only; no device work) */
    int32_t wlo[2] = {0, 14}, whi[2] = {20, 32}, gap_lo[2] = {0, 22};
    mc_wl_args wa;
    memset(&wa, 0, sizeof wa);
    wa.L = 8; wa.nwin = 2; wa.lo = wlo; wa.hi = whi; wa.walkers = 64; wa.check_sweeps = 1;
    wa.flat = 0.8; wa.lnf_final = 1e-4; wa.max_sweeps = 10; wa.max_pass = 10; wa.seed = 1;
    size_t wsb = mc_wl_workspace_bytes(&wa);
    CHECK(wsb > 0);
    double wp[2 * 21], wl[33];
    mc_wl_window_stats wst[2];
    CHECK(mc_wl_run(ctx, &wa, FAKE, FAKE, wp, wl, wst, FAKE, wsb - 1, NULL) == MC_E_WORKSPACE);
    wa.lnf_final = 2.0;
    CHECK(mc_wl_run(ctx, &wa, FAKE, FAKE, wp, wl, wst, FAKE, wsb, NULL) == MC_E_RANGE);
    wa.lnf_final = 1e-4; wa.lo = gap_lo;
    CHECK(mc_wl_run(ctx, &wa, FAKE, FAKE, wp, wl, wst, FAKE, wsb, NULL) == MC_E_RANGE);
    CHECK(mc_win_drive(ctx, 8, 2, wlo, whi, 32, 1, 10, FAKE, FAKE, FAKE, wsb, NULL) == MC_E_RANGE);
    int64_t winc[2] = {1, -1};
    uint8_t wact[2] = {1, 1};
    CHECK(mc_wl_sweeps(ctx, 8, 2, wlo, whi, 64, winc, wact, 0.8, 1, 0, 1, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, wsb,
                       NULL) == MC_E_RANGE);
    mc_muca_win_args ma;
    memset(&ma, 0, sizeof ma);
    ma.L = 8; ma.nwin = 2; ma.lo = wlo; ma.hi = whi; ma.walkers = 64; ma.eq_sweeps = 2; ma.rec_sweeps = 0;
    ma.max_iter = 5; ma.flat = 0.8; ma.max_pass = 10; ma.seed = 1;
    mc_muca_win_stats mst[2];
    CHECK(mc_muca_windows_workspace_bytes(&ma) == wsb);
    CHECK(mc_muca_windows_run(ctx, &ma, FAKE, FAKE, wp, wl, mst, FAKE, wsb, NULL) == MC_E_RANGE);

    /* launch-shape file: round trip, then malformed files */
    CHECK(mc_tuning_save(ctx, argv[1]) == MC_OK);
    CHECK(mc_tuning_load(c2, argv[1]) == MC_OK);
    CHECK(mc_get_tile_plan(c2, &g2, &H, &K, &T) == MC_OK && H == 16 && K == 4 && T == 512);
    CHECK(mc_get_pa_group(c2, 32, &G) == MC_OK && G == 16);
    CHECK(mc_tuning_load(c2, argv[2]) == MC_E_INVAL);
    CHECK(mc_tuning_load(c2, argv[3]) == MC_E_INVAL);
    CHECK(mc_tuning_load(c2, "/nonexistent/dir/file") == MC_E_IO);
    CHECK(mc_tuning_save(c2, "/nonexistent/dir/file") == MC_E_IO);
    mc_ctx_destroy(ctx);
    mc_ctx_destroy(c2);
    puts("host code sanitized ok");
    return 0;
}
"""


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm compilers")
def test_host_code_under_asan_and_ubsan(tmp_path):
    kernels = sorted(glob.glob(os.path.join(OBJS, "k_*.hip.o")))
    if not kernels:
        pytest.skip("the library's kernel objects are not built")
    objs = []
    for unit in HOST_UNITS:
        obj = str(tmp_path / (unit + ".o"))
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
               "-c", os.path.join(CSRC, unit + ".hip"), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    lib = str(tmp_path / "libmcspin_san.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined", "-o", lib] + objs + kernels,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    src = tmp_path / "drv.c"
    src.write_text(DRIVER)
    exe = str(tmp_path / "drv")
    r = subprocess.run([CLANG, "-std=c99", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-I", os.path.join(ROOT, "include"), str(src), lib, "-Wl,-rpath," + str(tmp_path),
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    (tmp_path / "long.txt").write_text("libmcspin-launch-shapes 1\n" + "x" * 1000 + "\n")
    (tmp_path / "junk.txt").write_text("libmcspin-launch-shapes 1\ntile 2 4096 4096 1 3 16 4\npa\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path / "shapes.txt"), str(tmp_path / "long.txt"), str(tmp_path / "junk.txt")],
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and "host code sanitized ok" in r.stdout, (r.returncode, r.stdout, r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
