"""Learned initial weights for the parallel-walker multicanonical method.

The multicanonical recursion (Sec. "Multicanonical simulations", Eq.
weight_modification) starts from flat weights and needs many iterations to
build ln W over the whole energy window.  Here the weights the method itself
converges to at small L train a small MLP on the GPU (mc_mlp_training_set,
mc_mlp_train), whose prediction at a larger L (mc_mlp_lnw_init) replaces the
flat start; the plain recursion remains the fallback when a prediction is not
finite.  Both arms then run the identical recursion, walker start and
iteration schedule to a flat histogram and the same production run.

This module only sequences library calls; every step runs in libmcspin.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import torch

from . import MUCA_HOT

TRAIN_L = (16, 24, 32, 48)
TEST_L = (64, 96, 128)
WALKERS = 4096

# Iterations: 2 unrecorded + R recorded sweeps, R = 10 doubled (up to a cap
# that grows with the walkers' equilibration time) after every iteration that
# reached the whole window without improving the flatness of the one before.
# Walkers start hot and are first thermalised to the initial weights by
# PREP_SWEEPS canonical sweeps per walker (a no-op for flat weights).
REC_MAX = {8: 40, 12: 40, 16: 40, 24: 80, 32: 160, 48: 320, 64: 640, 96: 1280, 128: 2560}
PREP_SWEEPS = 400


def run_arm(ctx, L, seed, lnW_init=None, walkers=WALKERS, eq_sweeps=2, rec_sweeps=10, rec_max=None,
            max_iter=8000, prod_sweeps=0, flat=0.8, start=MUCA_HOT, eq_scale=0, prep_sweeps=PREP_SWEEPS,
            rec_rule=1):
    """One multicanonical run (mc_muca_run); adds wall time and total sweeps
    of all walkers (multicanonical sweeps; the preparation sweeps are listed
    apart) to the result."""
    rec_max = REC_MAX.get(L, 10) if rec_max is None else rec_max
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = [t0]

    def progress(_user, it, flatness, sweeps):
        # a line at most every 20 s of a long run, on stderr
        now = time.perf_counter()
        if now - last[0] >= 20.0:
            last[0] = now
            phase = "iteration %d, flatness %.3f" % (it, flatness) if it > 0 else "production"
            print("multicanonical L=%d: %s, %d sweeps per walker, %.0f s" % (L, phase, sweeps, now - t0),
                  file=sys.stderr, flush=True)

    r = ctx.muca_run(L, walkers, seed, eq_sweeps, rec_sweeps, max_iter, prod_sweeps, flat=flat, lnW_init=lnW_init,
                     start=start, rec_max=rec_max, eq_scale=eq_scale, prep_sweeps=prep_sweeps, rec_rule=rec_rule,
                     progress=progress)
    r["seconds"] = time.perf_counter() - t0
    r["total_sweeps"] = int(r["sweeps_per_walker"]) * walkers
    r["prep_sweeps_per_walker"] = prep_sweeps
    r.pop("spins", None)
    return r


def training_weights(ctx, Ls=TRAIN_L, prod_sweeps=400, seed0=19, **kw):
    """Converged weights at each training size: ln W = -ln g_est from a plain
    run to a flat histogram plus a production run (the recursion applied once
    more, to the production histogram)."""
    out, runs = {}, {}
    for L in Ls:
        r = run_arm(ctx, L, seed0 + L, prod_sweeps=prod_sweeps, **kw)
        runs[L] = r
        if not r["converged"]:
            raise RuntimeError("plain multicanonical run at L=%d did not converge" % L)
        lng = r["lng"]
        lnW = -np.where(np.isfinite(lng), lng, 0.0)
        out[L] = lnW - lnW[-1]
    return out, runs


def train_network(ctx, lnW_by_L, seed=1, epochs=50000, lr=1e-3):
    """Full-batch Adam on the (E/N, 1/L) -> entropy-deficit samples of the
    converged weights; returns the device parameters and the loss curve."""
    X, Y = ctx.mlp_training_set(lnW_by_L)
    params = ctx.mlp_init(seed)
    log = ctx.mlp_train(params, torch.from_numpy(X).to(params.device), torch.from_numpy(Y).to(params.device),
                        epochs, lr=lr)
    return params, log.cpu().numpy()


def compare(ctx, L, params, seed=None, prod_sweeps=0, **kw):
    """Plain and learned arms at one size, same seed, start and schedule."""
    seed = 19 + L if seed is None else seed
    lnW0, fallback = ctx.mlp_lnw_init(params, L)
    plain = run_arm(ctx, L, seed, prod_sweeps=prod_sweeps, **kw)
    learned = run_arm(ctx, L, seed, lnW_init=None if fallback else lnW0, prod_sweeps=prod_sweeps, **kw)
    learned["fallback"] = bool(fallback)
    return {"plain": plain, "learned": learned, "lnW_init": lnW0}
