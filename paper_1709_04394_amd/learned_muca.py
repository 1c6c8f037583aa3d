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


def refined_weights(ctx, L, lnW, H):
    """The recursion (Eq. weight_modification, mc_muca_update) applied to a
    production histogram H at the weights lnW: ln W - ln H, i.e. -ln g_est,
    normalised to 0 at E = 0.  Every level that has states must have been
    visited (the level without states, k = 1, keeps its weight, which no
    move can reach)."""
    H = np.asarray(H, dtype=np.int64)
    reach = np.ones(H.size, dtype=bool)
    reach[1] = False
    if not np.all(H[reach] > 0):
        raise RuntimeError("L=%d: the production histogram left %d window levels unvisited"
                           % (L, int(np.sum(H[reach] == 0))))
    out, _ = ctx.muca_update(L, lnW, H)
    return out


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
        out[L] = refined_weights(ctx, L, r["lnW"], r["H_prod"])
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


# ---------------------------------------------------------------------------
# Long production at fixed converged weights, split over independent runs.
# At L = 128 the error of ln g = ln H - ln W is set by how many times the
# walkers cross the energy window, so reaching a given accuracy takes hundreds
# of thousands of sweeps per walker; separate runs (each from its own walker
# start and burn-in, different seeds) add their histograms.

def production(ctx, L, lnW, seed, burn, sweeps, walkers=WALKERS, chunk=1000, label=""):
    """Recorded histogram of `sweeps` multicanonical sweeps per walker at fixed
    weights lnW, after a stratified walker start and `burn` unrecorded sweeps;
    sweeps are numbered from 0 over burn-in and production.  Returns the int64
    histogram over the window levels."""
    from . import MUCA_STRATIFIED

    spins, E = ctx.muca_start(L, walkers, seed, start=MUCA_STRATIFIED)
    ws = ctx.muca_workspace(L, walkers)
    H = torch.zeros(L * L // 2 + 1, dtype=torch.int64, device=ctx.device)
    t0 = time.perf_counter()
    last, sw = t0, 0
    for rec, n in ((False, burn), (True, sweeps)):
        done = 0
        while done < n:
            k = min(chunk, n - done)
            ctx.muca_sweeps(L, spins, E, lnW, seed, sw, k, rec, H=H if rec else None, ws=ws)
            done += k
            sw += k
            torch.cuda.synchronize()
            now = time.perf_counter()
            if now - last > 20:
                last = now
                print("%s seed %d: %s %d/%d, %.0f s" % (label, seed, "production" if rec else "burn-in", done, n,
                                                       now - t0), file=sys.stderr, flush=True)
    return H.cpu().numpy()


def lng_errors(H, lnW, lng_exact):
    """max |ln g_est - ln g_exact| over the levels with states, ln g_est =
    ln H - ln W: (a) after matching the normalisations (log-sum-exp over those
    levels), (b) after the best additive constant (half the spread of the
    differences; the method fixes ln g only up to a constant)."""
    m = np.isfinite(lng_exact)
    with np.errstate(divide="ignore"):
        lng = np.where(H > 0, np.log(np.maximum(H, 1)), -np.inf) - lnW
    if not np.all(np.isfinite(lng[m])):
        return float("inf"), float("inf")
    a, b = lng[m], lng_exact[m]
    c = np.logaddexp.reduce(b) - np.logaddexp.reduce(a)
    d = b - a
    return float(np.max(np.abs(a + c - b))), float((d.max() - d.min()) / 2)


def main(argv=None):
    """Stages of the L = 128 comparison run to the accuracy target:
      converge --L 128 --out DIR        training sizes, MLP, both arms to a flat
                                        histogram; DIR/weights.npz, DIR/converge.json
      produce --dir DIR --arm A --seed S --burn B --sweeps P
                                        one production run; DIR/H_A_S.npy
      score --dir DIR --exact FILE      errors per run and per arm (runs summed)"""
    import argparse
    import glob
    import json
    import os

    p = argparse.ArgumentParser(prog="python -m paper_1709_04394_amd.learned_muca")
    sub = p.add_subparsers(dest="stage", required=True)
    c = sub.add_parser("converge")
    c.add_argument("--L", type=int, default=128)
    c.add_argument("--out", required=True)
    q = sub.add_parser("produce")
    q.add_argument("--dir", required=True)
    q.add_argument("--arm", choices=("plain", "learned"), required=True)
    q.add_argument("--seed", type=int, required=True)
    q.add_argument("--burn", type=int, default=20000)
    q.add_argument("--sweeps", type=int, required=True)
    q.add_argument("--refined", action="store_true",
                   help="run at ln W = -ln g estimated from the arm's earlier runs (summed), saved as "
                        "DIR/weights_refined_A.npy; the histogram goes to DIR/HR_A_S.npy")
    s = sub.add_parser("score")
    s.add_argument("--dir", required=True)
    s.add_argument("--exact", required=True, help="stored exact ln g over the window levels (text)")
    a = p.parse_args(argv)

    if a.stage == "score":
        w = np.load(os.path.join(a.dir, "weights.npz"))
        conv = json.load(open(os.path.join(a.dir, "converge.json")))
        ex = np.loadtxt(a.exact)
        out = {}
        for arm in ("plain", "learned"):
            files = sorted(glob.glob(os.path.join(a.dir, "H_%s_*.npy" % arm)))
            if not files:
                continue
            runs = {os.path.basename(f)[:-4]: lng_errors(np.load(f), w["lnW_" + arm], ex) for f in files}
            Hs = sum(np.load(f) for f in files)
            lse, best = lng_errors(Hs, w["lnW_" + arm], ex)
            out[arm] = dict(conv[arm], runs=runs, production_records=int(Hs.sum()),
                            max_abs_lng_error=lse, max_abs_lng_error_best_constant=best)
            rf = os.path.join(a.dir, "weights_refined_%s.npy" % arm)
            rfiles = sorted(glob.glob(os.path.join(a.dir, "HR_%s_*.npy" % arm)))
            if rfiles and os.path.exists(rf):
                lnWr = np.load(rf)
                out[arm]["refined_runs"] = {os.path.basename(f)[:-4]: lng_errors(np.load(f), lnWr, ex)
                                            for f in rfiles}
        print(json.dumps(out, indent=1))
        return

    from . import Context

    ctx = Context(0)
    if a.stage == "converge":
        os.makedirs(a.out, exist_ok=True)
        lnW_by_L, _ = training_weights(ctx)
        params, log = train_network(ctx, lnW_by_L)
        r = compare(ctx, a.L, params, prod_sweeps=0)
        conv = {arm: {k: (bool(r[arm][k]) if k == "converged" else float(r[arm][k]))
                      for k in ("iterations", "sweeps_per_walker", "total_sweeps", "seconds", "min_over_max",
                                "converged")} for arm in ("plain", "learned")}
        conv["mlp_loss"] = [float(log[0]), float(log[-1])]
        np.savez(os.path.join(a.out, "weights.npz"), lnW_plain=r["plain"]["lnW"], lnW_learned=r["learned"]["lnW"],
                 lnW_init=r["lnW_init"], L=a.L)
        json.dump(conv, open(os.path.join(a.out, "converge.json"), "w"))
        print(json.dumps(conv), flush=True)
    else:
        w = np.load(os.path.join(a.dir, "weights.npz"))
        L = int(w["L"])
        lnW = w["lnW_" + a.arm]
        if a.refined:
            files = sorted(glob.glob(os.path.join(a.dir, "H_%s_*.npy" % a.arm)))
            if not files:
                raise SystemExit("no earlier runs of arm %s in %s" % (a.arm, a.dir))
            lnW = refined_weights(ctx, L, lnW, sum(np.load(f) for f in files))
            np.save(os.path.join(a.dir, "weights_refined_%s.npy" % a.arm), lnW)
        H = production(ctx, L, lnW, a.seed, a.burn, a.sweeps, label=a.arm)
        np.save(os.path.join(a.dir, "%s_%s_%d.npy" % ("HR" if a.refined else "H", a.arm, a.seed)), H)
        print(json.dumps({"arm": a.arm, "seed": a.seed, "burn": a.burn, "sweeps": a.sweeps}), flush=True)


if __name__ == "__main__":
    main()
