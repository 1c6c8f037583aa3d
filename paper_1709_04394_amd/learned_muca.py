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

def production(ctx, L, lnW, seed, burn, sweeps, walkers=WALKERS, chunk=1000, label="", checkpoints=None):
    """Recorded histogram of `sweeps` multicanonical sweeps per walker at fixed
    weights lnW, after a stratified walker start and `burn` unrecorded sweeps;
    sweeps are numbered from 0 over burn-in and production.  Returns the int64
    histogram over the window levels, or, with checkpoints (increasing counts
    of recorded sweeps, the last = sweeps), the cumulative histogram at each
    checkpoint as an array [len(checkpoints)][levels].  The walker count is
    free here: production runs at fixed weights, so more walkers (up to the
    16384 whose lattices fill every compute unit once at L = 128) give more
    statistics per sweep at about the same wall time."""
    from . import MUCA_STRATIFIED

    cps = [sweeps] if checkpoints is None else list(checkpoints)
    if sorted(cps) != cps or cps[-1] != sweeps or cps[0] < 1:
        raise ValueError("checkpoints must increase and end at sweeps")
    spins, E = ctx.muca_start(L, walkers, seed, start=MUCA_STRATIFIED)
    ws = ctx.muca_workspace(L, walkers)
    H = torch.zeros(L * L // 2 + 1, dtype=torch.int64, device=ctx.device)
    t0 = time.perf_counter()
    last, sw = t0, 0
    out = []
    done = 0
    while done < burn:
        k = min(chunk, burn - done)
        ctx.muca_sweeps(L, spins, E, lnW, seed, sw, k, False, ws=ws)
        done += k
        sw += k
        torch.cuda.synchronize()
        now = time.perf_counter()
        if now - last > 20:
            last = now
            print("%s seed %d: burn-in %d/%d, %.0f s" % (label, seed, done, burn, now - t0), file=sys.stderr, flush=True)
    done = 0
    for cp in cps:
        while done < cp:
            k = min(chunk, cp - done)
            ctx.muca_sweeps(L, spins, E, lnW, seed, sw, k, True, H=H, ws=ws)
            done += k
            sw += k
            torch.cuda.synchronize()
            now = time.perf_counter()
            if now - last > 20:
                last = now
                print("%s seed %d: production %d/%d, %.0f s" % (label, seed, done, sweeps, now - t0),
                      file=sys.stderr, flush=True)
        out.append(H.cpu().numpy())
    return out[-1] if checkpoints is None else np.stack(out)


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


def arm_summary(r):
    """The sweep counts of one arm's run to a flat histogram: multicanonical
    sweeps per walker, plus the walker preparation (the same for both arms)."""
    return {"converged": bool(r["converged"]), "iterations": int(r["iterations"]),
            "sweeps_per_walker": int(r["sweeps_per_walker"]),
            "prep_sweeps_per_walker": int(r["prep_sweeps_per_walker"]),
            "sweeps_per_walker_incl_prep": int(r["sweeps_per_walker"]) + int(r["prep_sweeps_per_walker"]),
            "seconds": round(float(r["seconds"]), 2), "final_min_over_max": float(r["min_over_max"])}


def score_markdown(out):
    """The score stage's summed runs as markdown: per arm and seed the error
    after each checkpoint of the accumulated production, and where the
    target was first met."""
    t = out["target"]
    lines = []
    for arm in ("plain", "learned"):
        for sd, v in out["arms"][arm]["summed_production"].items():
            lines += ["## %s arm (weights of seed %s; runs %s)" % (arm, sd, ", ".join(v["runs"])), "",
                      "| Production walker-sweeps | Error (log-sum-exp) | Error (best constant) |", "|---|---|---|"]
            lines += ["| %.3g | %.4f | %.4f |" % (c["walker_sweeps"], c["error_logsumexp"], c["error_best_constant"])
                      for c in v["curve"]]
            lines.append("")
            fl, hit = v["flat_walker_sweeps"], v["production_walker_sweeps_to_target"]
            if hit:
                lines.append("Within %g after %.3g production walker-sweeps; with the %.3g walker-sweeps of the flat "
                             "phase, %.3g in total." % (t, hit, fl, fl + hit))
            else:
                last = v["curve"][-1]
                lines.append("Not within %g after %.3g production walker-sweeps (last error %.4f); flat phase %.3g "
                             "walker-sweeps." % (t, last["walker_sweeps"], last["error_logsumexp"], fl))
            lines.append("")
    return "\n".join(lines)


def main(argv=None):
    """Stages of the learned-vs-plain comparison at one size:
      converge --L L --seeds S,.. --out DIR
            training sizes and the MLP (once), then both arms to a flat
            histogram for every seed: DIR/lnW_<arm>_<S>.npy, DIR/lnW_init.npy,
            DIR/mlp_params.npy, DIR/converge.json; run again on the same DIR,
            it reuses the network and skips the seeds already run
      produce --dir DIR --arm A --seed S --pseed P --walkers W --burn B
              --checkpoints C1,..,Cn
            production at the arm's converged weights of seed S (walker seed
            P): cumulative histograms after C1 .. Cn sweeps,
            DIR/prod_<arm>_<S>_<P>.npy
      score --dir DIR --exact FILE [--target 0.01] [--markdown]
            max |ln g error| of every production checkpoint, after matching
            the normalisations by log-sum-exp over the window levels with
            states (the accuracy metric) and after the best constant; the
            walker-sweeps at the first checkpoint within the target; the
            same for the runs at one seed's weights added together, with
            the flat phase's walker-sweeps; sweeps to flat per arm over the
            seeds.  JSON, or with --markdown one table per arm and seed of
            the runs added together"""
    import argparse
    import glob
    import json
    import os

    p = argparse.ArgumentParser(prog="python -m paper_1709_04394_amd.learned_muca")
    sub = p.add_subparsers(dest="stage", required=True)
    c = sub.add_parser("converge")
    c.add_argument("--L", type=int, required=True)
    c.add_argument("--seeds", required=True)
    c.add_argument("--out", required=True)
    q = sub.add_parser("produce")
    q.add_argument("--dir", required=True)
    q.add_argument("--arm", choices=("plain", "learned"), required=True)
    q.add_argument("--seed", type=int, required=True)
    q.add_argument("--pseed", type=int, required=True)
    q.add_argument("--walkers", type=int, default=16384)
    q.add_argument("--burn", type=int, default=20000)
    q.add_argument("--checkpoints", required=True)
    s = sub.add_parser("score")
    s.add_argument("--dir", required=True)
    s.add_argument("--exact", required=True, help="stored exact ln g over the window levels (text)")
    s.add_argument("--target", type=float, default=0.01)
    s.add_argument("--markdown", action="store_true", help="tables of the summed runs instead of JSON")
    a = p.parse_args(argv)

    if a.stage == "score":
        conv = json.load(open(os.path.join(a.dir, "converge.json")))
        ex = np.loadtxt(a.exact)
        out = {"L": conv["L"], "target": a.target, "metric": "max |ln g_est - ln g_exact| over the window levels "
               "with states, normalisations matched by log-sum-exp", "arms": {}}
        for arm in ("plain", "learned"):
            seeds = conv["seeds"]
            flat = [conv["runs"][str(sd)][arm]["sweeps_per_walker_incl_prep"] for sd in seeds]
            row = {"sweeps_to_flat_incl_prep": flat, "mean": float(np.mean(flat)),
                   "min": int(min(flat)), "max": int(max(flat)), "production": {}}
            for f in sorted(glob.glob(os.path.join(a.dir, "prod_%s_*.npy" % arm))):
                meta = json.load(open(f[:-4] + ".json"))
                lnW = np.load(os.path.join(a.dir, "lnW_%s_%d.npy" % (arm, meta["seed"])))
                Hs = np.load(f)
                errs = [lng_errors(H, lnW, ex) for H in Hs]
                reach = [cp for cp, e in zip(meta["checkpoints"], errs) if e[0] <= a.target]
                row["production"][os.path.basename(f)[:-4]] = dict(
                    meta, errors_logsumexp=[e[0] for e in errs], errors_best_constant=[e[1] for e in errs],
                    walker_sweeps_to_target=(reach[0] * meta["walkers"]) if reach else None)
            # the runs at one seed's weights, in walker-seed order, their
            # histograms added: the error after each checkpoint of the
            # accumulated production, and the walker-sweeps (flat phase, 4096
            # walkers, plus production) at the first within the target
            summed = {}
            for sd in seeds:
                files = sorted(glob.glob(os.path.join(a.dir, "prod_%s_%d_*.npy" % (arm, sd))),
                               key=lambda f: json.load(open(f[:-4] + ".json"))["pseed"])
                if not files:
                    continue
                lnW = np.load(os.path.join(a.dir, "lnW_%s_%d.npy" % (arm, sd)))
                base = None
                done_ws = 0
                curve = []
                for f in files:
                    meta = json.load(open(f[:-4] + ".json"))
                    Hs = np.load(f).astype(np.int64)
                    for cp, H in zip(meta["checkpoints"], Hs):
                        tot = H if base is None else base + H
                        e = lng_errors(tot, lnW, ex)
                        curve.append({"walker_sweeps": done_ws + cp * meta["walkers"], "error_logsumexp": e[0],
                                      "error_best_constant": e[1]})
                    base = Hs[-1] if base is None else base + Hs[-1]
                    done_ws += meta["checkpoints"][-1] * meta["walkers"]
                flat_ws = conv["runs"][str(sd)][arm]["sweeps_per_walker_incl_prep"] * WALKERS
                hit = [c["walker_sweeps"] for c in curve if c["error_logsumexp"] <= a.target]
                summed[str(sd)] = {"runs": [os.path.basename(f)[:-4] for f in files], "curve": curve,
                                   "flat_walker_sweeps": flat_ws,
                                   "production_walker_sweeps_to_target": hit[0] if hit else None,
                                   "total_walker_sweeps_to_target": flat_ws + hit[0] if hit else None}
            row["summed_production"] = summed
            out["arms"][arm] = row
        pl, le = out["arms"]["plain"]["mean"], out["arms"]["learned"]["mean"]
        out["mean_sweeps_to_flat_ratio_learned_over_plain"] = le / pl
        print(score_markdown(out) if a.markdown else json.dumps(out, indent=1))
        return

    from . import Context

    ctx = Context(0)
    if a.stage == "converge":
        os.makedirs(a.out, exist_ok=True)
        seeds = [int(x) for x in a.seeds.split(",")]
        pfile, cfile = os.path.join(a.out, "mlp_params.npy"), os.path.join(a.out, "converge.json")
        if os.path.exists(pfile) and os.path.exists(cfile):
            # resume: the trained network and the seeds already run are kept
            # (training is seeded, so retraining would give the same network)
            params = torch.from_numpy(np.load(pfile)).to(ctx.device)
            conv = json.load(open(cfile))
            if int(conv["L"]) != a.L:
                raise SystemExit("%s holds L=%d, not L=%d" % (cfile, conv["L"], a.L))
            conv["seeds"] = list(dict.fromkeys([int(x) for x in conv["seeds"]] + seeds))
        else:
            lnW_by_L, _ = training_weights(ctx)
            params, log = train_network(ctx, lnW_by_L)
            np.save(pfile, params.cpu().numpy())
            conv = {"L": a.L, "seeds": seeds, "mlp_loss": [float(log[0]), float(log[-1])], "runs": {}}
        for sd in seeds:
            if str(sd) in conv["runs"]:
                continue
            r = compare(ctx, a.L, params, seed=sd, prod_sweeps=0)
            conv["runs"][str(sd)] = {arm: arm_summary(r[arm]) for arm in ("plain", "learned")}
            conv["runs"][str(sd)]["learned"]["fallback"] = bool(r["learned"]["fallback"])
            for arm in ("plain", "learned"):
                np.save(os.path.join(a.out, "lnW_%s_%d.npy" % (arm, sd)), r[arm]["lnW"])
            np.save(os.path.join(a.out, "lnW_init.npy"), r["lnW_init"])
            json.dump(conv, open(os.path.join(a.out, "converge.json"), "w"), indent=1)
            print(json.dumps({"seed": sd, "runs": conv["runs"][str(sd)]}), flush=True)
    else:
        conv = json.load(open(os.path.join(a.dir, "converge.json")))
        L = int(conv["L"])
        lnW = np.load(os.path.join(a.dir, "lnW_%s_%d.npy" % (a.arm, a.seed)))
        cps = [int(x) for x in a.checkpoints.split(",")]
        t0 = time.perf_counter()
        Hs = production(ctx, L, lnW, a.pseed, a.burn, cps[-1], walkers=a.walkers, label=a.arm, checkpoints=cps)
        base = os.path.join(a.dir, "prod_%s_%d_%d" % (a.arm, a.seed, a.pseed))
        np.save(base + ".npy", Hs)
        meta = {"arm": a.arm, "seed": a.seed, "pseed": a.pseed, "walkers": a.walkers, "burn": a.burn,
                "checkpoints": cps, "seconds": round(time.perf_counter() - t0, 1)}
        json.dump(meta, open(base + ".json", "w"))
        print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
