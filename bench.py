#!/usr/bin/env python3
"""Throughput benchmark of the checkerboard sweep on one MI355X.

Workload (the paper's benchmark size, Sec. "Checkerboard scheme": L = 4096):
three 4096 x 4096 periodic 2D Ising lattices, int8 spins, hot start from seed
7, checkerboard Metropolis at beta in {0.40, beta_c, 0.50}, Philox4x32-10
randomness, (E, M) recorded after every sweep.  One step = one library call of
100 full sweeps of
each of the three lattices, including the per-sweep measurement; the default
100 steps are the 10^4 sweeps per temperature of that workload.

Prints one JSON line: spin flips per ns (attempted single-site updates per ns,
the inverse of the paper's t_flip), the roofline fraction of the dominant
kernel (algorithmic bytes 2 B per flip: each spin read once and written once
per sweep), and the CPU oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
BETAS = (0.40, BETA_C, 0.50)
L = 4096
SEED = 7
HBM_PEAK_GBS = 8000.0
BYTES_PER_FLIP = 2.0
SWEEPS_PER_STEP = 100
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tile2d_L4096x3_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "k_tile2d_L4096x3_valu.txt")
# integer VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD
# every 4 cycles (16 lanes per cycle), at 2.4 GHz
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
# the dominant kernel's source files, hashed together in this order
KERNEL_SRC = [os.path.join(ROOT, "paper_1709_04394_amd", "csrc", f) for f in ("k_tile2d.hip", "em_slots.hpp")]
MLP_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# bands of 16 rows, 4 sweeps per launch, 512 threads: the autotuner's usual
# pick on this workload (it alternates with 3 sweeps per launch within 1 %)
PROFILED_PLAN = "16,2,512"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--tile-plan", default=PROFILED_PLAN,
                   help="H,K,threads: the launch shape (default: the shape the committed counter summaries were "
                        "taken with)")
    p.add_argument("--tune", action="store_true", help="pick the launch shape with the autotuner instead")
    p.add_argument("--no-rows", action="store_true", help="skip the other hot-path rows' throughput lines")
    p.add_argument("--skip-rows", default="",
                   help="comma-separated rows to leave out: wl (the Wang-Landau run), mlp (the training graph, "
                        "which a counter-collecting profiler run does not survive)")
    p.add_argument("--muca", default="64",
                   help="comma-separated test sizes (of 64,96,128) of the learned-vs-plain multicanonical "
                        "comparison added to the line (default 64, about a minute; 128 takes many minutes)")
    p.add_argument("--no-muca", action="store_true", help="skip the multicanonical comparison")
    p.add_argument("--muca-prod", type=int, default=8000,
                   help="production sweeps per arm at L = 64 (16384 walkers), scaled by (L/64)^2 for larger L")
    p.add_argument("--copy-probe", action="store_true",
                   help="only run plain 1 GiB device-to-device copies (calibrates HBM byte counters)")
    return p.parse_args()


def measured_traffic(plan):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by what
    the counter reads for a plain copy of known size), or None when that
    summary was taken on another kernel source or launch shape."""
    kv = _kv_for_kernel(TRAFFIC_FILE, plan)
    if kv is None:
        return None
    return 1024.0 * (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_scale"]) +
                     float(kv["write_kib_per_launch"]) * float(kv["write_scale"]))


def _kv_for_kernel(path, plan):
    """key: value lines of a committed counter summary, or None when it was
    taken on another kernel source or launch shape."""
    import hashlib

    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    src = h.hexdigest()
    if kv.get("kernel_source_sha256") != src or kv.get("tile_plan") != "%d,%d,%d" % tuple(plan):
        return None
    return kv


def measured_valu(plan, launch_s):
    """VALU issue of the dominant kernel: wave64 VALU instructions per launch
    (SQ_INSTS_VALU from the committed counter summary) over the live average
    launch duration, against the chip's integer VALU issue peak."""
    kv = _kv_for_kernel(VALU_FILE, plan)
    if kv is None:
        return None
    n = float(kv["valu_insts_per_launch"])
    rate = n / launch_s
    return {"instructions_per_launch": n, "achieved": rate, "peak": VALU_PEAK_WAVE_INSTS,
            "unit": "wave64 VALU instructions/s", "frac": rate / VALU_PEAK_WAVE_INSTS,
            "note": "peak = 256 CUs x 4 SIMDs x one wave64 instruction per 4 cycles x 2.4 GHz; multi-cycle "
                    "instructions (64-bit multiplies in Philox) occupy a SIMD longer, so this undercounts issue"}


def _events_ms(torch, fn, reps):
    """Median event-timed duration of fn() on the current stream."""
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return sorted(out)[len(out) // 2]


def row_measurements(torch, mcs, ctx, dev, skip=()):
    """Throughput of the other hot-path rows on their workloads' shapes, each
    timed with events around library calls (inputs resident in HBM), with the
    algorithmic bytes that an unfused sweep moves: int8 2 B per flip (+3 B of
    couplings per site for the spin glass), MSC64 0.25 B per flip (1 bit in
    and out).  Short runs: these are throughput figures, not physics."""
    rows = {}
    HB = mcs.HEATBATH

    def sweep_row(name, geom, flips_per_sweep, bytes_per_flip, beta, rule, nsw, J=None, start=mcs.HOT, seed=11):
        lat = mcs.lattice_tensor(geom, dev)
        ctx.init(geom, lat, start, seed, 0)
        EM = torch.empty((nsw, geom.count * (64 if geom.layout == mcs.MSC64 else 1), 2), dtype=torch.int64,
                         device=dev)
        nb = ctx.sweep_workspace_bytes(geom)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if nb else None
        ctx.sweep(geom, lat, beta, seed, 1, rule=rule, J=J, EM=EM[:1], ws=ws)
        sweep0 = [1]

        def run():
            ctx.sweep(geom, lat, beta, seed, nsw, sweep0=sweep0[0], rule=rule, J=J, EM=EM, ws=ws)
            sweep0[0] += nsw

        ms = _events_ms(torch, run, 3)
        fpn = flips_per_sweep * nsw / (ms * 1e6)
        gbs = fpn * bytes_per_flip
        rows[name] = {"value": fpn, "unit": "spin flips/ns", "ms_per_sweep": ms / nsw,
                      "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": gbs / HBM_PEAK_GBS}}
        del lat, EM, ws

    g = mcs.make_geom(3, 256)
    sweep_row("3d_int8_heatbath_256", g, 256 ** 3, 2.0, 0.2216546, HB, 20)

    # the 3D workload's four runs in one call: beta in {0.2216546, 0.25}, each
    # from a cold and a hot start (seed 11), four tiles per CU instead of one
    g4 = mcs.make_geom(3, 256, count=4)
    g2 = mcs.make_geom(3, 256, count=2)
    lat4 = mcs.lattice_tensor(g4, dev)
    ctx.init(g2, lat4[:2], mcs.COLD, 11, 0)
    ctx.init(g2, lat4[2:], mcs.HOT, 11, 2)
    betas4 = [0.2216546, 0.25, 0.2216546, 0.25]
    ws4 = torch.empty(ctx.sweep_workspace_bytes(g4), dtype=torch.uint8, device=dev)
    EM4 = torch.empty((20, 4, 2), dtype=torch.int64, device=dev)
    ctx.sweep_betas(g4, lat4, betas4, 11, 2, rule=HB, EM=EM4[:2], ws=ws4)
    s4 = [2]

    def run4():
        ctx.sweep_betas(g4, lat4, betas4, 11, 20, sweep0=s4[0], rule=HB, EM=EM4, ws=ws4)
        s4[0] += 20

    ms4 = _events_ms(torch, run4, 3)
    fpn4 = 4 * 256 ** 3 * 20 / (ms4 * 1e6)
    rows["3d_int8_heatbath_256_x4"] = {"value": fpn4, "unit": "spin flips/ns", "ms_per_sweep": ms4 / 20,
                                       "roofline": {"bound": "hbm", "achieved": fpn4 * 2.0, "peak": HBM_PEAK_GBS,
                                                    "unit": "GB/s", "frac": fpn4 * 2.0 / HBM_PEAK_GBS}}
    del lat4, ws4, EM4
    g = mcs.make_geom(2, L, layout=mcs.MSC64, count=1)
    sweep_row("2d_msc64_4096", g, 64 * L * L, 0.25, BETA_C, mcs.METROPOLIS, 10, seed=7)
    g = mcs.make_geom(3, 256, layout=mcs.MSC64, count=1)
    sweep_row("3d_msc64_heatbath_256", g, 64 * 256 ** 3, 0.25, 0.2216546, HB, 5)
    g = mcs.make_geom(3, 32)
    J = torch.empty(3 * 32 ** 3, dtype=torch.int8, device=dev)
    ctx.couplings(g, J, 13)
    sweep_row("3d_ea_int8_32", g, 32 ** 3, 2.0 + 3.0, 1.0, mcs.METROPOLIS, 200, J=J, seed=13)

    # the spin glass 32^3 multi-spin coded across 4096 disorder realisations
    # (64 word lattices of 64), one random number per site shared by the coded
    # copies; realisation 0 has the single-realisation row's couplings
    gsg = mcs.make_geom(3, 32, layout=mcs.MSC64, count=64)
    wsg = mcs.lattice_tensor(gsg, dev)
    ctx.init(gsg, wsg, mcs.HOT, 13, 0)
    Jsg = torch.empty((64, 3 * gsg.N), dtype=torch.int64, device=dev)
    ctx.couplings_msc64(gsg, Jsg, 13, 0)
    nsg = 50
    EMsg = torch.empty((nsg, 64 * 64, 2), dtype=torch.int64, device=dev)
    ctx.sweep_sg_msc64(gsg, wsg, Jsg, 1.0, 13, 1, EM=EMsg[:1])
    ssg = [1]

    def run_sg():
        ctx.sweep_sg_msc64(gsg, wsg, Jsg, 1.0, 13, nsg, sweep0=ssg[0], EM=EMsg)
        ssg[0] += nsg

    ms = _events_ms(torch, run_sg, 3)
    fpn = 4096.0 * gsg.N * nsg / (ms * 1e6)
    # algorithmic bytes per spin update: the spin word (1 bit in, 1 out) and
    # the three coupling words of the site (3 bits) per realisation
    rows["3d_ea_sg_msc64_32_x4096realisations"] = {
        "value": fpn, "unit": "spin flips/ns", "ms_per_sweep": ms / nsg,
        "roofline": {"bound": "hbm", "achieved": fpn * 5.0 / 8.0, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": fpn * 5.0 / 8.0 / HBM_PEAK_GBS}}
    del wsg, Jsg, EMsg

    # double checkerboard with k hits per tile load (a different Markov chain,
    # the paper's fastest 2D variant): three 4096^2 lattices at beta_c (the
    # headline's size and count), tiles of 128 x 128, per-sweep E and M;
    # attempted updates per ns (k per site and sweep), each call includes
    # packing the lattices at its start and unpacking them at its end
    g1 = mcs.make_geom(2, L, count=3)
    lat1 = mcs.lattice_tensor(g1, dev)
    ctx.init(g1, lat1, mcs.HOT, SEED, 0)
    wsd = torch.empty(ctx.dcb_workspace_bytes(g1), dtype=torch.uint8, device=dev)
    for kh, nsw in ((1, 100), (10, 10), (100, 2)):
        EMd = torch.empty((nsw, 3, 2), dtype=torch.int64, device=dev)
        ctx.sweep_dcb(g1, lat1, BETA_C, SEED, 1, 128, kh, EM=EMd[:1], ws=wsd)
        sw0 = [1]

        def run_dcb():
            ctx.sweep_dcb(g1, lat1, BETA_C, SEED, nsw, 128, kh, sweep0=sw0[0], EM=EMd, ws=wsd)
            sw0[0] += nsw

        ms = _events_ms(torch, run_dcb, 3)
        fpn = 3.0 * L * L * kh * nsw / (ms * 1e6)
        # the kernel's own algorithmic bytes: the packed lattice read and
        # written once per sweep (2 bits per site), i.e. 0.25 / k B per
        # attempted update; far below HBM speed, the kernel is bound by VALU
        # issue at k >= 10 and by its per-launch latency at k = 1
        bpu = 0.25 / kh
        rows["dcb_4096x3_T128_k%d" % kh] = {"value": fpn, "unit": "spin flips/ns", "ms_per_sweep": ms / nsw,
                                          "hits": kh, "tile": 128,
                                          "roofline": {"bound": "hbm", "achieved": fpn * bpu, "peak": HBM_PEAK_GBS,
                                                       "unit": "GB/s", "frac": fpn * bpu / HBM_PEAK_GBS,
                                                       "bytes_per_update": bpu}}
    del lat1, wsd

    # population annealing: 4 populations x 16384 replicas, L in {16, 32, 64, 128},
    # 200 steps of theta = 10 sweeps (the whole anneal, one captured graph)
    import numpy as np

    Ls, R = [16, 32, 64, 128], 16384
    beta = np.arange(201) / 200.0
    pops = ctx.pa_population_tensors(Ls, R)
    nb = ctx.pa_workspace_bytes(Ls, R, 10, beta)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    import time as _t

    flips = 200 * 10 * R * sum(x * x for x in Ls)

    def anneal_twice():
        # the first call captures and instantiates the graph; the second,
        # identical call (a fresh anneal) launches the graph the context kept
        out = []
        for _ in range(2):
            t0 = _t.perf_counter()
            ctx.pa_anneal(Ls, R, 10, 17, beta, pops, step_first=1, nsteps=200, ws=ws)
            out.append(_t.perf_counter() - t0)
        return out

    el0, el = anneal_twice()
    rows["pa_4x16384_L16-128_200steps"] = {"value": flips / (el * 1e9), "unit": "spin flips/ns", "seconds": el,
                                           "seconds_first_call": el0,
                                           "groups": [ctx.get_pa_group(L) for L in Ls],
                                           "note": "whole blocking call: 200 steps, ln Z and histograms; the first "
                                                   "call also captures and instantiates the graph"}
    # the same anneal after timing replicas per workgroup on its first 20 steps
    t0 = _t.perf_counter()
    G = ctx.tune_pa(Ls, R, 10, 17, beta, pops, ws=ws)
    tune_s = _t.perf_counter() - t0
    el0, el = anneal_twice()
    rows["pa_4x16384_L16-128_200steps_tuned"] = {"value": flips / (el * 1e9), "unit": "spin flips/ns",
                                                 "seconds": el, "seconds_first_call": el0, "groups": G,
                                                 "tune_seconds": tune_s}
    for Lp in Ls:
        ctx.set_pa_group(Lp, 0)
    del pops, ws

    # parallel tempering: 128 independent sets (as for disorder realisations
    # or independent runs, the extra parallelism a GPU needs) of 32
    # temperatures (beta 0.35 .. 0.55 around beta_c) of 64 x 64 lattices, 10
    # sweeps per round, 200 rounds of sweeps and device exchanges in one
    # graph; the second, identical call (fresh start) launches the graph the
    # context kept
    Lp, nTp, nSp, thp, rdp = 64, 32, 128, 10, 200
    bp = [0.35 + 0.2 * i / (nTp - 1) for i in range(nTp)]
    wsp = torch.empty(ctx.pt_workspace_bytes(Lp, bp, nSp, thp, rdp), dtype=torch.uint8, device=dev)
    pt_times = []
    for _ in range(2):
        stp = ctx.pt_state(Lp, nTp, nSp, 23)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        ctx.pt_run(Lp, bp, thp, 23, stp, 0, rdp, record=True, ws=wsp)
        pt_times.append(_t.perf_counter() - t0)
    pflips = float(nSp * nTp) * Lp * Lp * thp * rdp
    acc_rate = stp["accepted"].sum(axis=0) / (nSp * (rdp / 2.0))
    rows["pt_2d_L64_32temps_x128sets_200rounds"] = {
        "value": pflips / (pt_times[1] * 1e9), "unit": "spin flips/ns", "seconds": pt_times[1],
        "seconds_first_call": pt_times[0], "group": ctx.get_pa_group(Lp),
        "exchange_acceptance_min_max": [float(acc_rate.min()), float(acc_rate.max())],
        "note": "whole blocking call: 200 rounds of 10 sweeps and an exchange, energies recorded per round; "
                "the first call also captures and instantiates the graph"}
    del wsp, stp

    # multicanonical walkers: 4096 walkers of 128 x 128, sequential updates
    Lm, Wm = 128, 4096
    spins, E = ctx.muca_start(Lm, Wm, 147)
    wsm = ctx.muca_workspace(Lm, Wm)
    H = torch.zeros(Lm * Lm // 2 + 1, dtype=torch.int64, device=dev)
    lnW = np.zeros(Lm * Lm // 2 + 1)
    ctx.muca_sweeps(Lm, spins, E, lnW, 147, 0, 1, 1, H, wsm)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    ctx.muca_sweeps(Lm, spins, E, lnW, 147, 1, 4, 1, H, wsm)
    torch.cuda.synchronize()
    el = _t.perf_counter() - t0
    rows["muca_4096_walkers_L128"] = {"value": Wm * Lm * Lm * 4 / (el * 1e9), "unit": "single-site updates/ns",
                                      "ms_per_sweep": el * 250.0}
    del spins, E, wsm, H

    # Wang-Landau in energy windows: the 64 x 64 torus's levels [-2N, 0] in
    # 64 windows of 40 levels overlapping by 8, 256 walkers per window (16384
    # walkers), ln f from 1 down to below 1e-6; the whole blocking run,
    # then its matched ln g against the exact one, and the sweeps' own rate
    if "wl" not in skip:
        rows.update(wl_row(torch, mcs, ctx, dev))

    if "mlp" in skip:
        return rows
    # MLP for initial weights: full-batch Adam epochs (hand-written forward,
    # backward and update kernels, replayed graph) on a training set shaped
    # like the one of converged weights at L = 16, 24, 32, 48 (here the smooth
    # synthetic ln W = -N h(k / 2N), h the binary entropy), then the
    # prediction of initial ln W at L = 128
    def synth_lnW(Lt):
        N = Lt * Lt
        x = np.arange(N // 2 + 1) / (2.0 * N)
        with np.errstate(divide="ignore", invalid="ignore"):
            h = -np.where(x > 0, x * np.log(np.maximum(x, 1e-300)), 0.0) - (1 - x) * np.log1p(-x)
        return -N * h

    X, Y = ctx.mlp_training_set({Lt: synth_lnW(Lt) for Lt in (16, 24, 32, 48)})
    Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    params = ctx.mlp_init(1)
    ctx.mlp_train(params, Xd, Yd, 500)
    torch.cuda.synchronize()
    epochs = 5000
    t0 = _t.perf_counter()
    ctx.mlp_train(params, Xd, Yd, epochs)
    torch.cuda.synchronize()
    el = _t.perf_counter() - t0
    n = int(Yd.numel())
    # 2 -> 64 -> 64 -> 1: forward 2 (2*64 + 64*64 + 64) flop per sample, backward
    # about twice that (input gradients of the first layer are not needed)
    flop = 3 * 2 * (2 * 64 + 64 * 64 + 64) * n * epochs
    t1 = _t.perf_counter()
    ctx.mlp_lnw_init(params, 128)
    el_pred = _t.perf_counter() - t1
    # the library is built without packed FP32 instructions, so the attainable
    # FP32 vector peak is the non-packed one: 256 CUs x 64 lanes x 2 flop (FMA)
    # x 2.4 GHz = 78.6 TFLOP/s (157.3 with packed FP32)
    rows["mlp_train_2-64-64-1"] = {"value": epochs / el, "unit": "epochs/s", "samples": n,
                                   "us_per_epoch": el / epochs * 1e6, "predict_L128_ms": el_pred * 1e3,
                                   "roofline": {"bound": "alu", "achieved": flop / el / 1e12, "peak": MLP_PEAK_TFLOPS,
                                                "unit": "TFLOP/s", "frac": flop / el / 1e12 / MLP_PEAK_TFLOPS},
                                   "note": "launch-bound: 4417 parameters, a few thousand samples per epoch; peak is "
                                           "FP32 vector without packed instructions (disabled in the build)"}
    return rows


def wl_windows(L, nwin, overlap=8):
    """nwin windows of equal width over the levels 0..N/2, consecutive ones
    sharing `overlap` levels (the last one ends at N/2)."""
    K = L * L // 2
    width = -(-(K + 1 + (nwin - 1) * overlap) // nwin)
    lo = [min(i * (width - overlap), K - width + 1) for i in range(nwin)]
    hi = [x + width - 1 for x in lo]
    hi[-1] = K
    return lo, hi


def wl_row(torch, mcs, ctx, dev, L=64, nwin=64, M=256, lnf_final=1e-6):
    import numpy as np

    lo, hi = wl_windows(L, nwin)
    ws = ctx.wl_workspace(L, lo, hi, M)
    last = [time.perf_counter()]
    t0 = time.perf_counter()

    def progress(_u, done, min_stage, sweep):
        now = time.perf_counter()
        if now - last[0] > 20:
            last[0] = now
            print("Wang-Landau L=%d: %d of %d windows done, lowest stage %d, sweep %d, %.0f s"
                  % (L, done, nwin, min_stage, sweep, now - t0), file=sys.stderr, flush=True)

    r = ctx.wl_run(L, lo, hi, M, 3, lnf_final, max_sweeps=200000, progress=progress, ws=ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ex = exact_lng(L)
    lse, best = lng_error(r["lng"], ex), lng_error_best_constant(r["lng"], ex)
    # the sweep rate: 20 sweeps of every window from the run's final states at
    # ln f = 2^-20 (estimates and counts from a fresh start, as in the run)
    W = nwin * M
    wmax = max(h - l for l, h in zip(lo, hi)) + 1
    G = torch.zeros((W, wmax), dtype=torch.int64, device=dev)
    H = torch.zeros((W, wmax), dtype=torch.int32, device=dev)
    fl = torch.zeros(W, dtype=torch.int32, device=dev)
    spins, E = r["spins"], r["E"]
    inc, act = [1 << 12] * nwin, [1] * nwin
    ctx.wl_sweeps(L, lo, hi, M, inc, act, 3, 1 << 40, 1, spins, E, G, H, fl, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.wl_sweeps(L, lo, hi, M, inc, act, 3, (1 << 40) + 1, 20, spins, E, G, H, fl, ws=ws)
    torch.cuda.synchronize()
    el_sw = time.perf_counter() - t1
    return {"wl_L64_64windows_x256walkers": {
        "value": el, "unit": "seconds to ln f < %g" % lnf_final, "converged": all(r["converged"]),
        "sweeps_per_window_max": int(max(r["sweeps"])), "sweeps_per_window_mean": float(np.mean(r["sweeps"])),
        "stages": int(min(r["stages"])), "max_abs_lng_error": lse, "max_abs_lng_error_best_constant": best,
        "sweep_rate": {"value": W * L * L * 20 / (el_sw * 1e9), "unit": "single-site updates/ns",
                       "ms_per_sweep": el_sw * 50.0},
        "windows": {"count": nwin, "levels": hi[0] - lo[0] + 1, "overlap": 8, "walkers_per_window": M}}}


def exact_lng(L):
    """Exact ln g over the window levels from the stored files (written by
    tests/golden/make_exact_lng.py from the oracle's exact density of states)."""
    import numpy as np

    return np.loadtxt(os.path.join(ROOT, "tests", "golden", "lng_L%d.txt" % L))


def lng_error(lng_est, lng_ex):
    """max |ln g_est - ln g_exact| over the window levels with states, after
    matching the two normalisations (log-sum-exp over those levels)."""
    import numpy as np

    m = np.isfinite(lng_ex)
    if not np.all(np.isfinite(lng_est[m])):
        return float("inf")
    a, b = lng_est[m], lng_ex[m]
    c = np.logaddexp.reduce(b) - np.logaddexp.reduce(a)
    return float(np.max(np.abs(a + c - b)))


def lng_error_best_constant(lng_est, lng_ex):
    """max |ln g_est + c - ln g_exact| over the window levels with states, for
    the best constant c (the method fixes ln g only up to a constant): half the
    spread of the differences."""
    import numpy as np

    m = np.isfinite(lng_ex)
    if not np.all(np.isfinite(lng_est[m])):
        return float("inf")
    d = lng_ex[m] - lng_est[m]
    return float((d.max() - d.min()) / 2)


def muca_comparison(torch, mcs, ctx, sizes, prod64):
    """Learned vs plain initial weights: train on the method's converged
    weights at L = 16, 24, 32, 48, compare the sweeps to a flat histogram
    (min/max >= 0.8) at the test sizes from the same seed, then the same
    production run in both arms (16384 walkers, stratified start, burn-in),
    scored against the exact g(E): max |ln g error| after log-sum-exp
    matching of the normalisations (the accuracy metric), and after the best
    additive constant."""
    import numpy as np  # noqa: F401

    from paper_1709_04394_amd import learned_muca as lm

    t0 = time.perf_counter()
    lnW_by_L, runs = lm.training_weights(ctx)
    train = {str(L): {"iterations": r["iterations"], "total_sweeps": r["total_sweeps"],
                      "seconds": round(r["seconds"], 2)} for L, r in runs.items()}
    params, log = lm.train_network(ctx, lnW_by_L)
    out = {"walkers": lm.WALKERS, "train_sizes": list(lm.TRAIN_L), "training_runs": train,
           "mlp": {"epochs": int(log.size), "loss_first": float(log[0]), "loss_last": float(log[-1])},
           "schedule": "hot walker starts thermalised by %d canonical sweeps at the initial weights' -dlnW/dE "
                       "(16 groups; flat weights: none needed); iterations of 2 unrecorded + R recorded sweeps, "
                       "R = 10 doubled up to %s after every iteration that reached the whole window without "
                       "improving the previous flatness; flat = min/max >= 0.8"
                       % (lm.PREP_SWEEPS, {L: lm.REC_MAX[L] for L in sizes}), "sizes": {}}
    for L in sizes:
        c = lm.compare(ctx, L, params, prod_sweeps=0)
        ex = exact_lng(L)
        prod = prod64 * L * L // (64 * 64)
        burn = max(2000, prod // 4)
        row = {"production": {"walkers": 16384, "burn_in_sweeps": burn, "sweeps": prod}}
        for arm in ("plain", "learned"):
            r = c[arm]
            a = lm.arm_summary(r)
            tp = time.perf_counter()
            H = lm.production(ctx, L, r["lnW"], 1000 + L, burn, prod, walkers=16384, label=arm)
            lse, best = lm.lng_errors(H, r["lnW"], ex)
            a.update({"max_abs_lng_error": lse, "max_abs_lng_error_best_constant": best,
                      "production_seconds": round(time.perf_counter() - tp, 2)})
            row[arm] = a
        row["learned"]["fallback"] = bool(c["learned"]["fallback"])
        row["learned"]["initial_max_abs_lnW_error"] = lng_error(-c["lnW_init"], ex)
        pl, le = row["plain"], row["learned"]
        row["sweeps_ratio_learned_over_plain"] = (le["sweeps_per_walker_incl_prep"] / pl["sweeps_per_walker_incl_prep"]
                                                  if pl["converged"] and le["converged"] else None)
        out["sizes"][str(L)] = row
        print(json.dumps({"muca_progress": L, "row": row}), file=sys.stderr, flush=True)
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def copy_probe():
    """Five plain copies of 1 GiB between two device buffers: each reads and
    writes exactly 2^30 bytes, the yardstick for the FETCH_SIZE / WRITE_SIZE
    counters of the sweep kernel."""
    import torch

    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "copies": 5}))


def cpu_baseline(target_s):
    """The oracle (plain C, OpenMP over rows) on a bounded sample of the same
    workload: sweeps of one 4096^2 lattice at beta_c until ~target_s of work."""
    import numpy as np  # noqa: F401

    import oracle

    oracle.build()
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    s = oracle.init(2, L, oracle.HOT, SEED, 1)
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.sweep(2, L, s, BETA_C, SEED, 1, n, 1)
        n += 1
        el = time.perf_counter() - t0
        if el >= target_s or n >= 200:
            break
    flips = float(L) * L * n
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    out = {"value": flips / (el * 1e9), "unit": "spin flips/ns", "cores": threads, "kind": "oracle",
           "sample": "%d Metropolis sweeps (with per-sweep E, M) of one 4096^2 int8 lattice at beta_c, %.1f s"
                     % (n, el)}
    # the same oracle on one thread (OpenMP's thread count set in-process),
    # a few sweeps of the same lattice
    try:
        import ctypes

        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return out
    gomp.omp_set_num_threads(1)
    try:
        t0, m = time.perf_counter(), 0
        while True:
            oracle.sweep(2, L, s, BETA_C, SEED, 1, n + m, 1)
            m += 1
            el1 = time.perf_counter() - t0
            if el1 >= target_s / 3 or m >= 20:
                break
    finally:
        gomp.omp_set_num_threads(threads)
    out["single_thread"] = {"value": float(L) * L * m / (el1 * 1e9), "cores": 1,
                            "sample": "%d more sweeps of the same lattice, %.1f s" % (m, el1)}
    return out


def run_env(torch):
    """Where the line was measured: the device name, the HIP and torch versions
    and the host threads; an item that cannot be read is null."""
    env = {"gpu": None, "hip": getattr(torch.version, "hip", None), "torch": torch.__version__,
           "host_threads": len(os.sched_getaffinity(0))}
    try:
        if torch.cuda.is_available():
            env["gpu"] = torch.cuda.get_device_name(0)
    except RuntimeError:
        pass
    return env


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only (the workload is one MI355X's share); "
              "--gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        copy_probe()
        return
    import torch

    import paper_1709_04394_amd as mcs

    dev = torch.device("cuda", 0)
    ctx = mcs.Context(0)
    # the three temperatures run as three lattices of one batched call
    g = mcs.make_geom(2, L, count=3)
    lat = mcs.lattice_tensor(g, dev)
    ctx.init(g, lat, mcs.HOT, SEED, 0)
    nws = ctx.sweep_workspace_bytes(g)
    ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
    # launch shape: fixed, or from the autotuner (results never depend on it)
    if a.tune:
        sa, sb = mcs.lattice_tensor(g, dev), mcs.lattice_tensor(g, dev)
        plan = ctx.tune_sweep(g, sa, sb, BETA_C, sweeps=16)
        del sa, sb
    else:
        H, K, T = (int(x) for x in a.tile_plan.split(","))
        ctx.set_tile_plan(g, H, K, T)
        plan = ctx.get_tile_plan(g)
    SPS = SWEEPS_PER_STEP
    EM = torch.empty((a.steps, SPS, 3, 2), dtype=torch.int64, device=dev)
    EMw = torch.empty((SPS, 3, 2), dtype=torch.int64, device=dev)

    def step(t, em):
        ctx.sweep_betas(g, lat, BETAS, SEED, SPS, sweep0=t * SPS, replica0=0, EM=em, ws=ws)

    for t in range(a.warmup):
        step(t, EMw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for t in range(a.steps):
        step(a.warmup + t, EM[t])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    flips = 3.0 * L * L * SPS * a.steps
    value = flips / (ms * 1e6)

    # dominant kernel: the packed -> packed fused launch (K sweeps of the three
    # lattices with per-sweep E, M) that fills all but the first and last
    # launch of a call.  Its average duration is the slope between calls of
    # 2K and 22K sweeps (2 and 22 launches; both have the one int8 load and the
    # one int8 store), timed with events on the stream the launches run on, so
    # it includes the dispatch gap between back-to-back launches.
    H, K, T = plan
    EMk = torch.empty((22 * K, 3, 2), dtype=torch.int64, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def call_ms(n, sweep0):
        x, y = ev(), ev()
        x.record()
        ctx.sweep_betas(g, lat, BETAS, SEED, n, sweep0=sweep0, replica0=0, EM=EMk[:n], ws=ws)
        y.record()
        torch.cuda.synchronize()
        return x.elapsed_time(y)

    slopes = []
    sweep0 = (a.warmup + a.steps) * SPS
    for _ in range(7):
        t_short = call_ms(2 * K, sweep0)
        sweep0 += 2 * K
        t_long = call_ms(22 * K, sweep0)
        sweep0 += 22 * K
        slopes.append((t_long - t_short) / 20.0)
    launch_ms = sorted(slopes)[len(slopes) // 2]
    achieved = BYTES_PER_FLIP * 3 * L * L * K / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(plan)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_tile2d<%d,true>, packed rows in and out: %d sweeps of three 4096^2 lattices with "
                      "per-sweep E, M per launch" % (K, K),
            "avg_launch_us": launch_ms * 1e3, "tile_plan": {"H": H, "K": K, "threads": T},
            "algorithmic_bytes_per_launch": BYTES_PER_FLIP * 3 * L * L * K}
    valu = measured_valu(plan, launch_ms * 1e-3)

    out = {"metric": "spin flips/ns, % roofline (2D Ising L=4096); MUCA sweeps-to-flat learned/plain",
           "value": value, "unit": "spin flips/ns",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i8",
           "data": "synthetic: hot-start lattices from Philox seed 7",
           "config": {"workload": "2D Ising 4096x4096 periodic, int8 spins, checkerboard Metropolis, "
                                  "beta in {0.40, beta_c, 0.50}, per-sweep E and M",
                      "L": L, "lattices": 3, "betas": list(BETAS), "sweeps_per_step": SWEEPS_PER_STEP},
           "roofline": roof, "valu": valu}
    if not a.no_rows:
        out["rows"] = row_measurements(torch, mcs, ctx, dev, skip=[x for x in a.skip_rows.split(",") if x])
    if not a.no_muca and a.muca:
        out["muca"] = muca_comparison(torch, mcs, ctx, [int(x) for x in a.muca.split(",")], a.muca_prod)
        # the metric's second part: sweeps to a flat histogram, learned / plain
        out["muca_sweeps_to_flat_learned_over_plain"] = {
            str(L): r["sweeps_ratio_learned_over_plain"] for L, r in out["muca"]["sizes"].items()}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    out["env"] = run_env(torch)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
