#!/usr/bin/env python3
"""Throughput benchmark of the checkerboard sweep on one MI355X.

Workload (the paper's benchmark size, Sec. "Checkerboard scheme": L = 4096):
three 4096 x 4096 periodic 2D Ising lattices, int8 spins, hot start from seed
7, checkerboard Metropolis at beta in {0.40, beta_c, 0.50}, Philox4x32-10
randomness, (E, M) recorded after every sweep.  One step = sixteen full sweeps of
each of the three lattices, including the per-sweep measurement; the default
625 steps are the 10^4 sweeps per temperature of that workload.

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
SWEEPS_PER_STEP = 16


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=625)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    return p.parse_args()


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
    return {"value": flips / (el * 1e9), "unit": "spin flips/ns", "cores": threads, "kind": "oracle",
            "sample": "%d Metropolis sweeps (with per-sweep E, M) of one 4096^2 int8 lattice at beta_c, %.1f s"
                      % (n, el)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X; "
              "--gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
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
    # launch shape from the autotuner (results never depend on it)
    sa, sb = mcs.lattice_tensor(g, dev), mcs.lattice_tensor(g, dev)
    plan = ctx.tune_sweep(g, sa, sb, BETA_C, sweeps=16)
    del sa, sb
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

    # dominant kernel: the fused sweep launch (K sweeps of the three lattices,
    # no measurement), timed with events around pairs of launches on the
    # stream they run on
    H, K, T = plan
    npair = 100
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(npair)]
    torch.cuda.synchronize()
    for i in range(npair):
        evs[i][0].record()
        ctx.sweep_betas(g, lat, BETAS, SEED, 2 * K, sweep0=10 ** 7 + 2 * K * i, replica0=0, ws=ws)
        evs[i][1].record()
    torch.cuda.synchronize()
    launch_ms = sum(x.elapsed_time(y) for x, y in evs) / (2 * npair)
    achieved = BYTES_PER_FLIP * 3 * L * L * K / (launch_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_tile2d<%d,false>: %d sweeps of three 4096^2 int8 lattices per launch" % (K, K),
            "avg_launch_us": launch_ms * 1e3, "tile_plan": {"H": H, "K": K, "threads": T}}

    out = {"metric": "spin flips/ns, % roofline (2D Ising L=4096)", "value": value, "unit": "spin flips/ns",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i8",
           "data": "synthetic: hot-start lattices from Philox seed 7",
           "config": {"workload": "2D Ising 4096x4096 periodic, int8 spins, checkerboard Metropolis, "
                                  "beta in {0.40, beta_c, 0.50}, per-sweep E and M",
                      "L": L, "lattices": 3, "betas": list(BETAS), "sweeps_per_step": SWEEPS_PER_STEP},
           "roofline": roof}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
