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
KERNEL_SRC = os.path.join(ROOT, "paper_1709_04394_amd", "csrc", "k_tile2d.hip")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--tile-plan", default=None,
                   help="H,K,threads: use this launch shape instead of the autotuner's")
    p.add_argument("--copy-probe", action="store_true",
                   help="only run plain 1 GiB device-to-device copies (calibrates HBM byte counters)")
    return p.parse_args()


def measured_traffic(plan):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by what
    the counter reads for a plain copy of known size), or None when that
    summary was taken on another kernel source or launch shape."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if kv.get("kernel_source_sha256") != src or kv.get("tile_plan") != "%d,%d,%d" % tuple(plan):
        return None
    return 1024.0 * (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_scale"]) +
                     float(kv["write_kib_per_launch"]) * float(kv["write_scale"]))


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
    return {"value": flips / (el * 1e9), "unit": "spin flips/ns", "cores": threads, "kind": "oracle",
            "sample": "%d Metropolis sweeps (with per-sweep E, M) of one 4096^2 int8 lattice at beta_c, %.1f s"
                      % (n, el)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X; "
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
    # launch shape from the autotuner (results never depend on it)
    if a.tile_plan:
        H, K, T = (int(x) for x in a.tile_plan.split(","))
        ctx.set_tile_plan(g, H, K, T)
        plan = ctx.get_tile_plan(g)
    else:
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
