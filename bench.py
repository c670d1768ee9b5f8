#!/usr/bin/env python3
"""Benchmark: lattice updates per second of the fused collide-and-stream
step on a synthetic four-directional braided unit cell, on one GPU.

One benchmark "step" is one lattice Boltzmann step over the whole cell,
including the FP64 check-step reductions at the production interval
(one observable evaluation every ``--check-every`` steps).  The line printed
by rank 0 carries the HBM roofline of the step kernel (achieved algorithmic
GB/s against MI355X's 8 TB/s) and the CPU oracle's throughput on a bounded
sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    # name: (n, precision, bytes per lattice update of the step kernel)
    "braid256_f32": (256, "f32", 57.0),
    "braid128_f32": (128, "f32", 57.0),
    "braid256_f64": (256, "f64", 113.0),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=4000)
    p.add_argument("--warmup", type=int, default=400)
    p.add_argument("--workload", default="braid256_f32", choices=sorted(WORKLOADS))
    p.add_argument("--check-every", type=int, default=200)
    p.add_argument("--launch", default="", help="vec,bx,by (default: autotune cache or built-in)")
    p.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1503_08718_amd", "tuned_launch.txt"))
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-steps", type=int, default=0, help="oracle steps on the full cell (0 = auto)")
    return p.parse_args()


def cpu_baseline(m, prec_bytes, sample_steps):
    """The oracle, as it is, on a bounded sample of the same cell."""
    import oracle

    o = oracle.from_medium(m)
    o.set_bc(0, 1.0, 0.0, (0, 0, 0))
    o.init()
    n = m.phase.size
    steps = sample_steps or max(2, int(round(2e9 / n)))  # ~10-30 s of CPU work
    o.step(1)  # first touch of the buffers
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": n * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps on the same {m.nx}x{m.ny}x{m.nz} braided cell "
                      f"(x gradient, periodic sides), OpenMP over z-planes"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 (a single cell is not sharded)"}))
        sys.exit(2)
    import torch

    import workloads
    from paper_1503_08718_amd import load
    from paper_1503_08718_amd.solver import Medium

    load()
    n, prec, bpl = WORKLOADS[args.workload]
    m = workloads.braid(n, n, n, 30.0, 0.5)
    g = Medium(m.phase, m.k, precision=prec, device="cuda:0")
    g.set_bc(0, 1.0, 0.0, ("periodic", "periodic", "periodic"))
    if args.launch:
        g.set_launch(*[int(v) for v in args.launch.split(",")])  # vec,bx,by[,nt]
    elif os.path.exists(args.tune_cache):
        g.load_tuned(args.tune_cache)
    g.init()
    K = args.check_every
    # warm-up: the same graphs the timed region replays
    g.solve(1e-30, "keff", args.warmup, check_every=K)
    torch.cuda.synchronize()
    # timed region: whole job = steps with a check every K steps; the kernel
    # time of the plain step is taken from hip events around plain steps
    t0 = time.perf_counter()
    r = g.solve(1e-30, "keff", args.warmup + args.steps, check_every=K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nodes = n ** 3
    mlups = nodes * args.steps / wall / 1e6
    # live kernel timing with hip events on the medium's stream (plain steps only)
    kt_steps = max(64, min(args.steps, 2000))
    ms = g.time_steps(kt_steps)
    kern_us = ms * 1e3 / kt_steps
    achieved = bpl * nodes / (kern_us * 1e-6) / 1e9
    line = {
        "metric": "MLUPS (lattice updates per second, millions) of the fused collide+stream step, with % of HBM peak",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {
            "workload": f"synthetic four-directional braided cell {n}^3, braiding angle 30 deg, yarn fraction 0.5, "
                        f"k_axial 10 / k_trans 1 / matrix 0.2, x gradient, periodic sides, {prec.upper()}",
            "nodes": nodes,
            "check_every": K,
            "launch": dict(zip(("vec", "bx", "by", "nt"), g.info()["launch"])),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": "k_step",
            "kernel_us": round(kern_us, 3),
            "bytes_per_update": bpl,
        },
        "keff_after": round(r["keff"], 6),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(m, bpl, args.cpu_sample_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
