#!/usr/bin/env python3
"""Benchmarks of the MI355X lattice Boltzmann conductivity solver (one GPU).

Default mode (the contract line): lattice updates per second of the fused
collide-and-stream step on a synthetic four-directional braided unit cell
(256^3, FP32).  One benchmark "step" is one lattice Boltzmann step over the
whole cell, including the FP64 check-step reductions at the production
interval (one observable evaluation every ``--check-every`` steps).  The line
carries the HBM roofline of the step kernel (algorithmic bytes per update /
kernel time, against MI355X's 8 TB/s) and the CPU oracle's throughput on a
bounded sample of the same workload.

Other modes (each prints one JSON line):
  --mode copy       a plain 1 GiB device copy, the calibration of HBM counters
  --mode solve      steady-state solves of one braided cell (k_T: x gradient,
                    k_L: z gradient), FP32 against an FP64 reference
  --mode sweep      the parametric sweep of braided cells of uneven size,
                    batched, to k_eff at 1e-4: unit cells per hour
  --mode warmstart  held-out cells solved from a zero start and from the
                    learned warm start: steps and cells per hour
  --mode paper      the paper's unit cell (Eqs. 32-37) over braiding angle
                    and fibre fraction: k_T, k_L, trends, periodic vs adiabatic
  --mode network    the warm-start network's BF16 matrix-core work: one
                    inference and one training iteration, TFLOP/s and
                    fraction of the dense BF16 peak
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
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak
TUNE_CACHE = os.path.join(ROOT, "paper_1503_08718_amd", "tuned_launch.txt")
WORKLOADS = {
    # name: (n, precision)
    "braid256_f32": (256, "f32"),
    "braid128_f32": (128, "f32"),
    "braid256_f64": (256, "f64"),
    "braid128_f64": (128, "f64"),
}
STORAGE_VALUES = {"populations": 7, "moments": 4}


def bytes_per_update(prec: str, storage: str) -> float:
    """Algorithmic HBM bytes of one lattice update: the state read and
    written once (7 populations or 4 moments) plus the phase byte."""
    return 2.0 * STORAGE_VALUES[storage] * (8 if prec == "f64" else 4) + 1.0
# HBM bytes per k_step launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# (KiB per dispatch, mean over the dispatches), each scaled by the counter's
# reading for a copy of known size (mrtlbm_stream_copy, 1 GiB); keyed by
# workload, storage and launch shape (vec, bx, by, nt, map).  Drop an entry
# whenever its kernel changes.
MEASURED_TRAFFIC = {
    ("braid256_f32", "moments", (4, 64, 4, 2, 1)): 563_201_378,
    ("braid256_f32", "populations", (4, 64, 2, 3, 0)): 956_425_998,
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=4000)
    p.add_argument("--warmup", type=int, default=400)
    p.add_argument("--mode", default="throughput",
                   choices=["throughput", "copy", "solve", "sweep", "warmstart", "paper", "network"])
    p.add_argument("--workload", default="braid256_f32", choices=sorted(WORKLOADS))
    p.add_argument("--check-every", type=int, default=200)
    p.add_argument("--storage", default="moments", choices=sorted(STORAGE_VALUES))
    p.add_argument("--launch", default="", help="vec,bx,by[,nt[,map]] (default: autotune cache, else built-in)")
    p.add_argument("--tune-cache", default=TUNE_CACHE)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-steps", type=int, default=0, help="oracle steps on the full cell (0 = auto)")
    # solve / sweep / warmstart
    p.add_argument("--n", type=int, default=128)
    p.add_argument("--gamma", type=float, default=30.0)
    p.add_argument("--vf", type=float, default=0.5)
    p.add_argument("--axes", default="0,2")
    p.add_argument("--sides", default="periodic", choices=["periodic", "adiabatic"])
    p.add_argument("--tol", type=float, default=1e-4)
    p.add_argument("--ref-tol", type=float, default=1e-7)
    p.add_argument("--no-ref", action="store_true")
    p.add_argument("--precision", default="", choices=["", "f32", "f64"], help="solve mode: one solve per axis")
    p.add_argument("--start", default="",
                   help="zero | linear | learned (solve mode, default zero); sweep and warmstart modes take a "
                        "comma list (defaults zero,learned and zero,linear,learned)")
    p.add_argument("--ref-only", action="store_true", help="sweep / warmstart: only the FP64 references")
    p.add_argument("--ref-cells", type=int, default=0, help="sweep mode: FP64 reference for the first K cells")
    p.add_argument("--ref-start", default="zero", choices=["zero", "linear"],
                   help="start of the FP64 reference solves (sweep and warmstart modes)")
    p.add_argument("--ref-out", default="", help="write the FP64 references to this JSON file")
    p.add_argument("--ref-in", default="", help="take the FP64 references from this JSON file instead of solving")
    p.add_argument("--max-steps", type=int, default=20_000_000)
    p.add_argument("--inference-grid", default="isotropic", choices=["isotropic", "cube"],
                   help="learned start: network grid with one coarsening factor on all axes, or always n^3")
    p.add_argument("--cells", type=int, default=64)
    p.add_argument("--seed", type=int, default=1503)
    p.add_argument("--model", default=os.path.join(ROOT, "paper_1503_08718_amd", "warmstart_model.pt"))
    return p.parse_args()


def _medium(m, prec, args):
    from paper_1503_08718_amd.solver import Medium

    g = Medium(m.phase, m.k, precision=prec, device="cuda:0", storage=args.storage)
    if args.launch:
        g.set_launch(*[int(v) for v in args.launch.split(",")])
    elif os.path.exists(args.tune_cache):
        g.load_tuned(args.tune_cache)
    return g


def host_cpu() -> dict:
    """What lscpu says about the host (model name, sockets, cores)."""
    import subprocess

    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "Vendor ID", "CPU family", "Model", "L3 cache"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        info["usable_cpus"] = len(os.sched_getaffinity(0))
    except OSError:
        pass
    return info


def cpu_baseline(m, sample_steps):
    """The oracle, as it is, on a bounded sample of the same cell: the same
    source built on this host with -O3 -march=native -ffp-contract=off
    -fopenmp (oracle.TIMING_FLAGS), all usable threads, then one thread."""
    import oracle

    o = oracle.Oracle(m.phase, m.k, timing=True)
    o.set_bc(0, 1.0, 0.0, (0, 0, 0))
    o.init()
    n = m.phase.size
    steps = sample_steps or max(2, int(round(5e9 / n)))  # ~10-30 s of CPU work on 16 cores
    o.step(1)  # first touch of the buffers
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    # and on one thread, over a few seconds' worth of steps
    o.set_threads(1)
    s1 = max(1, int(round(1.2e8 / n)))
    t0 = time.perf_counter()
    o.step(s1)
    dt1 = time.perf_counter() - t0
    cpu = host_cpu()
    return {"value": round(n * steps / dt / 1e6, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "single_thread_value": round(n * s1 / dt1 / 1e6, 2), "cpu_model": cpu.get("Model name", ""),
            "host": cpu, "build_flags": " ".join(oracle.TIMING_FLAGS),
            "sample": f"{steps} FP64 oracle steps on the same {m.nx}x{m.ny}x{m.nz} braided cell "
                      f"(x gradient, periodic sides), OpenMP over z-planes on {cores} threads; {s1} more steps "
                      f"on one thread for single_thread_value"}


def mode_throughput(args):
    import torch

    import workloads

    n, prec = WORKLOADS[args.workload]
    bpl = bytes_per_update(prec, args.storage)
    m = workloads.braid(n, n, n, 30.0, 0.5)
    g = _medium(m, prec, args)
    g.set_bc(0, 1.0, 0.0, ("periodic", "periodic", "periodic"))
    g.init()
    K = args.check_every
    # bring the GPU to its working clocks (a short timed region must not
    # start from idle), then start the state afresh
    g.time_steps(2000)
    g.init()
    # warm-up: the same graphs the timed region replays
    g.solve(1e-30, "keff", args.warmup, check_every=K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = g.solve(1e-30, "keff", args.warmup + args.steps, check_every=K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nodes = n ** 3
    mlups = nodes * args.steps / wall / 1e6
    # the step kernel's own time: hip events around 2000 plain steps on the
    # medium's stream, right after the timed region
    kt_steps = 2000
    ms = g.time_steps(kt_steps)
    kern_us = ms * 1e3 / kt_steps
    achieved = bpl * nodes / (kern_us * 1e-6) / 1e9
    launch = dict(zip(("vec", "bx", "by", "nt", "map"), g.info()["launch"]))
    traffic = MEASURED_TRAFFIC.get((args.workload, args.storage, tuple(launch.values())))
    line = {
        "metric": "MLUPS (million lattice updates per second) of the fused collide+stream step, with % of HBM peak",
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
            "state_storage": args.storage,
            "check_every": K,
            "launch": launch,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_vs_algorithmic": None if traffic is None else round(traffic / (bpl * nodes), 4),
            "kernel": "k_step",
            "kernel_us": round(kern_us, 3),
            "bytes_per_update": bpl,
            "algorithmic_bytes_per_launch": int(bpl * nodes),
        },
        "keff_after": round(r["keff"], 6),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(m, args.cpu_sample_steps)
    return line


def mode_copy(args):
    """HBM copy ceilings with the library's hand-written streaming copy
    (mrtlbm_stream_copy): 1 GiB read and 1 GiB written per copy, split over
    1, 2, 4 or 7 separate arrays (the step kernel streams 4 or 7 state
    arrays), plain and non-temporal loads/stores; hip events on the stream
    the copies run on."""
    import torch

    from paper_1503_08718_amd import _lib

    L = _lib.load()
    total = 1 << 30
    a = torch.ones(total // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    out = {"mode": "copy", "bytes_read_per_copy": total, "kernel": "k_stream_copy", "copies": []}
    reps = 20
    for streams in (1, 2, 4, 7):
        n16 = (total // 16) // streams
        for nt in (0, 1):
            def run():
                _lib.check(L.mrtlbm_stream_copy(a.data_ptr(), b.data_ptr(), n16, streams, nt, stream.cuda_stream))
            for _ in range(3):
                run()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                run()
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            moved = 2 * 16 * n16 * streams
            out["copies"].append({"arrays": streams, "nt": nt, "us": round(ms * 1e3, 2),
                                  "GB_s": round(moved / (ms * 1e-3) / 1e9, 1),
                                  "frac_of_peak": round(moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    return out


def mode_network(args):
    """The warm-start network on its 64^3 grid with seeded random weights and
    inputs: one inference (forward at batch 1 and 4) and one training
    iteration (forward, loss, input and weight gradients, Adam; batch 4),
    each timed with HIP events on the network's stream over repeated
    passes.  FLOPs are the algorithmic 2 * voxels * 27 * C_in * C_out per
    convolution pass."""
    import torch

    from paper_1503_08718_amd import warmstart as ws

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    def train_iter(net):
        net.forward()
        net.loss_and_grad()
        net.backward()
        net.adam()

    out = {"mode": "network", "grid": 64, "layers": len(ws.LAYERS), "peak_TFLOP_s": BF16_PEAK_TFLOPS,
           "data": "seeded random weights and inputs"}
    g = torch.Generator().manual_seed(args.seed)
    for batch in (1, 4):
        net = ws.Net(n=64, batch=batch, seed=0)
        net.act["x"].copy_(torch.rand(net.act["x"].shape, generator=g).to(torch.bfloat16))
        net.target.copy_(torch.rand(net.target.shape, generator=g) * 0.1)
        rec = {"batch": batch}
        ms = timed(net.forward, 20)
        f = ws.forward_flops(net)
        rec["forward"] = {"ms": round(ms, 4), "GFLOP": round(f / 1e9, 3), "TFLOP_s": round(f / ms / 1e9, 2),
                          "frac": round(f / ms / 1e9 / BF16_PEAK_TFLOPS, 4)}
        if batch == 4:
            ms = timed(lambda: train_iter(net), 10)
            f = ws.iteration_flops(net)
            rec["train_iteration"] = {"ms": round(ms, 4), "GFLOP": round(f / 1e9, 3),
                                      "TFLOP_s": round(f / ms / 1e9, 2),
                                      "frac": round(f / ms / 1e9 / BF16_PEAK_TFLOPS, 4)}
        out[f"batch{batch}"] = rec
        print(f"network batch {batch} done", file=sys.stderr, flush=True)
        del net
    return out


def _solve(m, prec, axis, sides, tol, args, T0=None, flux=False, start="zero", net=None, canonical=False):
    """One steady solve along axis.  The learned start (and canonical=True)
    solves the medium permuted so that the gradient runs along x; a given
    start field T0 must then be in that frame too."""
    import torch

    from paper_1503_08718_amd import warmstart

    mm = m
    swap = (0, 1, 2)
    if start == "learned" or canonical:
        # the network works on media whose gradient runs along x
        swap = {0: (0, 1, 2), 1: (1, 0, 2), 2: (2, 1, 0)}[axis]
        mm = m if axis == 0 else m.permuted(swap)
        axis = 0
    g = _medium(mm, prec, args)
    g.set_bc(axis, 1.0, 0.0, (sides,) * 3)
    t0 = time.perf_counter()
    if start == "learned":
        T, bad = warmstart.predict_start(net, mm, g)
        if bad:
            g.init()
        else:
            g.init(T.to(g.dtype), flux=True)
    elif start == "linear":
        shape = g.shape
        n = shape[2 - axis]
        lin = (1.0 - (torch.arange(n, dtype=torch.float64) + 0.5) / n).to(g.dtype)
        view = [1, 1, 1]
        view[2 - axis] = n
        g.init(lin.view(*view).expand(*shape).contiguous().to(g.device), flux=True)
    else:
        g.init(T0, flux=flux)
    torch.cuda.synchronize()
    r = g.solve(tol, "keff", args.max_steps, check_every=1000)
    torch.cuda.synchronize()
    r["seconds"] = round(time.perf_counter() - t0, 3)
    # flux column back in the cell's own axes (the exchange is its own inverse)
    r["keff_col"] = [r["keff_col"][swap[a]] for a in range(3)]
    return g, r


def mode_solve(args):
    """Steady solves of one braided cell.  Default: FP32 from --start, then an
    FP64 reference (tolerance --ref-tol) started from the FP32 field; with
    --precision the single requested solve (from --start) is run instead."""
    import workloads

    args.start = args.start or "zero"

    m = workloads.braid(args.n, args.n, args.n, args.gamma, args.vf)
    out = {"mode": "solve", "workload": f"braided cell {args.n}^3, gamma {args.gamma}, yarn fraction {args.vf}, "
                                        f"{args.sides} sides", "tol": args.tol, "solves": []}
    keys = ("keff", "keff_hot", "keff_cold", "keff_vol", "keff_col", "keff_leak", "steps", "seconds", "status")
    net = None
    if args.start == "learned":
        from paper_1503_08718_amd import warmstart

        net = warmstart.Net.from_file(args.model, batch=1)
    for axis in [int(a) for a in args.axes.split(",")]:
        if args.precision:
            g, r = _solve(m, args.precision, axis, args.sides, args.tol, args, start=args.start, net=net)
            rec = {"axis": "xyz"[axis], "precision": args.precision, "start": args.start,
                   "result": {k: r[k] for k in keys}, "MLUPS": round(m.phase.size * r["steps"] / r["seconds"] / 1e6, 1)}
        else:
            g32, r32 = _solve(m, "f32", axis, args.sides, args.tol, args, start=args.start, net=net)
            rec = {"axis": "xyz"[axis], "start": args.start, "f32": {k: r32[k] for k in keys}}
            if not args.no_ref:
                T = g32.temperature().double()
                g64, r64 = _solve(m, "f64", axis, args.sides, args.ref_tol, args, T0=T, flux=True,
                                  canonical=(args.start == "learned"))
                rec["f64_ref"] = {k: r64[k] for k in keys}
                rec["f32_rel_err"] = abs(r32["keff"] - r64["keff"]) / abs(r64["keff"])
                rec["f32_rel_err_vol"] = abs(r32["keff_vol"] - r64["keff_vol"]) / abs(r64["keff_vol"])
        out["solves"].append(rec)
        print(json.dumps(rec), flush=True)
    axes_done = [int(a) for a in args.axes.split(",")]
    if sorted(axes_done) == [0, 1, 2]:
        # full effective tensor: column a is the mean flux of the a-gradient solve
        import numpy as np

        K = np.zeros((3, 3))
        for a, rec in zip(axes_done, out["solves"]):
            r = rec["result"] if "result" in rec else rec["f32"]
            K[:, a] = r["keff_col"]
        out["tensor"] = K.tolist()
        out["tensor_asymmetry"] = float(np.abs(K - K.T).max() / np.abs(K).max())
        out["tensor_eigenvalues"] = np.linalg.eigvalsh(0.5 * (K + K.T)).tolist()
    return out


def mode_sweep(args):
    """The parametric sweep: braided cells of uneven size, angle and yarn
    fraction, x and z solves of every cell (z as the x solve of the cell with
    x and z exchanged) in one batched run per start, each to k_eff at --tol.
    Cells per hour count voxelisation, set-up (for the learned start: feature
    resampling, inference and interpolation) and the solves; training is a
    one-off and not counted; the batched step's shape is autotuned for the
    cell set inside the timed set-up.  With --ref-cells K the first K cells are also
    solved in FP64 to tol/100 and every start's error is reported on them."""
    import numpy as np
    import torch

    import workloads
    from paper_1503_08718_amd import warmstart as ws

    starts = [] if args.ref_only else [s for s in (args.start or "zero,learned").split(",") if s]
    t_start = time.perf_counter()
    specs = workloads.sweep_cells(args.seed, args.cells)
    media = ws.generate_media(specs)
    canon = [mm for m in media for mm in ws.canonical_media(m)]
    t_gen = time.perf_counter() - t_start
    net = ws.Net.from_file(args.model, batch=1) if "learned" in starts else None
    out = {"mode": "sweep", "cells": len(media), "solves_per_cell": 2, "tol": args.tol, "storage": args.storage,
           "inference_grid": args.inference_grid,
           "nodes_total": int(sum(m.phase.size for m in media)), "seconds_geometry": round(t_gen, 2),
           "sizes": [list(m.phase.shape[::-1]) for m in media]}
    ref = None
    if args.ref_in:
        with open(args.ref_in) as fh:
            saved = json.load(fh)
        if saved["cells"] < len(media) and args.ref_cells > saved["cells"]:
            raise SystemExit(f"{args.ref_in} holds references for {saved['cells']} cells")
        assert saved["seed"] == args.seed and saved["mode"] == "sweep", "reference file of another workload"
        ref = saved["keff"][:2 * (args.ref_cells or saved["cells"])]
        out["reference"] = {k: saved[k] for k in ("cells", "precision", "tol", "start", "all_converged", "seconds")}
        out["reference"]["file"] = os.path.basename(args.ref_in)
    elif args.ref_cells:
        sub = canon[:2 * args.ref_cells]
        t0 = time.perf_counter()
        _, rres, _, _ = ws.solve_fields(sub, tol=args.tol / 100, start=args.ref_start, net=net, batch=True,
                                        precision="f64", max_steps=args.max_steps, storage=args.storage,
                                        keep_fields=False, tune=True)
        ref = [r["keff"] for r in rres]
        out["reference"] = {"cells": args.ref_cells, "precision": "f64", "tol": args.tol / 100,
                            "start": args.ref_start, "all_converged": all(r["converged"] for r in rres),
                            "seconds": round(time.perf_counter() - t0, 1), "keff": ref,
                            "steps": [r["steps"] for r in rres]}
        if args.ref_out:
            with open(args.ref_out, "w") as fh:
                json.dump(dict(out["reference"], mode="sweep", seed=args.seed), fh)
        print(json.dumps({"reference": "done", "cells": args.ref_cells}), flush=True)
    for start in starts:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, res, setup, fb = ws.solve_fields(canon, tol=args.tol, start=start, net=net, batch=True,
                                            max_steps=args.max_steps, storage=args.storage, keep_fields=False,
                                            tune=True, grid=args.inference_grid)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        steps = [r["steps"] for r in res]
        lu = sum(m.phase.size * st for m, st in zip(canon, steps))
        rec = {"all_converged": all(r["converged"] for r in res), "fallbacks": fb,
               "seconds": round(wall, 2), "setup_seconds": round(setup, 2),
               "cells_per_hour": round(len(media) / ((t_gen + wall) / 3600.0), 1),
               "steps_mean": float(np.mean(steps)), "steps_min_max": [min(steps), max(steps)],
               "steps": steps,  # every solve, (x, z) per cell
               "effective_MLUPS": round(lu / max(wall - setup, 1e-9) / 1e6, 1),
               "k_T": [round(r["keff"], 6) for r in res[0::2]], "k_L": [round(r["keff"], 6) for r in res[1::2]]}
        if ref is not None:
            errs = [abs(r["keff"] - k) / abs(k) for r, k in zip(res, ref)]
            rec["max_rel_err_vs_reference"] = float(max(errs))
            rec["mean_rel_err_vs_reference"] = float(np.mean(errs))
            rec["rel_err_vs_reference"] = [float(f"{e:.3g}") for e in errs]  # every solve, (x, z) per cell
        out[start] = rec
        print(json.dumps({"start": start, "seconds": rec["seconds"], "steps_mean": rec["steps_mean"],
                          "cells_per_hour": rec["cells_per_hour"], "fallbacks": fb}), flush=True)
    return out


PAPER_TABLE3 = {  # interior braiding angle, fibre fraction -> (k_T, k_L), the paper's predictions (Table III)
    (25, 0.5): (0.639, 3.085), (25, 0.58): (0.727, 3.444), (40, 0.5): (1.015, 2.258), (40, 0.58): (1.160, 2.583)}


def paper_cells(angles, fractions, nxy=56):
    """The paper's unit cell dimensions (Eqs. 32-35) and yarn properties
    (Eqs. 36-37, epoxy 0.178, T300 7.81 / 0.675) on the synthetic braid."""
    import workloads

    cells = []
    for phi in fractions:
        lam_l, lam_t = workloads.yarn_conductivities(phi)
        for g in angles:
            geo = workloads.unit_cell_geometry(phi, g)
            nz = int(round(nxy * geo["h"] / geo["a"]))
            nz += nz % 2
            cells.append(dict(gamma=g, phi_f=phi, nx=nxy, ny=nxy, nz=nz, lam_l=lam_l, lam_t=lam_t,
                              a_mm=geo["a"], h_mm=geo["h"]))
    return cells


def mode_paper(args):
    """Fig. 9-style sweep: k_T (x gradient) and k_L (z gradient) of braided
    cells over interior braiding angle and fibre fraction, periodic sides,
    plus adiabatic sides at 25 deg (Sec. 5.2); all cells of one axis and side
    condition in one batched solve."""
    import torch

    import workloads
    from paper_1503_08718_amd.solver import batch_solve

    angles = [20, 25, 30, 35, 40, 45]
    fractions = [0.4, 0.5, 0.58]
    specs = paper_cells(angles, fractions)
    media = [workloads.braid(c["nx"], c["ny"], c["nz"], c["gamma"], workloads.PHI_Y_EXACT, c["lam_l"], c["lam_t"],
                             0.178) for c in specs]
    out = {"mode": "paper", "tol": args.tol, "cells": []}
    res = {}
    for sides in ("periodic", "adiabatic"):
        idx = range(len(specs)) if sides == "periodic" else [i for i, c in enumerate(specs) if c["gamma"] == 25]
        for axis in (0, 2):
            cells = []
            for i in idx:
                g = _medium(media[i], "f32", args)
                g.set_bc(axis, 1.0, 0.0, (sides,) * 3)
                g.init()
                cells.append(g)
            t0 = time.perf_counter()
            r, st = batch_solve(cells, tol=args.tol, kind="keff", max_steps=args.max_steps, check_every=1000)
            torch.cuda.synchronize()
            print(json.dumps({"sides": sides, "axis": "xyz"[axis], "status": st,
                              "seconds": round(time.perf_counter() - t0, 2)}), flush=True)
            for i, rr in zip(idx, r):
                res[(i, sides, axis)] = rr
    for i, c in enumerate(specs):
        rec = dict(c)
        rec["k_T"] = res[(i, "periodic", 0)]["keff"]
        rec["k_L"] = res[(i, "periodic", 2)]["keff"]
        if (i, "adiabatic", 0) in res:
            rec["k_T_adiabatic"] = res[(i, "adiabatic", 0)]["keff"]
            rec["k_L_adiabatic"] = res[(i, "adiabatic", 2)]["keff"]
        key = (c["gamma"], c["phi_f"])
        if key in PAPER_TABLE3:
            rec["paper_k_T"], rec["paper_k_L"] = PAPER_TABLE3[key]
        out["cells"].append(rec)
    kt = {(c["gamma"], c["phi_f"]): c["k_T"] for c in out["cells"]}
    kl = {(c["gamma"], c["phi_f"]): c["k_L"] for c in out["cells"]}
    out["trend_kT_rises_with_angle"] = all(kt[(a, f)] < kt[(b, f)] for f in fractions
                                           for a, b in zip(angles, angles[1:]))
    out["trend_kL_falls_with_angle"] = all(kl[(a, f)] > kl[(b, f)] for f in fractions
                                           for a, b in zip(angles, angles[1:]))
    out["trend_both_rise_with_fraction"] = all(kt[(a, f)] < kt[(a, g)] and kl[(a, f)] < kl[(a, g)]
                                               for a in angles for f, g in zip(fractions, fractions[1:]))
    out["periodic_above_adiabatic"] = all(c["k_T"] >= c["k_T_adiabatic"] and c["k_L"] >= c["k_L_adiabatic"]
                                          for c in out["cells"] if "k_T_adiabatic" in c)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 (a single cell is not sharded)"}))
        sys.exit(2)
    from paper_1503_08718_amd import load
    from paper_1503_08718_amd._lib import set_progress

    load()
    if args.mode != "throughput":
        set_progress(lambda msg: print(msg, file=sys.stderr, flush=True), 30.0)
    if args.mode == "throughput":
        line = mode_throughput(args)
    elif args.mode == "copy":
        line = mode_copy(args)
    elif args.mode == "solve":
        line = mode_solve(args)
    elif args.mode == "sweep":
        line = mode_sweep(args)
    elif args.mode == "paper":
        line = mode_paper(args)
    elif args.mode == "network":
        line = mode_network(args)
    else:
        from paper_1503_08718_amd import warmstart

        line = warmstart.bench(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
