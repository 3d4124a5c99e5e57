"""Benchmark: FP64 Mcell-updates/s of the fused all-regime step on the 3D
Rayleigh-Benard workload (256^3, Ra = 1e6, Pr = 1, seeded 1e-4 temperature
noise, periodic x/y, no-slip fixed-T walls), with the HBM roofline of the
fused step kernel and the oracle timed on the host cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints ONE JSON line.  Inputs are resident in HBM before the timed region;
the timed region is K steps of ars_step (one fused kernel launch per step,
dt kept on the device) bracketed by synchronisations and HIP events on the
stream the kernels run on.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def kernel_hash():
    h = hashlib.sha256()
    for f in ("ars_fused.hip", "ars_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_1903_09043_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(n_cells):
    """HBM bytes per launch of the fused step from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "fused_step_rb3d_256_counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(cfg, prob, prm, seed, budget_s=12.0):
    import numpy as np
    import oracle as O
    U = O.init(cfg, prob, prm, seed)
    ncell = 1
    for a in range(cfg["dim"]):
        ncell *= cfg["n"][a]
    steps = 0
    t0 = time.perf_counter()
    while True:
        dt = O.dt(cfg, U)
        U, rc, _ = O.step_dt(cfg, U, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50:
            break
    del U
    return dict(value=ncell * steps / el / 1e6, unit="Mcell-updates/s", cores=O.num_threads(), kind="oracle",
                sample=f"{steps} oracle step(s) of the same 256^3 workload ({ncell} cells each), "
                       f"{el:.1f} s on {O.num_threads()} host thread(s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--mode", choices=["step", "copy"], default="step",
                    help="copy: device-to-device copies of one state (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1903_09043_amd as A
    from paper_1903_09043_amd import workloads as W

    cfg, prob, prm, seed = W.config2(n=args.n)
    ncell = args.n ** 3
    if args.mode == "copy":
        # plain copy of one state (5 FP64 fields): reads and writes 40 B per cell
        a = torch.ones(5 * ncell, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"mode": "copy", "bytes_per_copy_each_way": a.numel() * 8,
                          "GBps_read_plus_write": 2 * a.numel() * 8 * args.steps / el / 1e9}), flush=True)
        return
    S = A.Solver(cfg).init(prob, prm, seed)
    if args.zchunk:
        S.ctx.set_zchunk(args.zchunk)
    stream = torch.cuda.current_stream()
    S.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    S.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = S.diagnostics()
    mcells = ncell * args.steps / (ms * 1e-3) / 1e6
    # dominant kernel: the fused step, one launch per step
    launch_s = ms * 1e-3 / args.steps
    alg_bytes = 2 * 5 * 8 * ncell  # read U^n + write U^{n+1}, 5 FP64 fields
    achieved = alg_bytes / launch_s / 1e9
    traffic = load_traffic(ncell)
    out = {
        "metric": "FP64 Mcell-updates/s (fused all-regime step, 3D RB 256^3)",
        "value": round(mcells, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D Rayleigh-Benard {args.n}^3, Ra=1e6, Pr=1, gamma=5/3, CFL 0.4, "
                               f"theta on, periodic x/y, no-slip fixed-T walls",
                   "cells": ncell, "zchunk": S.ctx.zchunk()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "final_state": {"t": S.t.item(), "max_u": d["max_u"], "fault": d["fault"]},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, prob, prm, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
