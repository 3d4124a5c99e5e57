"""Benchmark: FP64 Mcell-updates/s of the fused all-regime step on the 3D
Rayleigh-Benard workload (256^3, Ra = 1e6, Pr = 1, seeded 1e-4 temperature
noise, periodic x/y, no-slip fixed-T walls), with the HBM roofline of the
fused step kernel and the oracle timed on the host cores; beside it the
adjoint/forward time ratio (3D RB 128^3, Ra = 1e5, 200 steps, 16 revolve
slots) and the speedup of the batched launch over one launch sequence per
instance (512 2D RB instances, 500 steps each).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                  [--no-adjoint] [--no-batch]

Prints ONE JSON line.  Inputs are resident in HBM before every timed
region; the main timed region is K steps of ars_step (one fused kernel
launch per step, dt kept on the device) bracketed by synchronisations and
HIP events on the stream the kernels run on.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6  # MI355X dense FP64 matrix cores


def kernel_hash():
    h = hashlib.sha256()
    for f in ("ars_fused.hip", "ars_fused.h", "ars_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_1903_09043_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_counters():
    """The committed rocprofv3 counter summary of the fused step, if it was
    taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "fused_step_rb3d_256_counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d


def batch_counters():
    """The committed counter summary of the batched kernel, if taken on the
    current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "batch_rb2d_512_counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    h = hashlib.sha256()
    for f in ("ars_batch.hip", "ars_fused.h", "ars_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_1903_09043_amd", "csrc", f), "rb").read())
    return d if d.get("kernel_hash") == h.hexdigest()[:16] else None


def load_traffic(n_cells):
    """HBM bytes per launch of the fused step (FETCH_SIZE and WRITE_SIZE,
    scaled by a copy of known size) for the 256^3 workload."""
    d = load_counters()
    if d is None or n_cells != 256 ** 3:
        return None
    return d.get("bytes_per_launch")


def valu_view(ms_per_launch, n):
    """Instruction-issue view of the same kernel from the committed SQ
    counters (FP64 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T
    lane-ops/s): the balanced issue bound of the measured instruction count
    over the measured launch time."""
    d = load_counters()
    if d is None or "valu" not in d or n != 256:
        return None
    v = d["valu"]
    return {"valu_lane_instr_per_cell": v["valu_lane_instructions_per_cell"],
            "fp64_lane_instr_per_cell": v["fp64_lane_instructions_per_cell"],
            "valu_busy_frac": v["valu_busy_frac"], "issue_bound_ms": v["balanced_issue_bound_ms"],
            "issue_bound_frac": round(v["balanced_issue_bound_ms"] / ms_per_launch, 3)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_worker(budget_s):
    """Oracle steps of the 256^3 workload in this process (OpenMP threads as
    OMP_NUM_THREADS sets them); prints one JSON line."""
    import oracle as O
    from paper_1903_09043_amd import workloads as W
    cfg, prob, prm, seed = W.rb3d_ra1e6()
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
    print(json.dumps(dict(steps=steps, seconds=el, ncell=ncell, threads=O.num_threads())), flush=True)


def cpu_baseline(budget_s=12.0):
    """The oracle on the host cores, serial and with every core: each run in
    a child process (OpenMP fixes its thread count at start-up)."""
    import subprocess
    runs = {}
    for tag, env_threads in (("serial", "1"), ("threaded", None)):
        env = dict(os.environ)
        if env_threads:
            env["OMP_NUM_THREADS"] = env_threads
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(budget_s)], env=env,
                           capture_output=True, text=True, check=True)
        runs[tag] = json.loads(r.stdout.strip().splitlines()[-1])
    model = cpu_model()

    def fig(d):
        return dict(value=d["ncell"] * d["steps"] / d["seconds"] / 1e6, cores=d["threads"],
                    sample=f"{d['steps']} oracle step(s) of the same 256^3 workload ({d['ncell']} cells each), "
                           f"{d['seconds']:.1f} s on {d['threads']} host thread(s) of {os.cpu_count()} ({model})")

    thr, ser = fig(runs["threaded"]), fig(runs["serial"])
    out = dict(value=thr["value"], unit="Mcell-updates/s", cores=thr["cores"], kind="oracle", sample=thr["sample"],
               serial=dict(value=ser["value"], unit="Mcell-updates/s", cores=1, sample=ser["sample"]),
               cpu_model=model, host_cpus=os.cpu_count())
    return out


def timed(torch, fn, stream=None):
    """Milliseconds of fn() between HIP events on `stream` (default: the
    current stream), synchronised on both sides."""
    stream = stream or torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def spectrum_leg(torch, S, n, reps=20):
    """Kinetic-energy spectrum of the middle horizontal plane of the stepped
    state (ars_spectrum), off the step path.  A power-of-two plane takes the
    radix-2 FFT path (rows, then tiles of columns, in LDS), any other the
    dense DFT on the FP64 matrix cores.  Work counted as an FFT: 5 N log2 N
    flops per complex 2D transform of N points, 3 transforms, against the
    FP64 peak (vector and matrix: 78.6 TFLOP/s); for the dense path also the
    DFT it executes (4 flops per (kx, x) pair of the row transforms and 8
    per (ky, y) pair of the column transforms)."""
    import math
    S.spectrum()
    ms = timed(torch, lambda: [S.spectrum() for _ in range(reps)]) / reps
    fft = 3 * 5 * n * n * math.log2(n * n)
    pow2 = n & (n - 1) == 0
    out = {"plane": [n, n], "shells": int(S.spectrum().numel()), "ms_per_call": round(ms, 4),
           "path": "radix-2 FFT in LDS" if pow2 else "dense DFT on the FP64 matrix cores",
           "fft_equivalent_TFLOPs": round(fft / (ms * 1e-3) / 1e12, 4), "peak_TFLOPs": FP64_MFMA_PEAK_TFS}
    if not pow2:
        dense = 3 * n * n * (4 * n + 8 * n)
        out["dense_dft_TFLOPs"] = round(dense / (ms * 1e-3) / 1e12, 3)
        out["mfma_frac_of_executed_dense_dft"] = round(dense / (ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFS, 4)
    return out


def imex_leg(torch, A, W, n=1024, Ma=1e-3, expl_steps=5000, tol=1e-10):
    """Implicit acoustic (IMEX) steps against the explicit step on the low-
    Mach workload (Gresho vortex n^2, Mach 1e-3, theta on): the explicit
    step runs its 5000 CFL steps, the IMEX step reaches the same time with
    the transport + diffusive CFL step (dt_mode 2, CFL 0.4: about 440 times
    the acoustic one)."""
    cfg, prob, prm, seed = W.gresho(n=n, Ma=Ma, low_mach=1)
    A.Solver(cfg).init(prob, prm, seed).step(20)  # the explicit kernels loaded before the timed run
    E = A.Solver(cfg).init(prob, prm, seed)
    d0 = E.diagnostics()
    expl_ms = timed(torch, lambda: E.step(expl_steps))
    t_end = E.t.item()
    de = E.diagnostics()
    S2 = A.Solver(dict(cfg, dt_mode=2)).init(prob, prm, seed)
    dt_cfl = S2.dt.item()
    nst = max(1, int(np.ceil(t_end / dt_cfl)))
    sched = torch.full((nst,), t_end / nst, dtype=torch.float64, device="cuda")
    # one IMEX step on a scratch solver first: the timed run then finds its
    # kernels loaded, as the explicit run (timed after its own first steps
    # in the main leg) does
    A.Solver(cfg).init(prob, prm, seed).step_imex(sched[:1], tol=tol, max_iter=20000)
    S = A.Solver(cfg).init(prob, prm, seed)
    S.imex_workspace()  # allocated before the timed region, as the explicit run's buffers are
    its = {}

    def run_imex():
        its["n"] = S.step_imex(sched, tol=tol, max_iter=20000)
    imex_ms = timed(torch, run_imex)
    d = S.diagnostics()
    iters = its["n"]
    return {"workload": f"2D Gresho vortex {n}^2, Mach {Ma:g}, theta on, to t = {t_end:.6g}",
            "explicit_steps": expl_steps, "explicit_ms": round(expl_ms, 2),
            "imex_steps": nst, "imex_dt": t_end / nst, "acoustic_cfl": round(1.1 * (1.0 / Ma) * (t_end / nst) * n, 1),
            "solver_iterations": iters, "iterations_per_step": round(iters / nst, 1),
            "imex_ms": round(imex_ms, 2), "ms_per_iteration": round(imex_ms / max(iters, 1), 4),
            "speedup_vs_explicit": round(expl_ms / imex_ms, 3),
            "ke_ratio_imex": d["e_kin"] / d0["e_kin"], "ke_ratio_explicit": de["e_kin"] / d0["e_kin"],
            "mass_drift_imex": (d["mass"] - d0["mass"]) / d0["mass"],
            "energy_drift_imex": (d["e_total"] - d0["e_total"]) / d0["e_total"],
            "unknowns": 3 * n * n}


def recomputed_steps(A, n, s):
    """Forward steps the adjoint sweep recomputes: the plan's advances after
    its first adjoint step (its forward sweep before that is the forward
    run itself)."""
    from paper_1903_09043_amd.adjoint import OP_ADJOINT, OP_ADVANCE
    plan, _ = A.revolve_plan(n, s)
    first = next(i for i, (op, _, _) in enumerate(plan) if op == OP_ADJOINT)
    return sum(arg - step for op, step, arg in plan[first:] if op == OP_ADVANCE)


def adjoint_leg(torch, A, W, nsteps=200, slots=16, reps=10, end_to_end=True, k=20):
    """Adjoint/forward ratio on the 3D RB 128^3 workload: per step (k
    consecutive adjoint steps vs k consecutive fused steps at the same
    frozen dt, each sequence warm and timed as a whole, median of `reps`,
    divided by k: both sides carry their launches, neither a copy) and end
    to end (full gradient: forward, recomputation by the revolve plan and
    the adjoint sweep, over the forward run alone; the median of three
    calls after a first one, which is reported apart)."""
    from paper_1903_09043_amd.adjoint import RBProblem, rb_kinetic_energy
    cfg, prob, prm, seed = W.rb3d_ra1e5()
    pb = RBProblem(cfg, prob, prm, nsteps, slots)
    g = torch.Generator(device="cpu").manual_seed(1)
    dT = (1e-4 * (2 * torch.rand(pb.rho.shape, generator=g, dtype=torch.float64) - 1)).cuda()
    S = pb.solver(cfg["mu"], cfg["kappa"])
    S.U.copy_(pb.initial_state(dT))
    S.compute_dt()
    dt = S.dt.clone()
    lam = torch.randn(S.U.shape, generator=g, dtype=torch.float64).cuda()
    lam_n = torch.empty_like(lam)
    pg = torch.zeros(2, dtype=torch.float64, device="cuda")
    U0 = S.U.clone()
    dtk = dt.reshape(1).repeat(k).contiguous()  # k steps at the same dt (an even count: no copy back)

    def adjoint_k():
        for _ in range(k):
            S.step_adjoint(U0, lam, dt, lam_n=lam_n, param_grad=pg)
    adjoint_k()
    S.step_sched(dtk)
    fwd, adj = [], []
    for _ in range(reps):
        fwd.append(timed(torch, lambda: S.step_sched(dtk)) / k)
        adj.append(timed(torch, adjoint_k) / k)
    fwd.sort()
    adj.sort()
    f_ms, a_ms = fwd[reps // 2], adj[reps // 2]
    if not end_to_end:
        return {"step_ms_forward": round(f_ms, 4), "step_ms_adjoint": round(a_ms, 4),
                "ratio_per_step": round(a_ms / f_ms, 3)}
    # end to end
    mu = torch.tensor(cfg["mu"], dtype=torch.float64, requires_grad=True)
    ka = torch.tensor(cfg["kappa"], dtype=torch.float64, requires_grad=True)
    S.U.copy_(pb.initial_state(dT))
    S.compute_dt()
    fwd_ms = timed(torch, lambda: S.step(nsteps))
    x = dT.clone().requires_grad_()

    def grad():
        x.grad = mu.grad = ka.grad = None
        J = rb_kinetic_energy(x, mu, ka, pb)
        J.backward()
    # the first call also creates the solver and allocates the revolve
    # snapshots and the adjoint workspace; later calls reuse the cached blocks
    first_ms = timed(torch, grad)
    grad_ms = sorted(timed(torch, grad) for _ in range(3))[1]
    ok = bool(torch.isfinite(x.grad).all().item()) and mu.grad is not None
    g16 = (x.grad.clone(), mu.grad.clone(), ka.grad.clone())
    # the same gradient with every state kept (nsteps slots: 200 x 84 MB of
    # the 288 GB HBM), so nothing is recomputed
    pb_all = RBProblem(cfg, prob, prm, nsteps, nsteps)

    def grad_all():
        x.grad = mu.grad = ka.grad = None
        J = rb_kinetic_energy(x, mu, ka, pb_all)
        J.backward()
    grad_all()
    all_ms = sorted(timed(torch, grad_all) for _ in range(3))[1]
    same = bool(torch.equal(x.grad, g16[0]) and torch.equal(mu.grad, g16[1]) and torch.equal(ka.grad, g16[2]))
    del pb_all
    return {"workload": f"3D Rayleigh-Benard 128^3, Ra=1e5, Pr=1, {nsteps} steps, {slots} revolve slots, "
                        f"J = final kinetic energy, gradient w.r.t. dT0 (128^3 field), mu, kappa",
            "step_ms_forward": round(f_ms, 4), "step_ms_adjoint": round(a_ms, 4),
            "ratio_per_step": round(a_ms / f_ms, 3),
            "forward_run_ms": round(fwd_ms, 2), "gradient_ms": round(grad_ms, 2),
            "gradient_ms_first_call": round(first_ms, 2),
            "ratio_end_to_end": round(grad_ms / fwd_ms, 3),
            "plan_forward_steps": int(A.revolve_cost(nsteps, slots)),
            "recomputed_forward_steps": recomputed_steps(A, nsteps, slots), "gradient_finite": ok,
            "store_all": {"slots": nsteps, "snapshot_GB": round(nsteps * S.U.numel() * 8 / 1e9, 1),
                          "gradient_ms": round(all_ms, 2), "ratio_end_to_end": round(all_ms / fwd_ms, 3),
                          "bitwise_equal_to_16_slots": same}}


def small_configs_leg(torch, A, W):
    """Throughput of the two cache-resident single-problem workloads (no
    roofline claim: their states fit in L2 / MALL): 2D RB 64x32 for 1000
    steps (launch-bound) and the 2D Gresho vortex 1024^2 for 5000 steps with
    and without the low-Mach correction."""
    out = {}
    for name, (cfg, prob, prm, seed), n in (("rb2d_64x32", W.rb2d_64x32(), 1000),
                                           ("gresho_1024_theta_on", W.gresho_1024(low_mach=1), 5000),
                                           ("gresho_1024_theta_off", W.gresho_1024(low_mach=0), 5000)):
        S = A.Solver(cfg).init(prob, prm, seed)
        S.step(20)
        ms = timed(torch, lambda: S.step(n))
        cells = int(np.prod(cfg["n"]))
        out[name] = {"steps": n, "ms": round(ms, 2), "Mcell_per_s": round(cells * n / (ms * 1e-3) / 1e6, 1)}
        if name == "rb2d_64x32":
            # the same 1000 steps as ten replays of a captured 100-step graph
            g = S.capture(100)
            g.replay()
            torch.cuda.synchronize()

            def replay10():
                for _ in range(n // 100):
                    g.replay()
            msg = timed(torch, replay10)
            out[name + "_graph"] = {"steps": n, "ms": round(msg, 2),
                                    "Mcell_per_s": round(cells * n / (msg * 1e-3) / 1e6, 1)}
            del g
        del S
    return out


def batch_roofline(cell_updates, ms):
    """HBM view of the batched kernel: 64 algorithmic bytes per 2D cell
    update over the launch time.  The 512 states (235 MB, twice for the
    ping-pong) partly fit in the 256 MB MALL, so this is not an HBM-bound
    claim; traffic from the committed counters when they match the source."""
    achieved = cell_updates * 64 / (ms * 1e-3) / 1e9
    c = batch_counters()
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "cache_resident": "partly (235 MB x 2 vs 256 MB MALL)",
            "traffic": (c["read_bytes"] + c["write_bytes"]) if c else None,
            "valu_busy_frac": c["valu_busy_frac"] if c else None}


def batch_leg(torch, A, W, nsteps=500, loop=True):
    """Speedup of the batched persistent launch (graph-captured, one launch
    for all instances and steps) over the loop of ars_step(500) per
    instance on the same stream; every instance's final state must be
    bitwise equal between the two."""
    setups = W.rb2d_batch()
    cfgs = [c for c, *_ in setups]
    B = A.Batch(cfgs)
    for k, (cfg, prob, prm, seed) in enumerate(setups):
        U = A.Context(cfg).init_host(prob, prm, seed)
        B.view(k).copy_(torch.from_numpy(U))
    init = B.states.clone()
    tune = B.autotune(trial_steps=5)
    cells = sum(int(c["n"][0]) * int(c["n"][1]) for c in cfgs)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.capture(nsteps, s)
    torch.cuda.synchronize()
    batch_ms = timed(torch, lambda: B.replay(s), stream=s)
    _, _, fc, rc = B.read()
    rows, zc = B.tiling()
    if not loop:  # profiling the batched launch alone
        return {"batched_ms": round(batch_ms, 2), "cells": cells, "faults": int((fc >= 0).sum()), "rows": rows}
    # per-instance loop
    solvers = []
    for k, cfg in enumerate(cfgs):
        S = A.Solver(cfg)
        S.U.copy_(init[B.off[k]:B.off[k] + S.U.numel()].view(S.U.shape))
        S.compute_dt()
        solvers.append(S)

    def loop():
        for S in solvers:
            S.step(nsteps)
    loop_ms = timed(torch, loop)
    same = all(torch.equal(B.view(k), S.U) for k, S in enumerate(solvers))
    return {"workload": f"512 2D Rayleigh-Benard instances (64x32 / 128x64 / 256x128, Ra log-uniform "
                        f"[5e2, 5e3], Pr=1), {nsteps} steps each, per-instance CFL dt",
            "cells": cells, "cell_updates": cells * nsteps,
            "batched_ms": round(batch_ms, 2), "loop_ms": round(loop_ms, 2),
            "speedup": round(loop_ms / batch_ms, 3),
            "batched_Mcell_per_s": round(cells * nsteps / batch_ms / 1e3, 1),
            "loop_Mcell_per_s": round(cells * nsteps / loop_ms / 1e3, 1),
            "bitwise_equal": bool(same), "faults": int((fc >= 0).sum()),
            "roofline": batch_roofline(cells * nsteps, batch_ms),
            "tiling": {"rows": rows, "zc_policy": tune["zc_policy"], "tuner_candidates": tune["n_candidates"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-imex", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the cache-resident configs")
    ap.add_argument("--only", choices=["adjoint", "adjoint-step", "batch", "batch-kernel", "imex"], default=None,
                    help="run one side leg alone (profiling); prints its JSON object")
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--mode", choices=["step", "copy"], default="step",
                    help="copy: device-to-device copies of one state (calibrates the HBM byte counters)")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1903_09043_amd as A
    from paper_1903_09043_amd import workloads as W

    if args.only == "adjoint":
        print(json.dumps({"adjoint": adjoint_leg(torch, A, W)}), flush=True)
        return
    if args.only == "adjoint-step":
        print(json.dumps({"adjoint": adjoint_leg(torch, A, W, reps=5, end_to_end=False)}), flush=True)
        return
    if args.only == "batch":
        print(json.dumps({"batch": batch_leg(torch, A, W)}), flush=True)
        return
    if args.only == "imex":
        print(json.dumps({"imex": imex_leg(torch, A, W)}), flush=True)
        return
    if args.only == "batch-kernel":
        print(json.dumps({"batch": batch_leg(torch, A, W, loop=False)}), flush=True)
        return
    cfg, prob, prm, seed = W.rb3d_ra1e6(n=args.n)
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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "measured_hbm_GBps": round(traffic / launch_s / 1e9, 1) if traffic else None,
                     "valu_view": valu_view(ms / args.steps, args.n)},
        "final_state": {"t": S.t.item(), "max_u": d["max_u"], "fault": d["fault"]},
    }
    out["spectrum"] = spectrum_leg(torch, S, args.n)
    if not args.no_small:
        out["small_configs"] = small_configs_leg(torch, A, W)
    del S
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(torch, A, W)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batch"] = batch_leg(torch, A, W)
    if not args.no_imex:
        out["imex"] = imex_leg(torch, A, W)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
