#!/usr/bin/env python3
"""Throughput of the decorated-particle step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload two_stream|probe|landau_nonlinear]

One step = one pass of the whole hot path over the batch of particles: pending half-kick,
kinetic diagnostics, half-kick, drift, deposit, and the Poisson solve (run by the last
workgroup of the fused kernel).  Default workload: the two-stream instability, N = 2^20
decorated particles, Ng = 512, dt = 0.05, FP32 state with compensated deposition.

Prints ONE JSON line on stdout.  `value` = N * K / wall time of the K timed steps
(particle state resident in HBM, graph-replayed steps).  `roofline` times the fused kernel
alone with HIP events around each launch (direct launches on the library's stream, right
after the timed region) and divides its algorithmic bytes by that duration.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "decorated-particle updates/s (1 GPU, % HBM roofline); served p50/p99 step latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle per fused step: read Q, P, q*, p*, psi*; write Q, P, q*, p*
FUSED_BYTES = {"fp64": 72, "fp32c": 36, "fp32": 36, "fp32ts": 36}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_src_sha() -> str:
    p = os.path.join(ROOT, "paper_2605_21794_amd", "csrc", "vp_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(workload: str, n: int):
    """HBM bytes per fused-kernel launch from the committed rocprofv3 PMC summary, or None
    when there is none or the kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"pmc_k_fused_{workload}.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("kernel_src_sha") != kernel_src_sha() or rec.get("n") != n:
        return None
    return rec.get("traffic_bytes_per_launch")


def make_workload(name: str):
    import workloads as W
    if name == "two_stream":
        return W.two_stream(), "fp32c"
    if name == "probe":
        return W.two_stream(nx=8192, nv=8192), "fp32c"
    if name == "landau_nonlinear":
        return W.landau_nonlinear(), "fp32c"
    if name == "landau_linear":
        return W.landau_linear(), "fp64"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(state, w, budget_s: float, max_steps: int):
    """FP64 oracle steps on the same initial state until the time budget is spent."""
    import numpy as np
    import oracle as O
    st = tuple(np.asarray(state[k], dtype=np.float64).copy() for k in ("Q", "P", "qs", "ps", "psi"))
    fld = O.solve_field(st[0], st[3], st[4], w.L, w.ng)
    t0 = time.perf_counter()
    k = 0
    while k < max_steps:
        st, fld = O.step(st, fld, w.L, w.ng, w.dt)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": w.n * k / el, "unit": "decorated-particle updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{k} oracle.step calls (FP64 NumPy, single thread) on the full "
                      f"{w.name} state, N={w.n}, Ng={w.ng}, from t=0; {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="two_stream")
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not "
              "supported (instance sharding across GPUs is described in DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2605_21794_amd as vp

    w, prec = make_workload(args.workload)
    if args.precision:
        prec = args.precision
    log(f"workload {w.name}: N={w.n} Ng={w.ng} dt={w.dt} precision={prec}")
    t0 = time.perf_counter()
    state = w.state(np.float64 if prec == "fp64" else np.float32)
    log(f"initial state built in {time.perf_counter() - t0:.1f} s")

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()          # a non-null stream, so steps can be graph-captured
    torch.cuda.set_stream(stream)
    sim = vp.Simulation(state, w.L, w.ng, w.dt, prec, hist_cap=max(64, args.steps + args.warmup + 8))
    tuning_us = None
    if not args.no_tune:
        best, tuning_us = sim.tune(steps_per_trial=32)
        log(f"tuned launch shape {best} ({tuning_us:.2f} us/step)")
    tun = sim.get_tuning()

    sim.step(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")
    t_start = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log(f"timed {args.steps} steps in {elapsed * 1e3:.2f} ms")

    # per-launch timing of the fused kernel with HIP events on the library's stream
    sim.set_tuning(use_graph=0)
    ks = max(1, args.kernel_steps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(ks)]
    for a, b in evs:
        a.record(stream)
        sim.step(1)
        b.record(stream)
    torch.cuda.synchronize()
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    kern_avg_s = float(np.mean(kern_ms)) * 1e-3
    log(f"fused kernel: mean {kern_avg_s * 1e6:.2f} us over {ks} launches "
        f"(min {min(kern_ms) * 1e3:.2f} us)")
    sim.set_tuning(use_graph=tun["use_graph"])

    diag = sim.diagnostics(0, allow_nonfinite=True)
    finite = bool(np.isfinite(diag["H"]))
    n = w.n
    value = n * args.steps / elapsed
    bytes_per_launch = FUSED_BYTES[prec] * n
    achieved = bytes_per_launch / kern_avg_s / 1e9
    traffic = load_traffic(args.workload, n)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "decorated-particle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name, "n": n, "ng": w.ng, "L": w.L, "dt": w.dt,
            "precision": prec, "instances": 1, "launch": tun,
            "state_finite_after_run": finite, "t_end": diag["t"],
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_fused", "bytes_per_launch": bytes_per_launch,
            "kernel_us": kern_avg_s * 1e6,
        },
    }
    if not args.no_cpu:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(state, w, args.cpu_budget, 200)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
