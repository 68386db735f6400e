#!/usr/bin/env python3
"""Throughput of the decorated-particle step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload two_stream|probe|landau_nonlinear]
    python bench.py --workload landau_sweep      batched (256 uneven instances) vs plain
    python bench.py --workload served            continuous batching of a job stream
    python bench.py --workload sw_vs_pic         particle count against accuracy, decorated
                                                 particles against plain particle-in-cell
    python bench.py --workload cluster           k-means initialisation from markers
    python bench.py --launch 1024,8,1 --no-tune ...   fixed launch shape (threads, ppt, acc copies
                                                 [, persistent [, wave_reduce]])
    python bench.py --order lattice ...               lattice particle order instead of random
    python bench.py --copy-calibration                one device copy of a known size (for PMC scaling)
    python bench.py --pmc-summary F_DIR W_DIR COPY_F_DIR COPY_W_DIR --workload W --launch T,PPT,C[,1]

One step = one pass of the whole hot path over the batch of particles: the Poisson solve of
the previous deposit (every workgroup of the step kernel solves it), pending half-kick,
kinetic diagnostics, half-kick, drift, deposit.  --monopole runs the same workload as plain
particle-in-cell particles (p* = q* = 0, 20 bytes per update); --element-order 2 runs it
with P2 elements (the same 36 bytes per update, a load vector of 2 Ng nodes).  Default
workload: the two-stream instability, N = 2^20 decorated particles, Ng = 512, dt = 0.05,
FP32 state with compensated deposition.

Prints ONE JSON line on stdout.  `value` = N * K / wall time of the K timed steps
(particle state resident in HBM; graph-replayed fused launches, or persistent launches of
up to 1024 steps when the autotuner keeps that kernel).  `roofline` divides the step
kernel's algorithmic bytes per launch by its average launch duration, taken with HIP events
on the library's stream around the timed region.
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
MONOPOLE_BYTES = {"fp64": 40, "fp32c": 20, "fp32": 20, "fp32ts": 20}  # Q, P, psi* in; Q, P out
# particles with second moments: also read and write Mqq, Mqp, Mpp
MOMENT_BYTES = {"fp64": 120, "fp32c": 60, "fp32ts": 60}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def arith_dtype(prec: str) -> str:
    """The type the path computes in: float64 particle arithmetic and accumulation in every
    mode but the naive float32 one (the other float32 modes store float32 state only)."""
    return "f32" if prec == "fp32" else "f64"


# the files the kernels are compiled from (a counter reading belongs to their text)
KERNEL_SOURCES = ("vp_device.h", "vp_internal.h", "vp_kernels.hip", "vp_fused.hip",
                  "vp_persist.hip")


def code_tokens(text: str) -> str:
    """C/C++ source text with its comments removed and every run of whitespace made one
    space (string and character literals kept as written): what the compiler sees, so that
    an edit of comments or layout alone leaves a counter reading valid."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_src_sha() -> str:
    """Hash of the kernels' code (comments and layout left out)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2605_21794_amd", "csrc")
    for name in KERNEL_SOURCES:
        p = os.path.join(d, name)
        if os.path.exists(p):
            h.update(name.encode())
            h.update(code_tokens(open(p, encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def launch_key(tun: dict) -> list:
    """The launch shape a counter reading belongs to: threads, particles per thread, copies."""
    return [int(tun["threads"]), int(tun["ppt"]), int(tun["acc_copies"])]


def kernel_of(tun: dict) -> str:
    """The step kernel a tuning runs: the persistent one or one fused launch per step."""
    return "k_persist" if int(tun.get("persistent", 0)) else "k_fused"


def pmc_path(workload: str, launch: list, kernel: str = "k_fused") -> str:
    """Committed counter summary of a step kernel for one workload and launch shape."""
    t, p, c = launch
    return os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}_{t}x{p}x{c}.json")


def load_traffic(workload: str, n: int, precision: str, launch: list, kernel: str = "k_fused",
                 steps_per_launch: int = 1):
    """HBM bytes per launch of the step kernel from the committed rocprofv3 PMC summary, or
    None when there is none, when the kernel source changed since the counters were taken,
    or when this run's particle count, precision, launch shape or steps per launch is not
    the one they were taken at (the bytes scale with the storage type, the grid traffic
    with the shape, and a persistent launch's with its steps)."""
    p = pmc_path(workload, launch, kernel)
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if (rec.get("kernel_src_sha") != kernel_src_sha() or rec.get("n") != n
            or rec.get("precision") != precision or rec.get("launch") != list(launch)
            or rec.get("steps_per_launch", 1) != steps_per_launch):
        return None
    return rec.get("traffic_bytes_per_launch")


def _counter_rows(d: str):
    """Rows of every rocprofv3 counter_collection.csv under directory d."""
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def _per_dispatch(rows, counter: str, kernel_sub: str):
    """Mean over dispatches of kernels whose name contains kernel_sub of the counter (KiB)."""
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter or kernel_sub not in r["Kernel_Name"]:
            continue
        key = r["Dispatch_Id"]
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for kernels matching {kernel_sub!r}")
    vals = sorted(per.values())
    return sum(vals) / len(vals), len(vals)


COPY_BYTES = 1 << 30          # --copy-calibration copies this many bytes (reads and writes each)


def copy_calibration():
    import torch
    torch.cuda.set_device(0)
    n = COPY_BYTES // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {COPY_BYTES} bytes 3 times")


def base_workload(name: str) -> str:
    """The workload a bench line's name derives from (without its _p2 / _monopole suffixes)."""
    for suffix in ("_p2", "_monopole"):
        if name.endswith(suffix):
            name = name[:-len(suffix)]
    return name


def pmc_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, workload, precision, launch,
                kernel="k_fused", steps_per_launch=1):
    """Write profiles/pmc_<kernel>_<workload>_<shape>.json: FETCH_SIZE + WRITE_SIZE per launch,
    each scaled by the ratio of known bytes to what the same counter reads for a copy.
    `precision`, `launch` (threads, ppt, copies) and `steps_per_launch` (1 for k_fused; the
    steps of the one persistent launch of the counter runs for k_persist) name the counter
    runs' settings."""
    fetch_kib, nf = _per_dispatch(_counter_rows(fetch_dir), "FETCH_SIZE", kernel)
    write_kib, nw = _per_dispatch(_counter_rows(write_dir), "WRITE_SIZE", kernel)
    # the copy kernel is the largest dispatch in its run (torch launches a few small ones too)
    cf_rows = _counter_rows(cfetch_dir)
    cw_rows = _counter_rows(cwrite_dir)
    cf_kib = max(float(r["Counter_Value"]) for r in cf_rows if r["Counter_Name"] == "FETCH_SIZE")
    cw_kib = max(float(r["Counter_Value"]) for r in cw_rows if r["Counter_Name"] == "WRITE_SIZE")
    f_scale = COPY_BYTES / (cf_kib * 1024.0)
    w_scale = COPY_BYTES / (cw_kib * 1024.0)
    fetch_b = fetch_kib * 1024.0 * f_scale
    write_b = write_kib * 1024.0 * w_scale
    w, _ = make_workload(base_workload(workload))
    rec = {"kernel": kernel, "workload": workload, "n": w.n,
           "precision": precision, "launch": list(launch), "steps_per_launch": steps_per_launch,
           "kernel_src_sha": kernel_src_sha(),
           "fetch_kib_per_dispatch": fetch_kib, "write_kib_per_dispatch": write_kib,
           "dispatches": [nf, nw],
           "copy_bytes": COPY_BYTES, "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
           "traffic_bytes_per_launch": fetch_b + write_b,
           "traffic_bytes_per_particle": (fetch_b + write_b) / w.n,
           "traffic_bytes_per_update": (fetch_b + write_b) / (w.n * steps_per_launch)}
    out = pmc_path(workload, launch, kernel)
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def parse_launch(text: str) -> dict:
    """threads,ppt,acc_copies[,persistent[,wave_reduce]] -> tuning fields."""
    v = [int(x) for x in text.split(",")]
    out = {"threads": v[0], "ppt": v[1], "acc_copies": v[2]}
    if len(v) > 3:
        out["persistent"] = v[3]
    if len(v) > 4:
        out["wave_reduce"] = v[4]
    return out


def make_workload(name: str):
    import workloads as W
    if name == "two_stream":
        return W.two_stream(), "fp32c"
    if name == "probe":
        w = W.two_stream(nx=8192, nv=8192)
        w.name = "two_stream_probe"
        return w, "fp32c"
    if name == "landau_nonlinear":
        return W.landau_nonlinear(), "fp32c"
    if name == "landau_linear":
        return W.landau_linear(), "fp64"
    raise SystemExit(f"unknown workload {name}")


def run_sweep(args):
    """The uneven batched sweep (256 Landau instances): one fused launch per step for all
    instances (batched) against one launch per instance per step (plain), same kernels,
    same stream.  Prints one JSON line; `value` is the batched aggregate throughput."""
    import numpy as np
    import torch
    import paper_2605_21794_amd as vp
    import workloads as W
    prec = args.precision or "fp32c"
    ws = W.landau_sweep(n_inst=args.instances)
    dt_np = np.float64 if prec == "fp64" else np.float32
    sts = [w.state(dt_np) for w in ws]
    ntot = sum(w.n for w in ws)
    log(f"landau_sweep: {len(ws)} instances, sum N = {ntot}, precision {prec}")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    steps = args.steps

    # batched: one engine, one fused launch per step for every instance
    eng = vp.Engine(prec, max_slots=len(ws), stream=stream)
    for s, (w, st) in enumerate(zip(ws, sts)):
        eng.admit(s, st, w.L, w.ng, w.dt, hist_cap=max(64, steps + args.warmup + 8))
    if args.launch:
        eng.set_tuning(**parse_launch(args.launch))
    if not args.no_tune:
        best, us = eng.tune(steps_per_trial=99)
        log(f"batched: tuned launch shape {best} ({us:.2f} us/step)")
    tun = eng.get_tuning()
    eng.step(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    eng.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t0
    kern_avg_s = ev0.elapsed_time(ev1) * 1e-3 / steps
    log(f"batched: {steps} steps in {el_b * 1e3:.2f} ms ({kern_avg_s * 1e6:.2f} us per launch)")
    db = [eng.diagnostics(s, allow_nonfinite=True) for s in range(len(ws))]
    wb = [d["W"] for d in db]
    nonfinite = sum(1 for d in db if not d["finite"])
    # updates actually performed: an instance whose state went non-finite is frozen by the
    # engine, so it counts only the steps it took inside the timed region
    live = [min(steps, max(0, int(d["step"]) - args.warmup)) for d in db]
    upd_b = sum(w.n * k for w, k in zip(ws, live))
    eng.close()

    # plain: one engine per instance, one launch per instance per step (graph-replayed)
    sims = []
    for w, st in zip(ws, sts):
        sim = vp.Simulation(st, w.L, w.ng, w.dt, prec, stream=stream,
                            hist_cap=max(64, steps + args.warmup + 8))
        sim.set_tuning(threads=tun["threads"], ppt=tun["ppt"], acc_copies=tun["acc_copies"],
                       graph_steps=tun["graph_steps"])
        sims.append(sim)
    for sim in sims:
        sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    chunk = tun["graph_steps"]
    while done < steps:
        c = min(chunk, steps - done)
        for sim in sims:
            sim.step(c)
        done += c
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    log(f"plain: {steps} steps in {el_p * 1e3:.2f} ms")
    dp = [sim.diagnostics(0, allow_nonfinite=True) for sim in sims]
    wp = [d["W"] for d in dp]
    upd_p = sum(w.n * min(steps, max(0, int(d["step"]) - args.warmup)) for w, d in zip(ws, dp))
    rel = max((abs(a["W"] - b["W"]) / max(abs(b["W"]), 1e-300) for a, b in zip(db, dp)
               if a["finite"] and b["finite"]), default=None)   # None: no instance left finite
    for sim in sims:
        sim.close()

    value = upd_b / el_b
    # bytes of the updates actually performed (frozen instances move none), per launch
    bytes_per_launch = FUSED_BYTES[prec] * upd_b / steps
    achieved = bytes_per_launch / kern_avg_s / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "decorated-particle updates/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": el_b * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": arith_dtype(prec), "data": "synthetic",
        "config": {"workload": "landau_sweep", "instances": len(ws), "n_total": ntot,
                   "precision": prec, "launch": tun,
                   "plain_value": upd_p / el_p,
                   "batched_over_plain": (upd_b / el_b) / max(upd_p / el_p, 1e-300),
                   "max_rel_W_difference_batched_vs_plain": rel,
                   "nonfinite_instances": nonfinite},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_persist" if tun.get("persistent") else "k_fused",
                     "bytes_per_launch": bytes_per_launch,
                     "kernel_us": kern_avg_s * 1e6},
    }
    print(json.dumps(out), flush=True)


def served_block(prec: str, n_jobs: int = 32, slots: int = 64, chunk: int = 33,
                 load: float = 0.7) -> dict:
    """A short served stream for the default bench line: the first n_jobs of the seeded
    served recipe (Landau / two-stream / bump-on-tail, N = 2^U[12, 20], Ng 64..1024, horizons
    100-2000), continuously batched over one engine's slots on the whole device.  The
    engine's capacity is measured with every job arriving at t = 0; the same jobs then arrive
    as a Poisson stream at `load` times that capacity.  Step latency: per job and step, from
    the device clock stamps of consecutive history records."""
    import numpy as np
    import workloads as W
    from paper_2605_21794_amd.serve import Job, Server
    dt_np = np.float64 if prec == "fp64" else np.float32
    base = W.served_jobs(seed=0, n_jobs=n_jobs, rate=1.0)
    states = [w.state(dt_np) for _, w in base]

    def stream(rate):
        return [Job(state=st, L=w.L, ng=w.ng, dt=w.dt, horizon=w.nsteps,
                    arrival=(t / rate if rate else 0.0), name=w.name)
                for st, (t, w) in zip(states, base)]

    srv = Server(precision=prec, max_slots=slots, chunk=chunk)
    w0 = base[0][1]
    srv.run([Job(state=states[0], L=w0.L, ng=w0.ng, dt=w0.dt, horizon=66, name="warm")])
    sat = srv.run(stream(None))
    capacity = n_jobs / sat.wall_s
    rep = srv.run(stream(load * capacity))
    d = rep.as_dict()
    srv.backend.engine.close()
    log(f"served: capacity {capacity:.1f} jobs/s; at {load:g} x capacity {rep.updates_per_s:.3g} "
        f"updates/s, step p50/p99 {d['step_latency_us']['p50']:.1f}/"
        f"{d['step_latency_us']['p99']:.1f} us, job p50/p99 {d['job_latency_s']['p50']:.3f}/"
        f"{d['job_latency_s']['p99']:.3f} s")
    return {"workload": "served", "jobs": n_jobs, "slots": slots, "chunk": chunk,
            "precision": prec, "capacity_jobs_per_s": capacity,
            "saturated_updates_per_s": sat.updates_per_s, "load": load,
            "rate_jobs_per_s": load * capacity, "updates_per_s": rep.updates_per_s,
            "updates": rep.updates, "wall_s": rep.wall_s,
            "step_latency_us": d["step_latency_us"],
            "step_latency_source": d["step_latency_source"],
            "job_latency_s": d["job_latency_s"], "admission_wait_s": d["admission_wait_s"],
            "nonfinite_jobs": d["nonfinite_jobs"]}


def run_served(args):
    """Served request stream: seeded Poisson arrivals of mixed Landau / two-stream /
    bump-on-tail jobs, continuously batched over the slots of one engine.

    The engine's capacity is measured first (every job arriving at t = 0: jobs/s until the
    last one is done).  The stream is then replayed at arrival rates of the given fractions
    of that capacity, under a byte cap that forces queueing and under the whole device.
    Prints one JSON line: value = aggregate updates/s at the middle load on the whole device,
    with every run's updates/s and p50/p99 step latency, job latency and admission wait.
    (--rate R instead runs the stream once at R jobs/s.)"""
    import numpy as np
    import torch
    import workloads as W
    from paper_2605_21794_amd.serve import Job, Server
    prec = args.precision or "fp32c"
    dt_np = np.float64 if prec == "fp64" else np.float32
    base = W.served_jobs(seed=0, n_jobs=args.jobs, rate=1.0)  # arrival times at 1 job/s
    t0 = time.perf_counter()
    states = [w.state(dt_np) for _, w in base]
    work = sum(int(st["Q"].size) * w.nsteps for st, (_, w) in zip(states, base))
    log(f"served: {len(base)} jobs built in {time.perf_counter() - t0:.1f} s; "
        f"sum N*horizon = {work:.3g}")

    def stream(rate):
        """The same jobs; arrivals scaled to `rate` jobs/s (None: all at t = 0)."""
        return [Job(state=st, L=w.L, ng=w.ng, dt=w.dt, horizon=w.nsteps,
                    arrival=(t / rate if rate else 0.0), name=w.name)
                for st, (t, w) in zip(states, base)]

    torch.cuda.set_device(0)
    srv = Server(precision=prec, max_slots=args.slots, chunk=args.chunk)
    if args.launch:
        srv.backend.engine.set_tuning(**parse_launch(args.launch))
    if args.use_graph is not None:
        srv.backend.engine.set_tuning(use_graph=args.use_graph)
    log(f"served: engine tuning {srv.backend.engine.get_tuning()}")
    full_budget = srv.budget
    w0 = base[0][1]
    srv.run([Job(state=states[0], L=w0.L, ng=w0.ng, dt=w0.dt, horizon=66, name="warm")])

    def one(rate, budget, label):
        srv.budget = budget
        rep = srv.run(stream(rate))
        d = rep.as_dict()
        log(f"served [{label}]: wall {rep.wall_s:.3f} s, {rep.updates_per_s:.3g} updates/s, "
            f"step p50/p99 {d['step_latency_us']['p50']:.1f}/{d['step_latency_us']['p99']:.1f} us, "
            f"job p50/p99 {d['job_latency_s']['p50']:.3f}/{d['job_latency_s']['p99']:.3f} s, "
            f"wait p99 {d['admission_wait_s']['p99']:.3f} s, non-finite {d['nonfinite_jobs']}")
        return {"rate_jobs_per_s": rate, "budget_bytes": budget,
                "updates_per_s": rep.updates_per_s, "updates": rep.updates,
                "wall_s": rep.wall_s, "nonfinite_jobs": d["nonfinite_jobs"],
                "step_latency_us": d["step_latency_us"], "job_latency_s": d["job_latency_s"],
                "admission_wait_s": d["admission_wait_s"]}

    runs = []
    if args.rate:
        r = one(args.rate, int(args.budget_gib * (1 << 30)) if args.budget_gib else full_budget,
                f"{args.rate:g} jobs/s")
        runs.append(r)
        head, capacity = r, None
    else:
        sat = one(None, full_budget, "saturated")
        capacity = len(base) / sat["wall_s"]
        log(f"served: capacity {capacity:.1f} jobs/s ({sat['updates_per_s']:.3g} updates/s)")
        loads = [float(x) for x in args.loads.split(",")]
        # the largest job holds about 21.5 MB, and at these loads about 30 MB of the mix is
        # resident on average, so a cap of 32 MiB makes jobs queue for bytes where the whole
        # device never does
        cap_bytes = int((args.budget_gib or 1.0 / 32) * (1 << 30))
        head = None
        for budget, tag in ((cap_bytes, f"{cap_bytes / (1 << 30):g} GiB"), (full_budget, "device")):
            for f in loads:
                r = one(f * capacity, budget, f"{f:g} x capacity, {tag}")
                r["load"] = f
                runs.append(r)
                if budget == full_budget and head is None and f >= 0.7 - 1e-9:
                    head = r
        head = head or runs[-1]
        runs.insert(0, dict(sat, load="saturated"))
    out = {
        "metric": METRIC, "value": head["updates_per_s"], "unit": "decorated-particle updates/s",
        "n_gpus": 1, "steps": None, "warmup": None, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": arith_dtype(prec), "data": "synthetic",
        "config": {"workload": "served", "jobs": len(base), "slots": args.slots,
                   "chunk": args.chunk, "precision": prec,
                   "rate_jobs_per_s": head["rate_jobs_per_s"],
                   "budget_bytes": head["budget_bytes"]},
        "served": {"capacity_jobs_per_s": capacity, "headline": head, "runs": runs},
    }
    print(json.dumps(out), flush=True)


def run_sw_vs_pic(args):
    """Particle count against accuracy, decorated particles against plain particle-in-cell
    (the paper's quantitative comparison, on synthetic inputs): strong Landau damping
    (L = 12, A = 0.5, Ng = 128, dt = 0.2), float64, every run in one engine (one fused
    launch per kind and step).

    Methods at N = 128 x nv particles: decorated lattice (nx = Ng columns, nv rows),
    monopole-only on the same lattice (quiet start), monopole-only random markers (the
    standard start), and decorated particles clustered from ten times as many random
    markers by the GPU k-means initialisation (the paper's Algorithm 1; the paper clusters
    1e5 markers into 1e4 decorated particles).  Reference: monopole-only lattice of 1024 x 2048 particles, with a
    decorated run of the same size beside it.  Error: relative L2 of E_amp(t) against the
    reference over t <= 10 and t <= 20.  Bytes per update: 36 (decorated) and 20
    (monopole-only) in float32 storage; degrees of freedom 5 and 3 per particle.
    --element-order 2 runs every instance, the references included, with P2 elements on 32
    elements (64 nodes; four lattice columns per element, which P2 needs); --ng sets the
    mesh."""
    import numpy as np
    import torch
    import paper_2605_21794_amd as vp
    import workloads as W
    steps = 100
    order = args.element_order
    ng = args.ng if args.ng > 0 else (128 if order == 1 else 32)
    nvs = [8, 16, 32, 64, 128, 256, 512, 1024]
    runs = [("reference_pic", W.landau_strong(nx=1024, nv=2048, ng=ng), "lattice", True),
            ("reference_sw", W.landau_strong(nx=1024, nv=2048, ng=ng), "lattice", False)]
    for nv in nvs:
        w = W.landau_strong(nx=128, nv=nv, ng=ng)
        runs += [(f"sw_{nv}", w, "lattice", False), (f"pic_lattice_{nv}", w, "lattice", True),
                 (f"pic_random_{nv}", w, "random", True), (f"sw_kmeans_{nv}", w, "kmeans", False)]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    eng = vp.Engine("fp64", max_slots=len(runs), stream=stream)
    t0 = time.perf_counter()
    cluster_s = 0.0
    counts = []                      # particles admitted per run (k-means may leave clusters empty)
    for s_, (name, w, init, mono) in enumerate(runs):
        if init == "random":
            st = W.random_markers(w, w.n, seed=s_)
        elif init == "kmeans":
            mk = W.random_markers(w, 10 * w.n, seed=s_)
            torch.cuda.synchronize()
            tc = time.perf_counter()
            st = vp.cluster_markers(mk["Q"], mk["P"], mk["psi"], w.n, w.L, iters=10, seed=s_)
            torch.cuda.synchronize()
            cluster_s += time.perf_counter() - tc
        else:
            st = w.state()
        eng.admit(s_, st, w.L, w.ng, w.dt, hist_cap=steps + 8, monopole_only=mono,
                  element_order=order)
        counts.append(int(st["Q"].shape[0]))
    log(f"sw_vs_pic: {len(runs)} runs admitted in {time.perf_counter() - t0:.1f} s")
    eng.set_tuning(threads=512, ppt=4, acc_copies=4, graph_steps=33)
    eng.step(steps)
    torch.cuda.synchronize()
    status = eng.slot_status()

    def e_amp(slot):
        stp, fin = status[slot]
        h = eng.history(slot, 0, min(stp, steps), allow_nonfinite=True)
        if fin and stp >= steps:
            h.append(eng.diagnostics(slot))
        return np.array([r["e_amp"] for r in h]), fin

    ref, _ = e_amp(0)
    windows = {"t<=10": 51, "t<=20": 101}

    def errors(e):
        out = {}
        for k, m in windows.items():
            out[k] = (float(np.linalg.norm(e[:m] - ref[:m]) / np.linalg.norm(ref[:m]))
                      if e.size >= m and np.all(np.isfinite(e[:m])) else None)
        return out

    rows = []
    sw_ref, _ = e_amp(1)
    for s_, (name, w, init, mono) in enumerate(runs[2:], start=2):
        e, fin = e_amp(s_)
        r = {"run": name, "n": counts[s_], "method": "pic" if mono else "sw",
             "init": init,
             "bytes_per_update_f32": 20 if mono else 36, "dofs": (3 if mono else 5) * counts[s_],
             "finite_to_end": bool(fin and e.size > steps), "steps_done": int(status[s_][0]),
             "error": errors(e)}
        rows.append(r)
        log(f"{name:16s} N={counts[s_]:7d} err t<=10 {r['error']['t<=10']}  t<=20 {r['error']['t<=20']}"
            f"  steps {r['steps_done']}")

    def n_for(method, init, win, target):
        """Smallest N of the sweep whose error is at or below target (None if none)."""
        for r in rows:
            if r["method"] == method and r["init"] == init:
                e = r["error"][win]
                if e is not None and e <= target:
                    return r["n"]
        return None

    targets = (0.05, 0.02, 0.01)
    summary = {win: {f"{t:g}": {"sw_lattice": n_for("sw", "lattice", win, t),
                                "sw_kmeans": n_for("sw", "kmeans", win, t),
                                "pic_lattice": n_for("pic", "lattice", win, t),
                                "pic_random": n_for("pic", "random", win, t)}
                     for t in targets} for win in windows}
    head = summary["t<=10"]["0.02"]
    ratio = (head["pic_random"] / head["sw_lattice"]
             if head["sw_lattice"] and head["pic_random"] else None)
    out = {"metric": "particles for 2% E_amp error over t <= 10: random-marker PIC / decorated",
           "value": ratio, "unit": "x", "n_gpus": 1, "steps": steps, "warmup": 0,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "landau_strong sw_vs_pic", "L": 12.0, "alpha": 0.5,
                      "ng": ng, "element_order": order, "dt": 0.2, "nx": 128, "nv": nvs,
                      "reference": "monopole-only lattice 1024 x 2048"},
           "sw_vs_pic": {"reference_sw_vs_pic": errors(sw_ref), "kmeans_seconds": cluster_s,
                         "particles_for_error": summary, "rows": rows}}
    eng.close()
    print(json.dumps(out), flush=True)


def run_cluster(args):
    """Time the initialisation from markers (Algorithm 1 on the GPU): M random markers of
    the strong Landau case into M / 10 decorated particles (the paper's ratio), 10 Lloyd
    iterations.  value = markers x (iterations + 1) / s; the CPU oracle is timed on a
    bounded sample (a fortieth of the markers and clusters, brute-force assignment).  The
    config also reports mini-batch k-means (20 batches of M / 8) against it: time and
    within-cluster sum of squares."""
    import numpy as np
    import torch
    import paper_2605_21794_amd as vp
    import workloads as W
    m = args.markers
    k = m // 10
    iters = 10
    w = W.landau_strong()
    mk = W.random_markers(w, m, seed=0)
    torch.cuda.set_device(0)
    q, p, wt = (torch.from_numpy(mk[f]).cuda() for f in ("Q", "P", "psi"))
    vp.cluster_markers(q, p, wt, k, w.L, iters=1, seed=1)      # warm the kernels
    # the starting markers are drawn before the timed calls (a host permutation of m)
    inits = [torch.randperm(m, generator=torch.Generator().manual_seed(rep))[:k]
             .to(torch.int32).cuda() for rep in range(3)]
    times = []
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dec = vp.cluster_markers(q, p, wt, k, w.L, iters=iters, init_idx=inits[rep])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    best = min(times)
    n_out = int(dec["Q"].shape[0])
    log(f"cluster: {m} markers -> {n_out} decorated particles, {iters} iterations: "
        f"{best * 1e3:.1f} ms (runs {[round(t * 1e3, 1) for t in times]})")
    def wcss(assign):
        """Within-cluster weighted sum of squares of an assignment (centres at the means)."""
        a = assign.cpu().numpy()
        x, v, ww = mk["Q"], mk["P"], mk["psi"]
        W_ = np.bincount(a, weights=ww, minlength=k)
        live = W_ > 0
        mq = np.zeros(k)
        mp = np.zeros(k)
        mq[live] = np.bincount(a, weights=ww * x, minlength=k)[live] / W_[live]
        mp[live] = np.bincount(a, weights=ww * v, minlength=k)[live] / W_[live]
        return float(np.sum(ww * ((x - mq[a]) ** 2 + (v - mp[a]) ** 2)))

    lloyd_wcss = wcss(vp.cluster_markers(q, p, wt, k, w.L, iters=iters, init_idx=inits[0],
                                         return_assign=True)["assign"])
    # mini-batch k-means (the paper's option for large runs): nbatch batches of m / 8
    # markers drawn with replacement, against the Lloyd run's time and clustering quality
    batch, nbatch = max(1, m // 8), 20
    bidx = torch.from_numpy(np.random.default_rng(5).integers(0, m, (nbatch, batch),
                                                               dtype=np.int32)).cuda()
    vp.cluster_markers(q, p, wt, k, w.L, init_idx=inits[0], batch_idx=bidx[:1])   # warm up
    mb_times = []
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mb = vp.cluster_markers(q, p, wt, k, w.L, init_idx=inits[0], batch_idx=bidx,
                                return_assign=True)
        torch.cuda.synchronize()
        mb_times.append(time.perf_counter() - t0)
    mb_wcss = wcss(mb["assign"])
    log(f"mini-batch: {nbatch} batches of {batch}: {min(mb_times) * 1e3:.1f} ms; "
        f"within-cluster sum of squares {mb_wcss:.6g} against {lloyd_wcss:.6g} for Lloyd")
    out = {"metric": "marker assignments per second (k-means initialisation)",
           "value": m * (iters + 1) / best, "unit": "marker-iterations/s", "n_gpus": 1,
           "steps": iters, "warmup": 1, "ms_per_step": best * 1e3 / (iters + 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "cluster", "markers": m, "clusters": k,
                      "decorated_out": n_out, "iterations": iters, "seconds": best,
                      "lloyd_wcss": lloyd_wcss,
                      "minibatch": {"batch": batch, "nbatch": nbatch,
                                    "seconds": min(mb_times), "wcss": mb_wcss,
                                    "wcss_over_lloyd": mb_wcss / lloyd_wcss,
                                    "decorated_out": int(mb["Q"].shape[0])}}}
    if not args.no_cpu:
        import oracle as O
        ms, ks = m // 40, k // 40
        sub = {f: mk[f][:ms] for f in ("Q", "P", "psi")}
        init = np.random.default_rng(0).choice(ms, ks, replace=False)
        t0 = time.perf_counter()
        O.cluster_markers(sub["Q"], sub["P"], sub["psi"], init, 2, w.L)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": ms * 3 / el, "unit": "marker-iterations/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"oracle k-means of {ms} markers into {ks} clusters, "
                                         f"2 iterations + final assignment and moments "
                                         f"(brute force), {el:.1f} s"}
    print(json.dumps(out), flush=True)


GOLDEN_LN = os.path.join(ROOT, "tests", "golden", "landau_nonlinear_oracle.npz")


def run_precision_study(args):
    """Nonlinear Landau damping (alpha = 0.5, k = 0.5, Ng = 256, N = 2^22, dt = 0.05) in every
    precision mode from the same FP32 input bits, against the stored FP64 oracle history
    (written by tests/golden/make_landau_nonlinear_history.py).  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2605_21794_amd as vp
    import workloads as W
    ref = np.load(GOLDEN_LN, allow_pickle=False)
    keys = [str(k) for k in ref["keys"]]
    H = ref["hist"]
    steps = min(args.steps, int(ref["steps"]))
    w = W.landau_nonlinear()
    st32 = w.state(np.float32)
    col = {k: H[:steps + 1, keys.index(k)] for k in keys}
    t = col["t"]
    windows = [("t<=10", t <= 10.0), ("10<t<=50", (t > 10.0) & (t <= 50.0)),
               ("50<t<=100", (t > 50.0) & (t <= 100.0))]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    modes = {}
    for prec in args.modes.split(","):
        st = {k: (v.astype(np.float64) if prec == "fp64" else v) for k, v in st32.items()}
        sim = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=steps + 8, stream=stream)
        if args.launch:
            sim.set_tuning(**parse_launch(args.launch))
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sim.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) * 1e-3
        hist = sim.history(0, 0, steps, allow_nonfinite=True) + [sim.diagnostics(0, grid=True, allow_nonfinite=True)]
        g = {k: np.array([h[k] for h in hist]) for k in ("W", "K", "H", "charge", "momentum")}
        grid_bt_sum = float(np.sum(hist[-1]["bt"]))
        rec = {"updates_per_s": w.n * steps / sec, "ms": sec * 1e3,
               "finite": bool(np.all(np.isfinite(g["W"])))}
        for name, m in windows:
            if m.any():
                rec[f"W_rel_l2[{name}]"] = float(np.linalg.norm(g["W"][m] - col["W"][m]) /
                                                 np.linalg.norm(col["W"][m]))
        rec["H_drift_max_rel"] = float(np.max(np.abs(g["H"] - g["H"][0])) / abs(g["H"][0]))
        rec["charge_drift_max"] = float(np.max(np.abs(g["charge"] - g["charge"][0])))
        rec["momentum_drift_max"] = float(np.max(np.abs(g["momentum"] - g["momentum"][0])))
        rec["sum_bt_over_charge"] = grid_bt_sum / float(g["charge"][0])
        modes[prec] = rec
        log(f"{prec}: {json.dumps(rec)}")
        sim.close()
    oracle = {"H_drift_max_rel": float(np.max(np.abs(col["H"] - col["H"][0])) / abs(col["H"][0])),
              "momentum_drift_max": float(np.max(np.abs(col["momentum"] - col["momentum"][0])))}
    head = "fp32c" if "fp32c" in modes else next(iter(modes))
    out = {"metric": METRIC, "value": modes[head]["updates_per_s"],
           "unit": "decorated-particle updates/s", "n_gpus": 1, "steps": steps, "warmup": 0,
           "ms_per_step": modes[head]["ms"] / steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": arith_dtype(head),
           "data": "synthetic", "config": {"workload": "landau_nonlinear", "n": w.n, "ng": w.ng, "dt": w.dt,
                      "study": "precision"},
           "precision_study": modes, "oracle": oracle}
    print(json.dumps(out), flush=True)


# algorithmic bytes per particle of the unfused kernels (FP32 state; FP64 doubles them)
DEPOSIT_BYTES = 12      # read Q, p*, psi*
GATHER_PUSH_BYTES = 32  # read Q, P, q*, p*; write Q, P, q*, p* (kick and drift)


def run_primitives(args):
    """The unfused kernels on their own: vp_deposit (load vector of the current state) and
    vp_gather_push (kick + drift), each timed with HIP events over many back-to-back calls.
    Prints one JSON line with each kernel's achieved GB/s against the HBM peak."""
    import numpy as np
    import torch
    import paper_2605_21794_amd as vp
    w, prec = make_workload(args.workload)
    if args.precision:
        prec = args.precision
    scale = 2 if prec == "fp64" else 1
    state = w.state(np.float64 if prec == "fp64" else np.float32)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    sim = vp.Simulation(state, w.L, w.ng, w.dt, prec)
    reps = max(1, args.steps // 10)
    res = {}
    # each kernel at its own launch shape (unless --launch fixes one for both): the deposit
    # reads 12 B per particle and pays a per-tile grid clear and flush, so it wants big tiles;
    # the push streams 32 B per particle and wants many small ones
    shapes = {"k_deposit": args.launch or "1024,16,4", "k_gather_push": args.launch or "1024,4,1"}
    for name, fn, nbytes in (("k_deposit", sim.deposit, DEPOSIT_BYTES * scale),
                             ("k_gather_push",
                              lambda: sim.gather_push(0.5 * w.dt, w.dt), GATHER_PUSH_BYTES * scale)):
        sim.set_tuning(**parse_launch(shapes[name]))
        for _ in range(3):
            fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / reps
        gbs = nbytes * w.n / (us * 1e-6) / 1e9
        res[name] = {"us_per_launch": us, "bytes_per_particle": nbytes, "achieved_GBs": gbs,
                     "frac": gbs / HBM_PEAK_GBS, "launch": shapes[name]}
        log(f"{name}: {us:.2f} us per launch, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f} of peak)")
    sim.close()
    print(json.dumps({"metric": METRIC, "config": {"workload": w.name, "n": w.n, "ng": w.ng,
                                                   "precision": prec, "launches": reps},
                      "primitives": res}), flush=True)


def cpu_baseline(state, w, budget_s: float, max_steps: int, order: int = 1,
                 moments: bool = False):
    """FP64 oracle steps on the same initial state until the time budget is spent (P2
    steps with order 2, k = 3 steps with moments)."""
    import numpy as np
    import oracle as O
    names = O.K3_FIELDS if moments else ("Q", "P", "qs", "ps", "psi")
    st = tuple(np.asarray(state[k], dtype=np.float64).copy() for k in names)
    if moments:
        fld = O.solve_field_p2_k3(st[0], st[3], st[4], st[5], w.L, w.ng)
        step, name = O.step_k3, "oracle.step_k3"
    elif order == 2:
        fld = O.solve_field_p2(st[0], st[3], st[4], w.L, w.ng)
        step, name = O.step_p2, "oracle.step_p2"
    else:
        fld = O.solve_field(st[0], st[3], st[4], w.L, w.ng)
        step, name = O.step, "oracle.step"
    t0 = time.perf_counter()
    k = 0
    while k < max_steps:
        st, fld = step(st, fld, w.L, w.ng, w.dt)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": w.n * k / el, "unit": "decorated-particle updates/s", "cores": 1,
            "host_cpu_count": os.cpu_count(), "kind": "oracle",
            "sample": f"{k} {name} calls (FP64 NumPy, single thread) on the full "
                      f"{w.name} state, N={w.n}, Ng={w.ng}, from t=0; {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 1000; 99 for landau_sweep, the span in which "
                         "every instance of the sweep is still valid)")
    ap.add_argument("--warmup", type=int, default=198,
                    help="untimed steps before the timed region (they also build the step "
                         "graph, so keep at least two graphs' worth)")
    ap.add_argument("--workload", default="two_stream")
    ap.add_argument("--kernel-steps", type=int, default=0,
                    help="after the timed region, also time this many direct (non-graph) "
                         "launches one by one with events (reported as direct_launch_us)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-served", action="store_true",
                    help="leave out the short served stream of the default line")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--instances", type=int, default=256, help="landau_sweep instances")
    ap.add_argument("--sort-every", type=int, default=0,
                    help="sort particles by cell every this many steps (0: never)")
    ap.add_argument("--sort-chunk", type=int, default=0, help="particles per sorted chunk")
    ap.add_argument("--order", default="random", choices=("random", "lattice"),
                    help="particle order in memory of the lattice workloads")
    ap.add_argument("--markers", type=int, default=1 << 22, help="cluster: markers")
    ap.add_argument("--monopole", action="store_true",
                    help="run the workload as monopole-only (plain particle-in-cell) particles")
    ap.add_argument("--moments", action="store_true",
                    help="particles with second moments (k = 3; P2 elements)")
    ap.add_argument("--element-order", type=int, default=1, choices=(1, 2),
                    help="2: P2 elements (vertex and midpoint nodes) in place of P1")
    ap.add_argument("--ng", type=int, default=0,
                    help="sw_vs_pic: mesh elements (default 128 for P1, 32 for P2)")
    ap.add_argument("--primitives", action="store_true",
                    help="time vp_deposit and vp_gather_push on their own")
    ap.add_argument("--modes", default="fp64,fp32c,fp32ts,fp32",
                    help="precision study: the modes to run, in order")
    ap.add_argument("--precision-study", action="store_true",
                    help="landau_nonlinear in every precision mode against the stored oracle")
    ap.add_argument("--jobs", type=int, default=128, help="served: jobs in the stream")
    ap.add_argument("--rate", type=float, default=None,
                    help="served: one run at this many arrivals per second (default: measure "
                         "capacity, then run at --loads of it)")
    ap.add_argument("--loads", default="0.5,0.7,0.9",
                    help="served: arrival rates as fractions of the measured capacity")
    ap.add_argument("--slots", type=int, default=64, help="served: engine slots")
    ap.add_argument("--chunk", type=int, default=33, help="served: steps between decisions")
    ap.add_argument("--use-graph", type=int, default=None, choices=(0, 1),
                    help="served: replay captured graphs (1) or launch directly (0)")
    ap.add_argument("--budget-gib", type=float, default=None,
                    help="served: device bytes cap (default: 1/32 GiB for the capped runs)")
    ap.add_argument("--launch", default=None,
                    help="threads,ppt,acc_copies[,persistent] of the fused step (with --no-tune)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--pmc-summary", nargs=4, default=None,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"))
    args = ap.parse_args()
    if args.moments:
        if args.monopole:
            raise SystemExit("--moments needs dipoles (not --monopole)")
        args.element_order = 2
    if args.steps is None:
        args.steps = 99 if args.workload == "landau_sweep" else 1000
    if args.pmc_summary:
        if not args.launch:
            raise SystemExit("--pmc-summary needs --launch: the shape the counter runs used")
        tun = parse_launch(args.launch)
        kern = kernel_of(tun)
        pmc_summary(*args.pmc_summary, args.workload, args.precision or "fp32c",
                    launch_key(tun), kern, args.steps if kern == "k_persist" else 1)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(whole instances would shard across GPUs with no exchange, and one large "
              "instance would all-reduce its Ng-long load vector once per step)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "landau_sweep":
        run_sweep(args)
        return
    if args.workload == "served":
        run_served(args)
        return
    if args.workload == "sw_vs_pic":
        run_sw_vs_pic(args)
        return
    if args.workload == "cluster":
        run_cluster(args)
        return
    if args.precision_study:
        run_precision_study(args)
        return
    if args.primitives:
        run_primitives(args)
        return

    import numpy as np
    import torch
    import paper_2605_21794_amd as vp

    w, prec = make_workload(args.workload)
    w.order = args.order
    if args.precision:
        prec = args.precision
    log(f"workload {w.name}: N={w.n} Ng={w.ng} dt={w.dt} precision={prec} order={w.order}")
    t0 = time.perf_counter()
    if args.moments and prec not in MOMENT_BYTES:
        raise SystemExit(f"--moments runs in {sorted(MOMENT_BYTES)}, not {prec}")
    state = w.state(np.float64 if prec == "fp64" else np.float32, moments=args.moments)
    if args.monopole:  # plain particle-in-cell: the same lattice without its dipole moments
        state["qs"][:] = 0
        state["ps"][:] = 0
    log(f"initial state built in {time.perf_counter() - t0:.1f} s")

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()          # a non-null stream, so steps can be graph-captured
    torch.cuda.set_stream(stream)
    sim = vp.Simulation(state, w.L, w.ng, w.dt, prec, hist_cap=max(64, args.steps + args.warmup + 8),
                        sort_every=args.sort_every, sort_chunk=args.sort_chunk,
                        monopole_only=args.monopole, element_order=args.element_order)
    tuning_us = None
    if args.launch:
        sim.set_tuning(**parse_launch(args.launch))
    if not args.no_tune:
        best, tuning_us = sim.tune(steps_per_trial=99)
        log(f"tuned launch shape {best} ({tuning_us:.2f} us/step)")
    tun = sim.get_tuning()
    persistent = bool(tun.get("persistent", 0))
    if not persistent and tun["use_graph"]:
        # a graph no longer than the timed steps (a multiple of the ring period of 3), and
        # every graph the timed steps replay captured now, outside the timed region
        gs = max(3, min(int(tun["graph_steps"]), 3 * (args.steps // 3)))
        if gs != tun["graph_steps"]:
            sim.set_tuning(graph_steps=gs)
        sim.prepare_step(args.steps)
        tun = sim.get_tuning()
    timed_launches = ("persistent launches" if persistent else
                      "graph replays" if tun["use_graph"] else "direct launches")

    sim.step(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")
    # HIP events on the library's stream bracket the timed region: with one launch per step
    # (graph replays back to back) elapsed / steps is the fused kernel's average launch
    # duration; a persistent launch runs up to 1024 steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    kern_avg_s = ev0.elapsed_time(ev1) * 1e-3 / args.steps
    log(f"timed {args.steps} steps in {elapsed * 1e3:.2f} ms; fused kernel "
        f"{kern_avg_s * 1e6:.2f} us per launch (events)")

    direct_us = None
    if args.kernel_steps > 0:
        sim.set_tuning(use_graph=0)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.kernel_steps)]
        for a, b in evs:
            a.record(stream)
            sim.step(1)
            b.record(stream)
        torch.cuda.synchronize()
        direct_us = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e3
        log(f"direct launches: {direct_us:.2f} us each between events")
        sim.set_tuning(use_graph=tun["use_graph"])

    diag = sim.diagnostics(0, allow_nonfinite=True)
    finite = bool(np.isfinite(diag["H"]))
    n = w.n
    value = n * args.steps / elapsed
    # the persistent kernel carries monopole-only particles through the decorated path
    table = (MOMENT_BYTES if args.moments else
             MONOPOLE_BYTES if args.monopole and not persistent else FUSED_BYTES)
    bytes_per_step = table[prec] * n
    # a launch is one step, or up to 1024 steps of the persistent kernel
    steps_per_launch = min(args.steps, 1024) if persistent else 1
    launches = -(-args.steps // steps_per_launch)
    bytes_per_launch = bytes_per_step * steps_per_launch
    launch_s = ev0.elapsed_time(ev1) * 1e-3 / launches
    achieved = bytes_per_launch / launch_s / 1e9
    # counters of the kernel that ran, at this run's shape (and, for the persistent kernel,
    # its steps per launch: its particles stay on chip between the steps of one launch)
    suffix = (("_monopole" if args.monopole else "") + ("_p2" if args.element_order == 2 else "")
              + ("_k3" if args.moments else ""))
    traffic_key = args.workload + suffix
    traffic = load_traffic(traffic_key, n, prec, launch_key(tun), kernel_of(tun),
                           steps_per_launch)
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
        "dtype": arith_dtype(prec),
        "data": "synthetic",
        "config": {
            "workload": w.name + suffix, "n": n, "ng": w.ng, "element_order": args.element_order,
            "L": w.L, "dt": w.dt,
            "precision": prec, "instances": 1, "launch": tun, "timed_launches": timed_launches,
            "sort_every": args.sort_every, "sort_chunk": args.sort_chunk, "order": args.order,
            "state_finite_after_run": finite, "t_end": diag["t"],
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_persist" if persistent else "k_fused",
            "bytes_per_launch": bytes_per_launch, "steps_per_launch": steps_per_launch,
            "kernel_us": launch_s * 1e6, "us_per_step": kern_avg_s * 1e6,
            "direct_launch_us": direct_us,
        },
    }
    if persistent:
        out["roofline"]["note"] = (
            "persistent kernel: each thread keeps its particles in registers for all the steps "
            "of a launch; achieved counts the algorithmic bytes per update, traffic the bytes "
            "the counters measured per launch")
    sim.close()
    if not args.no_served:
        out["served"] = served_block(prec)
    if not args.no_cpu:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(state, w, args.cpu_budget, 500, args.element_order,
                                           args.moments)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
    # explicit teardown while the HIP runtime and any attached profiler are alive: every
    # engine closed, the device idle (nothing of the library is left for interpreter shutdown)
    import paper_2605_21794_amd as _vp
    _vp.close_all()
