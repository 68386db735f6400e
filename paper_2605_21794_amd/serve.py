"""Serving loop: continuous batching of simulation jobs over the slots of one engine.

Jobs (an initial decorated-particle state, its domain, mesh, time step and a horizon in
steps) arrive over time.  The loop keeps every admitted job's particle and field state
resident on the device, and advances all of them with one fused launch per step (the
batched engine of libvp).  A job is admitted as soon as a slot is free and its device bytes
fit in the budget (first come, first served: a job that does not fit blocks the ones behind
it, so none waits forever).  It is retired, with its state at its last integer step, exactly
when it reaches its horizon, or as soon as the engine has frozen it because its state turned
non-finite (polled for all slots at once after every chunk), which frees its slot and bytes
for the queue.

    srv = Server(precision="fp32c", max_slots=64, budget_bytes=8 << 30)
    report = srv.run(jobs)     # jobs: list of Job, each with its arrival time in seconds

Reported: step latency (per job and step: the device clock between the history records of
two consecutive steps, which the first workgroup of each job writes during each fused launch;
a step that spans a scheduling decision includes the host's time there), job latency (arrival
to retirement, wall clock), admission wait, aggregate particle updates per second.  The
device work goes through a backend with the Engine interface, so the scheduling logic can be
exercised without a GPU (a backend without device records reports the mean device time of
each chunk of steps as its step latency instead).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    state: dict                 # arrays Q, P, qs, ps, psi (host or device)
    L: float
    ng: int
    dt: float
    horizon: int                # steps to run
    arrival: float = 0.0        # seconds after the start of the run
    solver: str = "scan"
    name: str = ""
    # filled in by the server
    admitted_at: float = None
    finished_at: float = None
    slot: int = None
    steps_done: int = 0
    step_time_s: float = 0.0    # device time of the engine steps this job took part in
    result: dict = None         # final diagnostics
    final_state: dict = None    # state at the horizon (device tensors)
    history: list = None        # per-step records 0 .. steps-1 (with keep_history)
    step_latency_s: list = None  # device time of each of the job's steps between records

    @property
    def n(self) -> int:
        return int(np.asarray(self.state["Q"]).size) if not hasattr(self.state["Q"], "numel") \
            else int(self.state["Q"].numel())


@dataclass
class Report:
    jobs: list
    wall_s: float
    updates: int
    step_latency_us: dict = field(default_factory=dict)
    job_latency_s: dict = field(default_factory=dict)
    admission_wait_s: dict = field(default_factory=dict)
    nonfinite_jobs: int = 0
    step_latency_source: str = "device records"

    @property
    def updates_per_s(self) -> float:
        return self.updates / self.wall_s if self.wall_s > 0 else 0.0

    def as_dict(self) -> dict:
        return {"jobs": len(self.jobs), "nonfinite_jobs": self.nonfinite_jobs,
                "wall_s": self.wall_s, "updates": self.updates,
                "updates_per_s": self.updates_per_s, "step_latency_us": self.step_latency_us,
                "step_latency_source": self.step_latency_source,
                "job_latency_s": self.job_latency_s, "admission_wait_s": self.admission_wait_s}


def _pcts(x) -> dict:
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return {"p50": None, "p99": None, "max": None}
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)),
            "max": float(x.max())}


def _weighted_pcts(x, w) -> dict:
    """Percentiles of samples x with integer weights w (a sample counted w times)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    if x.size == 0:
        return {"p50": None, "p99": None, "max": None}
    o = np.argsort(x)
    x, c = x[o], np.cumsum(w[o])
    def q(p):
        return float(x[np.searchsorted(c, p * c[-1], side="left")])
    return {"p50": q(0.5), "p99": q(0.99), "max": float(x[-1])}


class Server:
    """Continuous batching over an engine's slots.

    backend: an object with the Engine interface used here (max_slots, admit, retire, step,
    diagnostics, job_bytes, frozen_slots); by default a GPU Engine of the given precision.
    chunk: most steps advanced between scheduling decisions (fewer when a resident job
    reaches its horizon sooner).
    retire_nonfinite: retire a job the engine has frozen (non-finite state) after the chunk
    in which it froze, instead of holding its slot until its horizon.
    keep_history: keep each job's per-step records (job.history) when the backend has them.
    """

    def __init__(self, precision="fp32c", max_slots: int = 64, budget_bytes: int = None,
                 chunk: int = 33, backend=None, clock=time.perf_counter, keep_state=False,
                 retire_nonfinite: bool = True, keep_history: bool = False):
        self.backend = backend if backend is not None else GpuBackend(precision, max_slots)
        self.max_slots = int(self.backend.max_slots)
        self.budget = budget_bytes if budget_bytes is not None else self.backend.default_budget()
        self.chunk = int(chunk)
        self.clock = clock
        self.keep_state = keep_state
        self.retire_nonfinite = retire_nonfinite
        self.keep_history = keep_history
        # a backend with device records gives their stamps as one array (record_stamps) and,
        # for keep_history, the records themselves (records)
        self.device_records = hasattr(self.backend, "record_stamps")

    def run(self, jobs: list, sleep=time.sleep) -> Report:
        for j in jobs:
            if int(j.horizon) < 1:
                raise ValueError(f"job {j.name!r}: horizon must be at least one step")
        pending = sorted(jobs, key=lambda j: j.arrival)
        queue = []                       # arrived, not yet admitted (FIFO)
        resident = {}                    # slot -> job
        used_bytes = 0
        step_samples = []                # (seconds per step, weight = job-steps), per chunk
        record_samples = []              # seconds per step of a job, from device records
        t0 = self.clock()
        nxt = 0
        while nxt < len(pending) or queue or resident:
            now = self.clock() - t0
            while nxt < len(pending) and pending[nxt].arrival <= now:
                queue.append(pending[nxt])
                nxt += 1
            # admission: first come, first served, by slot and byte budget
            while queue:
                job = queue[0]
                need = self.backend.job_bytes(job)
                if need > self.budget:
                    raise ValueError(f"job {job.name!r} needs {need} bytes, more than the budget "
                                     f"{self.budget}")
                free = [s for s in range(self.max_slots) if s not in resident]
                if not free or used_bytes + need > self.budget:
                    break
                queue.pop(0)
                slot = free[0]
                self.backend.admit(slot, job)
                job.slot = slot
                job.admitted_at = self.clock() - t0
                resident[slot] = job
                used_bytes += need
            if not resident:
                if nxt < len(pending):   # idle until the next arrival
                    wait = pending[nxt].arrival - (self.clock() - t0)
                    if wait > 0:
                        sleep(wait)
                continue
            k = min(self.chunk, min(j.horizon - j.steps_done for j in resident.values()))
            dev_s = self.backend.step(k)
            step_samples.append((dev_s / k, k * len(resident)))
            for j in resident.values():
                j.steps_done += k
                j.step_time_s += dev_s
            frozen = self.backend.frozen_slots() if self.retire_nonfinite else set()
            for slot in [s for s, j in resident.items() if j.steps_done >= j.horizon or s in frozen]:
                job = resident.pop(slot)
                if self.device_records:
                    # records 0 .. done-1; the last of them is written at retirement (the
                    # others during the fused launch of the following step), so the stamps of
                    # records 0 .. done-2 bracket done-2 steps
                    done = min(job.steps_done, self.backend.frozen_step(slot))
                    st_s = self.backend.record_stamps(slot, done) if done > 0 else []
                    st_s = st_s[:max(0, done - 1)]
                    job.step_latency_s = list(np.diff(st_s)) if len(st_s) > 1 else []
                    record_samples.extend(job.step_latency_s)
                    if self.keep_history and hasattr(self.backend, "records"):
                        job.history = self.backend.records(slot, done) if done > 0 else []
                job.result = self.backend.diagnostics(slot)
                st = self.backend.retire(slot)
                job.final_state = st if self.keep_state else None
                job.finished_at = self.clock() - t0
                used_bytes -= self.backend.job_bytes(job)
        wall = self.clock() - t0
        # updates actually performed: an instance whose state turned non-finite is frozen by
        # the engine and stops at the step its diagnostics report
        updates = sum(j.n * min(j.horizon, int(j.result.get("step", j.horizon)))
                      for j in pending)
        rep = Report(jobs=list(pending), wall_s=wall, updates=updates)
        rep.nonfinite_jobs = sum(1 for j in pending if not j.result.get("finite", True))
        if self.device_records:
            rep.step_latency_us = _pcts([1e6 * v for v in record_samples])
        else:
            rep.step_latency_source = "chunk means"
            rep.step_latency_us = _weighted_pcts([1e6 * v for v, _ in step_samples],
                                                 [w for _, w in step_samples])
        rep.job_latency_s = _pcts([j.finished_at - j.arrival for j in pending])
        rep.admission_wait_s = _pcts([j.admitted_at - j.arrival for j in pending])
        return rep


class GpuBackend:
    """The Engine of libvp: every step of every resident job runs in the HIP kernels."""

    def __init__(self, precision: str, max_slots: int):
        import torch
        from . import Engine, make_config, workspace_bytes
        self._torch = torch
        self._make_config = make_config
        self._workspace_bytes = workspace_bytes
        self.stream = torch.cuda.Stream()
        self.engine = Engine(precision, max_slots=max_slots, stream=self.stream)
        self.max_slots = max_slots
        self.precision = precision
        self.elem = 8 if precision == "fp64" else 4
        self._ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        from . import wall_clock_hz
        self.clock_hz = wall_clock_hz()

    def default_budget(self) -> int:
        free, _ = self._torch.cuda.mem_get_info()
        return int(0.8 * free)

    def job_bytes(self, job: Job) -> int:
        cfg = self._make_config(job.n, job.ng, job.L, job.dt, self.precision,
                                hist_cap=max(1, job.horizon + 1), solver=job.solver)
        return 5 * job.n * self.elem + self._workspace_bytes(cfg)

    def admit(self, slot: int, job: Job):
        with self._torch.cuda.stream(self.stream):
            self.engine.admit(slot, job.state, job.L, job.ng, job.dt,
                              hist_cap=max(1, job.horizon + 1), solver=job.solver)

    def step(self, k: int) -> float:
        a, b = self._ev
        a.record(self.stream)
        self.engine.step(k)
        b.record(self.stream)
        b.synchronize()
        return a.elapsed_time(b) * 1e-3

    def diagnostics(self, slot: int) -> dict:
        return self.engine.diagnostics(slot, allow_nonfinite=True)

    def frozen_slots(self) -> set:
        return {s for s, (_, finite) in self.engine.slot_status().items() if not finite}

    def frozen_step(self, slot: int) -> int:
        """Steps the slot has taken (a frozen instance stops counting)."""
        return int(self.engine.slot_status()[slot][0])

    def record_stamps(self, slot: int, count: int):
        """The device clock stamps of records 0 .. count-1 of a slot, in seconds (one numpy
        array, read without building a record object per step)."""
        return self.engine.history_array(slot, 0, count, allow_nonfinite=True)["stamp"] / \
            self.clock_hz

    def records(self, slot: int, count: int) -> list:
        """Per-step records 0 .. count-1 of a slot, each with its stamp in seconds."""
        recs = self.engine.history(slot, 0, count, allow_nonfinite=True)
        for r in recs:
            r["stamp_s"] = r["stamp"] / self.clock_hz
        return recs

    def retire(self, slot: int) -> dict:
        return self.engine.retire(slot)
