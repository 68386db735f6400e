"""Host logic of the serving loop, with a fake backend and a fake clock (no GPU)."""
import numpy as np
import pytest

from paper_2605_21794_amd.serve import Job, Server, _weighted_pcts


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Each step of k costs 1e-5 * k * (resident particles / 1000) seconds of fake time.
    A job named in `freeze_at` stops counting steps there, like an instance the engine has
    frozen because its state turned non-finite."""

    def __init__(self, clock, max_slots=3, freeze_at=None):
        self.clock = clock
        self.max_slots = max_slots
        self.resident = {}
        self.dev_step = {}
        self.freeze_at = dict(freeze_at or {})
        self.log = []
        self.peak_bytes = 0

    def default_budget(self):
        return 10 ** 9

    def job_bytes(self, job):
        return 100 * job.n

    def admit(self, slot, job):
        assert slot not in self.resident, "slot double-booked"
        self.resident[slot] = job
        self.dev_step[slot] = 0
        self.log.append(("admit", job.name, slot, self.clock()))
        self.peak_bytes = max(self.peak_bytes, sum(self.job_bytes(j) for j in self.resident.values()))

    def step(self, k):
        assert self.resident
        dt = 1e-5 * k * sum(j.n for j in self.resident.values()) / 1000.0
        self.clock.t += dt
        for s, j in self.resident.items():
            self.dev_step[s] = min(self.dev_step[s] + k, self.freeze_at.get(j.name, 1 << 60))
        return dt

    def _frozen(self, slot):
        return self.dev_step[slot] == self.freeze_at.get(self.resident[slot].name, -1)

    def frozen_slots(self):
        return {s for s in self.resident if self._frozen(s)}

    def diagnostics(self, slot):
        return {"step": self.dev_step[slot], "finite": not self._frozen(slot)}

    def retire(self, slot):
        job = self.resident.pop(slot)
        self.dev_step.pop(slot)
        self.log.append(("retire", job.name, slot, self.clock()))
        return {"Q": np.zeros(job.n)}


def make_jobs(spec):
    return [Job(state={"Q": np.zeros(n)}, L=1.0, ng=16, dt=0.1, horizon=h, arrival=a, name=nm)
            for nm, n, h, a in spec]


def test_every_job_runs_exactly_its_horizon_fifo():
    clk = FakeClock()
    be = FakeBackend(clk, max_slots=2)
    jobs = make_jobs([("a", 1000, 50, 0.0), ("b", 2000, 7, 0.0), ("c", 500, 40, 0.0),
                      ("d", 800, 3, 0.0005)])
    rep = Server(backend=be, chunk=10, clock=clk).run(jobs, sleep=clk.sleep)
    for j in jobs:
        assert j.steps_done == j.horizon and j.result["step"] == j.horizon
        assert j.finished_at >= j.admitted_at >= j.arrival
    admits = [e[1] for e in be.log if e[0] == "admit"]
    assert admits == ["a", "b", "c", "d"]          # first come, first served
    assert rep.updates == sum(j.n * j.horizon for j in jobs)
    assert len(be.resident) == 0


def test_budget_and_slots_are_respected():
    clk = FakeClock()
    be = FakeBackend(clk, max_slots=4)
    jobs = make_jobs([(f"j{i}", 1000 + 100 * i, 20 + i, 0.0001 * i) for i in range(9)])
    budget = 100 * 2500                             # at most two of these jobs at once
    Server(backend=be, budget_bytes=budget, chunk=8, clock=clk).run(jobs, sleep=clk.sleep)
    assert be.peak_bytes <= budget
    assert all(j.steps_done == j.horizon for j in jobs)


def test_head_of_line_job_blocks_later_ones_until_it_fits():
    clk = FakeClock()
    be = FakeBackend(clk, max_slots=4)
    jobs = make_jobs([("big0", 2000, 30, 0.0), ("big1", 2000, 5, 0.0), ("small", 10, 5, 0.0)])
    Server(backend=be, budget_bytes=100 * 2100, chunk=8, clock=clk).run(jobs, sleep=clk.sleep)
    order = [e[1] for e in be.log if e[0] == "admit"]
    assert order == ["big0", "big1", "small"]
    t_admit = {e[1]: e[3] for e in be.log if e[0] == "admit"}
    t_retire = {e[1]: e[3] for e in be.log if e[0] == "retire"}
    assert t_admit["big1"] >= t_retire["big0"]       # waited for the budget
    assert t_admit["small"] >= t_admit["big1"]       # no overtaking


def test_idle_server_waits_for_the_next_arrival():
    clk = FakeClock()
    be = FakeBackend(clk)
    jobs = make_jobs([("late", 100, 4, 2.5)])
    rep = Server(backend=be, clock=clk).run(jobs, sleep=clk.sleep)
    assert jobs[0].admitted_at >= 2.5 and rep.wall_s >= 2.5


def test_rejects_oversized_job_and_empty_horizon():
    clk = FakeClock()
    with pytest.raises(ValueError):
        Server(backend=FakeBackend(clk), budget_bytes=1000, clock=clk).run(
            make_jobs([("huge", 1000, 5, 0.0)]), sleep=clk.sleep)
    with pytest.raises(ValueError):
        Server(backend=FakeBackend(clk), clock=clk).run(make_jobs([("zero", 10, 0, 0.0)]),
                                                        sleep=clk.sleep)


@pytest.mark.parametrize("retire_nonfinite", [True, False])
def test_frozen_job_is_retired_early_and_frees_its_slot(retire_nonfinite):
    """A job the engine freezes at step 15 leaves after the chunk in which it froze (not at
    its horizon of 100), the queued job takes its slot then, and only the updates actually
    performed are counted."""
    clk = FakeClock()
    be = FakeBackend(clk, max_slots=2, freeze_at={"bad": 15})
    jobs = make_jobs([("bad", 1000, 100, 0.0), ("good", 1000, 60, 0.0), ("queued", 1000, 30, 0.0)])
    rep = Server(backend=be, chunk=10, clock=clk, retire_nonfinite=retire_nonfinite).run(
        jobs, sleep=clk.sleep)
    bad, good, queued = jobs
    assert bad.result == {"step": 15, "finite": False}
    assert rep.nonfinite_jobs == 1
    assert rep.updates == 1000 * (15 + 60 + 30)
    t_admit = {e[1]: e[3] for e in be.log if e[0] == "admit"}
    t_retire = {e[1]: e[3] for e in be.log if e[0] == "retire"}
    if retire_nonfinite:
        assert bad.steps_done == 20                       # the chunk in which it froze
        assert t_admit["queued"] == t_retire["bad"] < t_retire["good"]
    else:
        assert bad.steps_done == 100
        assert t_admit["queued"] == t_retire["good"] < t_retire["bad"]
    assert good.result == {"step": 60, "finite": True}


def test_weighted_percentiles():
    r = _weighted_pcts([3.0, 1.0, 2.0], [1, 98, 1])
    assert r["p50"] == 1.0 and r["max"] == 3.0
    assert _weighted_pcts([5.0, 7.0], [1, 1])["p99"] == 7.0


class RecordingBackend(FakeBackend):
    """FakeBackend with device records: the k steps of a chunk write the records of integer
    steps dev_step .. dev_step+k-1, stamped evenly over the chunk's fake time."""

    def __init__(self, clock, **kw):
        super().__init__(clock, **kw)
        self.stamps = {}

    def admit(self, slot, job):
        super().admit(slot, job)
        self.stamps[slot] = []

    def step(self, k):
        t0 = self.clock.t
        before = dict(self.dev_step)
        dt = super().step(k)
        for s in self.resident:
            n_new = self.dev_step[s] - before[s]
            self.stamps[s].extend(t0 + (i + 1) * dt / k for i in range(n_new))
        return dt

    def frozen_step(self, slot):
        return self.dev_step[slot]

    def record_stamps(self, slot, count):
        assert count <= len(self.stamps[slot])
        return np.asarray(self.stamps[slot][:count])

    def retire(self, slot):
        self.stamps.pop(slot)
        return super().retire(slot)


def test_step_latency_from_device_record_stamps():
    """With device records the per-step latency samples are the differences of consecutive
    record stamps (records 0 .. done-2 of each job), not chunk means: here each step costs
    1e-5 s per 1000 resident particles, so every sample is 2e-5 s while both jobs are
    resident and 1e-5 s once one is left."""
    clk = FakeClock()
    be = RecordingBackend(clk, max_slots=2)
    jobs = make_jobs([("a", 1000, 25, 0.0), ("b", 1000, 12, 0.0)])
    rep = Server(backend=be, chunk=10, clock=clk).run(jobs, sleep=clk.sleep)
    assert rep.step_latency_source == "device records"
    a, b = rep.jobs
    assert len(a.step_latency_s) == 25 - 2 and len(b.step_latency_s) == 12 - 2
    assert np.allclose(b.step_latency_s, 2e-5)
    # job a: 12 steps with b resident, then 13 alone; the step that straddles b's
    # retirement is stamped at the first step of the next chunk
    assert np.allclose(a.step_latency_s[:11], 2e-5)
    assert np.allclose(a.step_latency_s[11:], 1e-5)
    assert rep.step_latency_us["max"] == pytest.approx(20.0)
    assert rep.step_latency_us["p50"] == pytest.approx(20.0)
