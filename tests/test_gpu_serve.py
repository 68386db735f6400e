"""Serving loop on the GPU: jobs that arrive while others run are admitted as slots and
memory free up, run batched with the others, and end with the same result as alone and as
the oracle's run of the same job."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from fp32_reference import fp32_fused_reference

pytestmark = pytest.mark.gpu

FIELDS = ("Q", "P", "qs", "ps", "psi")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_jobs(dtype):
    from paper_2605_21794_amd.serve import Job
    ws = W.landau_sweep(seed=21, n_inst=5)
    horizons = [37, 12, 50, 25, 8]
    arrivals = [0.0, 0.0, 0.002, 0.004, 0.004]
    jobs = []
    for i, w in enumerate(ws):
        st = w.state(dtype)
        jobs.append(Job(state=st, L=w.L, ng=w.ng, dt=w.dt, horizon=horizons[i],
                        arrival=arrivals[i], solver="fft" if i == 3 else "scan",
                        name=f"job{i}"))
    return ws, jobs


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_each_job_same_alone_and_in_the_mix(vp, prec):
    from paper_2605_21794_amd.serve import Server
    dtype = np.float64 if prec == "fp64" else np.float32
    ws, jobs = small_jobs(dtype)
    # three slots for five jobs, and a budget that holds about two of them: jobs queue
    srv = Server(precision=prec, max_slots=3, chunk=9, keep_state=True, keep_history=True)
    budget = sorted(srv.backend.job_bytes(j) for j in jobs)
    srv.budget = budget[-1] + budget[-2]
    rep = srv.run(jobs)
    assert rep.updates == sum(j.n * j.horizon for j in jobs)
    assert rep.step_latency_source == "device records"
    assert rep.step_latency_us["p50"] > 0 and rep.step_latency_us["p99"] >= rep.step_latency_us["p50"]
    for w, j in zip(ws, jobs):
        # every served job against the oracle: float64 on the oracle's own run, float32
        # state on the oracle's sub-flows with the fused step's float32 storage points
        hist = j.history + [j.result]
        got = {k: v.detach().cpu().numpy() for k, v in j.final_state.items()}
        s64 = {k: np.asarray(v, dtype=np.float64) for k, v in j.state.items()}
        if prec == "fp64":
            ref_state, _, ref_hist = O.run(*(s64[k] for k in FIELDS), j.L, j.ng, j.dt,
                                           j.horizon)
            for k, r in zip(FIELDS, ref_state):
                assert np.allclose(got[k], r, rtol=0, atol=1e-11), (j.name, k)
            Wr = [h["W"] for h in ref_hist]
            assert rel_l2([h["W"] for h in hist], Wr) < 1e-10, j.name
        else:
            Wr, _, (Q, P, qs, ps) = fp32_fused_reference(s64, w, j.horizon)
            assert rel_l2([h["W"] for h in hist], Wr) < 1e-5, j.name
            for k, r in (("Q", Q), ("P", P), ("qs", qs), ("ps", ps)):
                assert rel_l2(got[k], r) < 1e-5, (j.name, k)
        assert [h["step"] for h in hist] == list(range(j.horizon + 1)), j.name
        # per-step device latencies: horizon - 2 samples per job, each a positive time
        assert len(j.step_latency_s) == j.horizon - 2 and min(j.step_latency_s) > 0, j.name
    for j in jobs:
        assert j.steps_done == j.horizon and j.result["step"] == j.horizon
        alone = vp.Simulation(j.state, j.L, j.ng, j.dt, prec, solver=j.solver)
        alone.step(j.horizon)
        ref = alone.state_numpy(0)
        got = {k: v.detach().cpu().numpy() for k, v in j.final_state.items()}
        for k in FIELDS:
            if prec == "fp64":
                assert np.allclose(got[k], ref[k], rtol=0, atol=1e-12), (j.name, k)
            else:
                assert rel_l2(got[k], ref[k]) < 1e-5, (j.name, k)
        da = alone.diagnostics(0)
        assert abs(j.result["W"] - da["W"]) <= (1e-10 if prec == "fp64" else 1e-5) * abs(da["W"])
        alone.close()


def test_frozen_job_leaves_early_and_the_others_are_unchanged(vp):
    """A job whose state holds a NaN is frozen by the engine; the server sees it in the
    status poll after its first chunk, retires it (result not finite, far short of its
    horizon) and gives its slot to the queue.  The other jobs end as they do alone."""
    from paper_2605_21794_amd.serve import Server
    ws, jobs = small_jobs(np.float64)
    bad = jobs[2]
    bad.state = {k: v.copy() for k, v in bad.state.items()}
    bad.state["P"][3] = np.nan
    srv = Server(precision="fp64", max_slots=2, chunk=5, keep_state=True)
    rep = srv.run(jobs)
    assert rep.nonfinite_jobs == 1
    assert bad.result["finite"] is False and bad.result["step"] < 5
    assert bad.steps_done < bad.horizon
    for j in jobs:
        if j is bad:
            continue
        assert j.result["finite"] and j.steps_done == j.horizon
        alone = vp.Simulation(j.state, j.L, j.ng, j.dt, "fp64", solver=j.solver)
        alone.step(j.horizon)
        ref = alone.state_numpy(0)
        got = {k: v.detach().cpu().numpy() for k, v in j.final_state.items()}
        for k in FIELDS:
            assert np.allclose(got[k], ref[k], rtol=0, atol=1e-12), (j.name, k)
        alone.close()
