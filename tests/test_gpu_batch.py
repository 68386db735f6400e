"""Batched engine: uneven instances advanced by one fused launch per step.

Each instance of a batch must evolve exactly as it would alone: against the FP64 oracle in
float64 (state to 1e-11, field-energy history to 1e-10), and against the same instance run
alone in the FP32 compensated mode (relative L2 <= 1e-5).  Slots admitted and retired in the
middle of a run must not disturb the other instances.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("Q", "P", "qs", "ps", "psi")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def sweep(n_inst, seed):
    """Uneven Landau instances of the sweep recipe (N from 2^12 to 2^16, Ng 64..256)."""
    return W.landau_sweep(seed=seed, n_inst=n_inst)


def oracle_run(st, w, nsteps):
    return O.run(*(np.asarray(st[k], dtype=np.float64) for k in FIELDS), w.L, w.ng, w.dt, nsteps)


def test_batch_fp64_matches_oracle_per_instance(vp):
    ws = sweep(6, seed=3)
    sts = [w.state() for w in ws]
    eng = vp.Engine("fp64", max_slots=len(ws))
    for s, (w, st) in enumerate(zip(ws, sts)):
        eng.admit(s, st, w.L, w.ng, w.dt, hist_cap=64, solver="fft" if s % 2 else "scan")
    nsteps = 12
    eng.step(nsteps)
    for s, (w, st) in enumerate(zip(ws, sts)):
        hist = eng.history(s, 0, nsteps) + [eng.diagnostics(s)]
        got = eng.state_numpy(s)
        ref_state, _, ref_hist = oracle_run(st, w, nsteps)
        for k, r in zip(FIELDS, ref_state):
            assert np.allclose(got[k], r, rtol=0, atol=1e-11), (s, k)
        for key in ("W", "K", "H"):
            g = np.array([h[key] for h in hist])
            r = np.array([h[key] for h in ref_hist])
            assert rel_l2(g, r) < 1e-10, (s, key)
        assert [h["step"] for h in hist] == list(range(nsteps + 1))


def test_batch_fp32c_matches_instances_alone(vp):
    ws = sweep(5, seed=7)
    sts = [w.state(np.float32) for w in ws]
    eng = vp.Engine("fp32c", max_slots=len(ws))
    for s, (w, st) in enumerate(zip(ws, sts)):
        eng.admit(s, st, w.L, w.ng, w.dt)
    eng.set_tuning(threads=512, ppt=2, acc_copies=4, graph_steps=6)
    eng.step(20)
    for s, (w, st) in enumerate(zip(ws, sts)):
        alone = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c")
        alone.set_tuning(threads=1024, ppt=4, acc_copies=1, graph_steps=9)
        alone.step(20)
        a, b = eng.state_numpy(s), alone.state_numpy(0)
        for k in FIELDS:
            assert rel_l2(a[k], b[k]) < 1e-5, (s, k)
        da, db = eng.diagnostics(s), alone.diagnostics(0)
        assert abs(da["W"] - db["W"]) <= 1e-5 * abs(db["W"]), s
        alone.close()


def test_admit_and_retire_mid_run_leave_others_unchanged(vp):
    """Slot 1 is retired after 7 steps and a new instance admitted there (at ring phase
    7 mod 3); slots 0 and 2 must match an uninterrupted run, and the new instance must
    match the oracle from its own start."""
    ws = sweep(4, seed=11)
    sts = [w.state() for w in ws]
    ref_eng = vp.Engine("fp64", max_slots=3)
    eng = vp.Engine("fp64", max_slots=3)
    for s in range(3):
        ref_eng.admit(s, sts[s], ws[s].L, ws[s].ng, ws[s].dt)
        eng.admit(s, sts[s], ws[s].L, ws[s].ng, ws[s].dt)
    ref_eng.step(16)
    eng.step(7)
    eng.retire(1)
    eng.admit(1, sts[3], ws[3].L, ws[3].ng, ws[3].dt, hist_cap=32)
    eng.step(9)
    for s in (0, 2):
        a, b = eng.state_numpy(s), ref_eng.state_numpy(s)
        for k in FIELDS:
            assert np.allclose(a[k], b[k], rtol=0, atol=1e-12), (s, k)
    got = eng.state_numpy(1)
    ref_state, _, ref_hist = oracle_run(sts[3], ws[3], 9)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11), k
    hist = eng.history(1, 0, 9)
    assert rel_l2([h["W"] for h in hist], [h["W"] for h in ref_hist[:9]]) < 1e-10
    assert eng.diagnostics(1)["step"] == 9


def test_retire_returns_integer_time_state(vp):
    """vp_retire applies the pending half-kick: the returned arrays are the state at the
    last integer step (the oracle's state after that many steps)."""
    w = sweep(1, seed=5)[0]
    st = w.state()
    eng = vp.Engine("fp64", max_slots=2)
    eng.admit(0, st, w.L, w.ng, w.dt)
    eng.step(5)
    out = eng.retire(0)
    got = {k: v.detach().cpu().numpy() for k, v in out.items()}
    ref_state, _, _ = oracle_run(st, w, 5)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11), k


def test_nonfinite_instance_is_frozen_and_others_continue(vp):
    """A NaN in one instance freezes that instance (its step counter stops, diagnostics
    report non-finite) and leaves the others exactly on their oracle trajectories."""
    ws = sweep(3, seed=13)
    sts = [w.state() for w in ws]
    bad = {k: v.copy() for k, v in sts[1].items()}
    bad["P"][5] = np.nan
    eng = vp.Engine("fp64", max_slots=3)
    eng.admit(0, sts[0], ws[0].L, ws[0].ng, ws[0].dt)
    eng.admit(1, bad, ws[1].L, ws[1].ng, ws[1].dt)
    eng.admit(2, sts[2], ws[2].L, ws[2].ng, ws[2].dt)
    eng.step(8)
    with pytest.raises(vp.VPError) as e:
        eng.diagnostics(1)
    assert e.value.status == vp._lib.VP_ERR_NONFINITE
    frozen_at = eng.diagnostics(1, allow_nonfinite=True)["step"]
    assert frozen_at < 8
    # the one-call status of every slot agrees
    assert eng.slot_status() == {0: (8, True), 1: (frozen_at, False), 2: (8, True)}
    for s in (0, 2):
        got = eng.state_numpy(s)
        ref_state, _, _ = oracle_run(sts[s], ws[s], 8)
        for k, r in zip(FIELDS, ref_state):
            assert np.allclose(got[k], r, rtol=0, atol=1e-11), (s, k)
        assert eng.diagnostics(s)["step"] == 8
