"""Persistent steps (many steps per cooperative launch, particles in registers between steps)
against one fused launch per step and against the FP64 oracle."""
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


def oracle_run(st, w, nsteps):
    return O.run(*(np.asarray(st[k], dtype=np.float64) for k in FIELDS), w.L, w.ng, w.dt, nsteps)


@pytest.mark.parametrize("threads,ppt,copies", [(1024, 4, 4), (512, 2, 1), (512, 8, 8)])
def test_persistent_fp64_matches_oracle(vp, threads, ppt, copies):
    w = W.landau_linear(seed=4, nx=96, nv=80, ng=64)   # 7680 particles, several tiles
    w.params["alpha"] = 0.2
    st = w.state()
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64)
    sim.set_tuning(threads=threads, ppt=ppt, acc_copies=copies, persistent=1)
    nsteps = 23
    sim.step(nsteps)
    got = sim.state_numpy(0)
    hist = sim.history(0, 0, nsteps) + [sim.diagnostics(0)]
    ref_state, _, ref_hist = oracle_run(st, w, nsteps)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11), k
    for key in ("W", "K", "H"):
        assert rel_l2([h[key] for h in hist], [h[key] for h in ref_hist]) < 1e-10, key
    assert [h["step"] for h in hist] == list(range(nsteps + 1))
    sim.close()


def test_persistent_fp32c_matches_fused_and_continues_across_modes(vp):
    w = W.two_stream(nx=256, nv=128, ng=128)
    st = w.state(np.float32)
    a = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=64)
    b = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=64)
    a.set_tuning(threads=1024, ppt=4, acc_copies=2, persistent=1)
    b.set_tuning(threads=1024, ppt=4, acc_copies=2, persistent=0)
    a.step(10)
    b.step(10)
    # switch modes in the middle: persistent -> fused and fused -> persistent
    a.set_tuning(persistent=0)
    b.set_tuning(persistent=1)
    a.step(11)
    b.step(11)
    sa, sb = a.state_numpy(0), b.state_numpy(0)
    for k in FIELDS:
        assert rel_l2(sa[k], sb[k]) < 1e-5, k
    ha, hb = a.history(0, 0, 21), b.history(0, 0, 21)
    assert rel_l2([h["W"] for h in ha], [h["W"] for h in hb]) < 1e-5
    assert a.diagnostics(0)["step"] == b.diagnostics(0)["step"] == 21
    a.close()
    b.close()


def test_persistent_batch_and_mid_run_admission(vp):
    ws = W.landau_sweep(seed=17, n_inst=4)
    sts = [w.state() for w in ws]
    eng = vp.Engine("fp64", max_slots=3)
    for s in range(3):
        eng.admit(s, sts[s], ws[s].L, ws[s].ng, ws[s].dt, solver="fft" if s == 1 else "scan")
    eng.set_tuning(threads=512, ppt=4, acc_copies=2, persistent=1)
    eng.step(8)
    eng.retire(2)
    eng.admit(2, sts[3], ws[3].L, ws[3].ng, ws[3].dt)
    eng.step(6)
    for s, (st, w, n) in enumerate(((sts[0], ws[0], 14), (sts[1], ws[1], 14), (sts[3], ws[3], 6))):
        got = eng.state_numpy(s)
        ref_state, _, _ = oracle_run(st, w, n)
        for k, r in zip(FIELDS, ref_state):
            assert np.allclose(got[k], r, rtol=0, atol=1e-11), (s, k)
        assert eng.diagnostics(s)["step"] == n


def test_persistent_with_sorting_matches_unsorted(vp):
    w = W.landau_linear(seed=2, nx=128, nv=64, ng=128)
    st = w.state()
    a = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", sort_every=4, sort_chunk=1024)
    b = vp.Simulation(st, w.L, w.ng, w.dt, "fp64")
    a.set_tuning(threads=512, ppt=4, persistent=1)
    a.step(13)
    b.step(13)
    da, db = a.diagnostics(0), b.diagnostics(0)
    for k in ("K", "W", "H", "momentum", "charge"):
        assert abs(da[k] - db[k]) <= 1e-10 * max(1.0, abs(db[k])), k


def test_persistent_rejects_shapes_that_do_not_fit(vp):
    w = W.two_stream(nx=512, nv=512, ng=64)
    sim = vp.Simulation(w.state(np.float32), w.L, w.ng, w.dt, "fp32c")
    with pytest.raises(vp.VPError) as e:
        sim.set_tuning(threads=512, ppt=2, persistent=1, acc_copies=1)  # 256 tiles: fits
        big = vp.Simulation(W.two_stream(nx=4096, nv=1024, ng=64).state(np.float32), w.L, 64,
                            w.dt, "fp32c")
        big.set_tuning(threads=512, ppt=2, persistent=1)         # 4096 tiles: cannot all be resident
    assert e.value.status == vp._lib.VP_ERR_ARG
    assert sim.get_tuning()["persistent"] == 1
    sim.step(3)
    assert sim.diagnostics(0)["step"] == 3


def test_persistent_runs_past_one_launch(vp):
    """1030 steps in one call are two cooperative launches (1024 steps, then 6), the second
    starting at ring phase 1024 mod 3; the history ring (64 records) wraps 16 times.  A ragged
    last tile (7680 particles in tiles of 4096).  dt = 0.01 keeps the run (t = 10.3) inside
    the ansatz's validity.  The bars are about a thousand times what permuting the particles
    alone (a different summation order) gives in the oracle over these steps: 4e-14 in the
    state, 1e-14 in the W history."""
    w = W.landau_linear(seed=4, nx=96, nv=80, ng=64)
    w.params["alpha"] = 0.2
    dt = 0.01
    st = w.state()
    sim = vp.Simulation(st, w.L, w.ng, dt, "fp64", hist_cap=64)
    sim.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=1)
    sim.step(1030)
    sim.step(5)                                   # continues from the odd phase
    nsteps = 1035
    got = sim.state_numpy(0)
    hist = sim.history(0, nsteps - 60, 60) + [sim.diagnostics(0)]
    ref_state, _, ref_hist = O.run(*(np.asarray(st[k], dtype=np.float64) for k in FIELDS),
                                   w.L, w.ng, dt, nsteps)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-10), k
    assert [h["step"] for h in hist] == list(range(nsteps - 60, nsteps + 1))
    ref_tail = ref_hist[nsteps - 60:]              # the oracle's record i is step i
    for key in ("W", "K", "H"):
        assert rel_l2([h[key] for h in hist], [h[key] for h in ref_tail]) < 1e-11, key
    with pytest.raises(vp.VPError) as e:
        sim.history(0, nsteps - 70, 10)           # overwritten records
    assert e.value.status == vp._lib.VP_ERR_RANGE
    sim.close()


@pytest.mark.parametrize("n", [1, 7, 257])
def test_persistent_edge_sizes(vp, n):
    """n = 1 and n below one wavefront in a persistent launch: one tile, most lanes empty;
    a particle at 0 and one on a node."""
    L, ng = 3.0, 16
    rng = np.random.default_rng(n)
    st = {"Q": rng.uniform(0, L, n), "P": rng.normal(size=n), "qs": 0.01 * rng.normal(size=n),
          "ps": 0.01 * rng.normal(size=n), "psi": rng.uniform(0.1, 1, n)}
    st["Q"][0] = 0.0
    if n > 1:
        st["Q"][1] = 5 * L / ng
    sim = vp.Simulation(st, L, ng, 0.05, "fp64", hist_cap=16)
    sim.set_tuning(threads=512, ppt=2, acc_copies=1, persistent=1)
    sim.step(5)
    got = sim.state_numpy(0)
    ref_state, _, ref_hist = O.run(*(np.asarray(st[k], dtype=np.float64) for k in FIELDS),
                                   L, ng, 0.05, 5)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11), k
    hist = sim.history(0, 0, 5) + [sim.diagnostics(0)]
    for key in ("W", "K", "H"):
        assert rel_l2([h[key] for h in hist], [h[key] for h in ref_hist]) < 1e-10, key
    sim.close()


@pytest.mark.parametrize("solver", ["scan", "fft"])
def test_persistent_at_the_largest_grid(vp, solver):
    """Ng = 1024 (the largest grid), 2^15 - 11 particles (a ragged tail), two launches
    (7 and 6 steps), float64 against the oracle."""
    w = W.landau_linear(seed=6, nx=2048, nv=16, ng=1024)
    w.params["alpha"] = 0.1
    st = {k: v[:-11] for k, v in w.state().items()}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=32, solver=solver)
    sim.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=1)
    sim.step(7)
    sim.step(6)
    nsteps = 13
    got = sim.state_numpy(0)
    hist = sim.history(0, 0, nsteps) + [sim.diagnostics(0)]
    ref_state, _, ref_hist = oracle_run(st, w, nsteps)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11), k
    for key in ("W", "K", "H"):
        assert rel_l2([h[key] for h in hist], [h[key] for h in ref_hist]) < 1e-10, key
    sim.close()


def test_persistent_wait_time_out_is_reported(vp, monkeypatch):
    """The bounded wait between persistent steps, forced from the host: a handle created
    with VP_PERSIST_SPIN_LIMIT = 0 gives up at its first unanswered poll, so every tile
    stops waiting in that launch and the launch drains (no wave is left spinning); the
    instance is flagged and reported with VP_ERR_HIP.  A handle created after it, with the
    default limit, steps the same state normally."""
    w = W.two_stream(nx=512, nv=512, ng=64)        # 2^18 particles, 64 tiles of 4096
    st = w.state(np.float32)
    monkeypatch.setenv("VP_PERSIST_SPIN_LIMIT", "0")
    bad = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c")
    monkeypatch.delenv("VP_PERSIST_SPIN_LIMIT")
    bad.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=1)
    status = None
    try:
        bad.step(40)
        bad.diagnostics(0)
    except vp.VPError as e:
        status = e.status
    assert status == vp._lib.VP_ERR_HIP
    bad.close()
    good = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c")
    ref = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c")
    good.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=1)
    ref.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=0)
    good.step(40)
    ref.step(40)
    dg, dr = good.diagnostics(0), ref.diagnostics(0)
    for key in ("W", "K", "H"):
        assert abs(dg[key] - dr[key]) <= 1e-5 * abs(dr[key]), key
    good.close()
    ref.close()
