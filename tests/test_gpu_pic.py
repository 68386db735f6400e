"""Monopole-only instances (p* = q* = 0: plain P1 particle-in-cell, the paper's eq.
pic_dynamics and the special case the decorated method reduces to) on the HIP path.

The fused step of such an instance streams only Q, P and psi*.  It must give the oracle's
trajectory with zero dipoles (float64: state to 1e-11, histories to 1e-10), the oracle's
particle update on the device's own field (bitwise), the history of a decorated instance
holding zero dipoles, and leave p* and q* exactly zero; a decorated and a monopole-only
instance can share an engine (one launch per kind and step).
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


def pic_state(w, dtype=np.float64):
    st = w.state(dtype)
    return {"Q": st["Q"], "P": st["P"], "psi": st["psi"]}


def oracle_pic(st, w, nsteps):
    z = np.zeros_like(np.asarray(st["Q"], dtype=np.float64))
    return O.run(np.asarray(st["Q"], dtype=np.float64), np.asarray(st["P"], dtype=np.float64),
                 z, z, np.asarray(st["psi"], dtype=np.float64), w.L, w.ng, w.dt, nsteps)


@pytest.mark.parametrize("threads,ppt,graph", [(512, 4, 1), (1024, 1, 0), (256, 8, 1)])
def test_monopole_fp64_matches_oracle(vp, threads, ppt, graph):
    w = W.landau_linear(seed=6, nx=96, nv=77, ng=64)   # 7392 particles: ragged last tile
    w.params["alpha"] = 0.2
    st = pic_state(w)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64, monopole_only=True)
    sim.set_tuning(threads=threads, ppt=ppt, acc_copies=2, use_graph=graph, graph_steps=6)
    nsteps = 23
    sim.step(nsteps)
    got = sim.state_numpy(0)
    hist = sim.history(0, 0, nsteps) + [sim.diagnostics(0)]
    ref_state, _, ref_hist = oracle_pic(st, w, nsteps)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11), k
    assert np.all(got["qs"] == 0.0) and np.all(got["ps"] == 0.0)
    for key in ("W", "K", "H", "momentum"):
        g = [h[key] for h in hist]
        r = [h[key] for h in ref_hist]
        assert rel_l2(g, r) < 1e-10 or np.max(np.abs(np.subtract(g, r))) < 1e-13, key
    sim.close()


@pytest.mark.parametrize("prec", ["fp32c", "fp32ts", "fp64"])
def test_monopole_first_step_bitwise_and_history_as_decorated(vp, prec):
    """The first fused step of a monopole-only instance is the oracle's half-kick and drift
    with zero dipoles applied to the device's own initial field, in float64 arithmetic
    rounded once to the state type: bitwise.  Over 20 steps its field-energy history equals
    that of a decorated instance holding zero dipoles within 1e-6 (they differ only in the
    order of the deposit's atomic sums)."""
    w = W.two_stream(nx=256, nv=96, ng=128)
    dt_np = np.float64 if prec == "fp64" else np.float32
    full = w.state(dt_np)
    zero = np.zeros_like(full["Q"])
    st = {"Q": full["Q"], "P": full["P"], "psi": full["psi"], "qs": zero, "ps": zero}
    a = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=64, monopole_only=True)
    b = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=64)
    for s in (a, b):
        s.set_tuning(threads=512, ppt=4, acc_copies=4, graph_steps=3)
    f0 = a.diagnostics(0, grid=True)
    a.step(1)
    raw = {k: v.detach().cpu().numpy() for k, v in a.state(0).items()}   # P owes a half-kick
    Q0, P0 = (st[k].astype(np.float64) for k in ("Q", "P"))
    z = np.zeros_like(Q0)
    P1, q1 = O.kick(Q0, P0, z, z, f0["E"], f0["g"], w.L, 0.5 * w.dt)
    Q1, p1 = O.drift(Q0, P1, q1, z, w.L, w.dt)
    for k, r in (("Q", Q1), ("P", P1), ("qs", q1), ("ps", p1)):
        assert np.array_equal(raw[k], r.astype(dt_np)), k
    b.step(1)
    a.step(19)
    b.step(19)
    ha, hb = a.history(0, 0, 20), b.history(0, 0, 20)
    assert rel_l2([h["W"] for h in ha], [h["W"] for h in hb]) < 1e-6
    sa = a.state_numpy(0)
    assert np.all(sa["qs"] == 0.0) and np.all(sa["ps"] == 0.0)
    a.close()
    b.close()


def test_mixed_engine_and_persistent(vp):
    """Decorated and monopole-only instances in one engine, fused (two launches per step)
    and then persistent (the decorated kernel carries the zero dipoles), each on its
    oracle trajectory."""
    ws = W.landau_sweep(seed=31, n_inst=4)
    kinds = [False, True, False, True]
    sts = []
    eng = vp.Engine("fp64", max_slots=4)
    for s, (w, mono) in enumerate(zip(ws, kinds)):
        st = w.state()
        if mono:
            st = {"Q": st["Q"], "P": st["P"], "psi": st["psi"]}
        sts.append(st)
        eng.admit(s, st, w.L, w.ng, w.dt, monopole_only=mono, solver="fft" if s == 2 else "scan")
    eng.set_tuning(threads=512, ppt=4, acc_copies=2, graph_steps=3)
    eng.step(7)
    eng.set_tuning(persistent=1)
    eng.step(5)
    for s, (w, st, mono) in enumerate(zip(ws, sts, kinds)):
        if mono:
            ref_state, _, _ = oracle_pic(st, w, 12)
        else:
            ref_state, _, _ = O.run(*(np.asarray(st[k], dtype=np.float64) for k in FIELDS),
                                    w.L, w.ng, w.dt, 12)
        got = eng.state_numpy(s)
        for k, r in zip(FIELDS, ref_state):
            assert np.allclose(got[k], r, rtol=0, atol=1e-11), (s, k)
        assert eng.diagnostics(s)["step"] == 12
    eng.close()


def test_monopole_admission_zeroes_dipoles_of_any_state(vp):
    """Arrays passed for qs and ps of a monopole-only instance are zeroed on admission, odd
    float counts included."""
    w = W.landau_linear(seed=2, nx=33, nv=31, ng=32)          # 1023 particles
    st = w.state(np.float32)
    st["qs"] = np.full_like(st["Q"], 3.0)
    st["ps"] = np.full_like(st["Q"], -2.0)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", monopole_only=True)
    raw = {k: v.detach().cpu().numpy() for k, v in sim.state(0).items()}
    assert np.all(raw["qs"] == 0.0) and np.all(raw["ps"] == 0.0)
    sim.step(4)
    s = sim.state_numpy(0)
    assert np.all(s["qs"] == 0.0) and np.all(s["ps"] == 0.0)
    sim.close()
