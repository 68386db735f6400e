"""A prescribed potential V(q) = A (1 - cos(2 pi m q / L)) added to the field, with or
without the particles' own field, on the HIP path against the oracle run with the same
options (float64: state to 1e-11, K / U / W / H histories to 1e-10).  The paper's
test-particle example (three decorated particles, charge e = 0, V = 1 - cos(kappa q),
L = 10) is the first case."""
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


def check(sim, st, L, ng, dt, nsteps, slot=0, **opts):
    got = sim.state_numpy(slot)
    hist = sim.history(slot, 0, nsteps) + [sim.diagnostics(slot)]
    ref_state, _, ref_hist = O.run(*(np.asarray(st[k], dtype=np.float64) for k in FIELDS), L, ng,
                                   dt, nsteps, **opts)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11), k
    for key in ("K", "U", "W", "H"):
        g = np.array([h[key] for h in hist])
        r = np.array([h[key] for h in ref_hist])
        assert np.max(np.abs(g - r)) <= 1e-10 * max(1e-300, np.max(np.abs(r))) or \
            np.max(np.abs(g - r)) < 1e-14, key
    return hist, ref_hist


@pytest.mark.parametrize("persistent", [0, 1])
def test_paper_test_particle_example(vp, persistent):
    L, ng, dt, nsteps = 10.0, 16, 0.05, 200
    st = {"Q": np.array([2.0, 5.0, 8.0]), "P": np.array([0.5, -0.3, 1.0]),
          "qs": np.array([0.1, -0.05, 0.02]), "ps": np.array([0.05, 0.1, -0.03]),
          "psi": np.array([10.0, 10.0, 10.0])}
    ext = {"amp": 1.0, "mode": 1}
    sim = vp.Simulation(st, L, ng, dt, "fp64", hist_cap=256, self_field=False, external=ext)
    sim.set_tuning(threads=512, ppt=2, acc_copies=1, graph_steps=9, persistent=persistent)
    sim.step(nsteps)
    hist, _ = check(sim, st, L, ng, dt, nsteps, ext=ext, self_field=False)
    assert all(h["W"] == 0.0 and h["e_amp"] == 0.0 for h in hist)
    H = np.array([h["H"] for h in hist])
    assert np.max(np.abs(H - H[0])) < 1e-2 * abs(H[0])        # H_SWPIC bounded
    sim.close()


@pytest.mark.parametrize("solver,persistent", [("scan", 0), ("fft", 0), ("scan", 1)])
def test_plasma_in_a_potential(vp, solver, persistent):
    """Landau plasma (self field on) in an added potential, the two projections with
    a nodal one too: every diagnostic and the state on the oracle's trajectory."""
    w = W.landau_linear(seed=9, nx=96, nv=80, ng=64)
    w.params["alpha"] = 0.2
    st = w.state()
    ext = {"amp": 0.3, "mode": 2}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64, solver=solver, external=ext)
    sim.set_tuning(threads=512, ppt=2, acc_copies=2, graph_steps=6, persistent=persistent)
    sim.step(23)
    hist, _ = check(sim, st, w.L, w.ng, w.dt, 23, ext=ext)
    assert max(abs(h["U"]) for h in hist) > 0.0
    sim.close()


def test_mixed_options_in_one_engine(vp):
    """Instances with a potential, without self field, with a nodal projection, monopole-only
    and plain, in one engine; each on its own oracle trajectory."""
    ws = W.landau_sweep(seed=41, n_inst=5)
    opts = [dict(), dict(external={"amp": 0.2, "mode": 1}),
            dict(external={"amp": 0.5, "mode": 3}, self_field=False),
            dict(projection="nodal", external={"amp": 0.1, "mode": 1}),
            dict(monopole_only=True, external={"amp": 0.4, "mode": 1})]
    eng = vp.Engine("fp64", max_slots=5)
    sts = []
    for s, (w, o) in enumerate(zip(ws, opts)):
        st = w.state()
        if o.get("monopole_only"):
            st["qs"] = np.zeros_like(st["Q"])
            st["ps"] = np.zeros_like(st["Q"])
        sts.append(st)
        eng.admit(s, st, w.L, w.ng, w.dt, hist_cap=32, **o)
    eng.set_tuning(threads=512, ppt=4, acc_copies=2, graph_steps=3)
    eng.step(11)
    for s, (w, st, o) in enumerate(zip(ws, sts, opts)):
        oracle_opts = {}
        if "external" in o:
            oracle_opts["ext"] = o["external"]
        if o.get("self_field") is False:
            oracle_opts["self_field"] = False
        if "projection" in o:
            oracle_opts["projection"] = o["projection"]
        check(eng, st, w.L, w.ng, w.dt, 11, slot=s, **oracle_opts)
    eng.close()


def test_fp32c_with_potential_tracks_float64(vp):
    """fp32c storage with a potential: 20 steps within 1e-5 of the float64 run (the same
    options, from the same float32 initial bits)."""
    w = W.two_stream(nx=256, nv=128, ng=128)
    st = w.state(np.float32)
    ext = {"amp": 0.05, "mode": 1}
    a = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=32, external=ext)
    b = vp.Simulation({k: v.astype(np.float64) for k, v in st.items()}, w.L, w.ng, w.dt, "fp64",
                      hist_cap=32, external=ext)
    a.step(20)
    b.step(20)
    ha, hb = a.history(0, 0, 20), b.history(0, 0, 20)
    for key in ("U", "H"):
        assert rel_l2([h[key] for h in ha], [h[key] for h in hb]) < 1e-5, key
    a.close()
    b.close()
