"""Decorated particles with second moments (k = 3, P2 elements) on the HIP path against the
k = 3 oracle: fused steps in several launch shapes with a ragged tail, the unfused primitive
composition, a prescribed potential without self field (the paper's test-particle system),
zero moments (bit for bit the k = 2 P2 run), the Casimir det M of every particle, float32
state against the oracle's sub-flows with the fused step's float32 storage points, the
full-size two-stream workload, and the configurations the library refuses.  Bars as for P2:
float64 trajectories 1e-10 (absolute), histories 1e-10 of their scale."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

K3 = O.K3_FIELDS


def lattice(ng, nx, nv, alpha=0.1, seed=0):
    w = W.landau_linear(seed=seed, nx=nx, nv=nv, ng=ng)
    w.params["alpha"] = alpha
    return w


def k3_state(w, dtype=np.float64):
    return w.state(dtype, moments=True)


def check_run(sim, st, w, nsteps, slot=0, ext=None, self_field=True, atol=1e-10):
    got = sim.state_numpy(slot)
    hist = sim.history(slot, 0, nsteps) + [sim.diagnostics(slot)]
    ref_state, _, ref_hist = O.run_k3({k: np.asarray(st[k], dtype=np.float64) for k in K3}, w.L,
                                      w.ng, w.dt, nsteps, ext=ext, self_field=self_field)
    for k, r in zip(K3, ref_state):
        scale = max(1.0, float(np.max(np.abs(r))))
        assert np.max(np.abs(np.asarray(got[k], dtype=np.float64) - r)) <= atol * scale, k
    for key in ("K", "W", "U", "H", "momentum"):
        g = np.array([h[key] for h in hist])
        r = np.array([h[key] for h in ref_hist])
        scale = max(1e-300, float(np.max(np.abs(r))))
        assert np.max(np.abs(g - r)) <= 1e-10 * scale or np.max(np.abs(g - r)) < 1e-14, key
    return got


@pytest.mark.parametrize("threads,ppt,copies,graph,solver", [
    (256, 1, 1, 3, "scan"), (512, 2, 8, 0, "scan"), (1024, 4, 3, 6, "fft"), (1024, 8, 2, 9, "scan")])
def test_fused_steps_match_the_oracle(vp, threads, ppt, copies, graph, solver):
    w = lattice(32, 128, 40)
    st = {k: v[:-37] for k, v in k3_state(w).items()}      # a ragged tail
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64, solver=solver, element_order=2)
    sim.set_tuning(threads=threads, ppt=ppt, acc_copies=copies, use_graph=1 if graph else 0,
                   graph_steps=max(1, graph))
    sim.step(20)
    check_run(sim, st, w, 20)
    sim.close()


def test_primitive_steps_equal_one_oracle_step(vp):
    w = lattice(16, 64, 24, alpha=0.2)
    st = k3_state(w)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", element_order=2)
    for _ in range(3):
        sim.gather_push(0.5 * w.dt, w.dt)
        sim.deposit()
        sim.poisson()
        sim.gather_push(0.5 * w.dt, 0.0)
    got = sim.state_numpy(0)
    ref = tuple(np.asarray(st[k], dtype=np.float64).copy() for k in K3)
    fld = O.solve_field_p2_k3(ref[0], ref[3], ref[4], ref[5], w.L, w.ng)
    for _ in range(3):
        ref, fld = O.step_k3(ref, fld, w.L, w.ng, w.dt)
    for k, r in zip(K3, ref):
        assert np.allclose(got[k], r, rtol=0, atol=1e-11 * max(1.0, np.max(np.abs(r)))), k
    d = sim.diagnostics(0, grid=True)
    assert np.max(np.abs(d["g"] - fld["g"])) <= 1e-12 * np.max(np.abs(fld["g"]))
    sim.close()


def test_zero_moments_are_the_k2_p2_run(vp):
    """With M = 0 every added term is an exact zero: the k = 3 run takes the k = 2 P2 run's
    values (to the order of the load's floating-point atomics)."""
    w = lattice(32, 128, 24)
    st = k3_state(w)
    for k in ("Mqq", "Mqp", "Mpp"):
        st[k] = np.zeros_like(st["Q"])
    a = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=32, element_order=2)
    b = vp.Simulation({k: st[k] for k in ("Q", "P", "qs", "ps", "psi")}, w.L, w.ng, w.dt, "fp64",
                      hist_cap=32, element_order=2)
    for s in (a, b):
        s.set_tuning(threads=512, ppt=2, acc_copies=1, graph_steps=3)
        s.step(12)
    sa, sb = a.state_numpy(0), b.state_numpy(0)
    for k in ("Q", "P", "qs", "ps"):
        assert np.allclose(sa[k], sb[k], rtol=0, atol=1e-12), k
    assert not np.any(sa["Mqq"]) and not np.any(sa["Mqp"]) and not np.any(sa["Mpp"])
    wa = np.array([h["W"] for h in a.history(0, 0, 12)])
    wb = np.array([h["W"] for h in b.history(0, 0, 12)])
    assert np.max(np.abs(wa - wb)) <= 1e-12 * np.max(wb)
    a.close()
    b.close()


def test_casimir_det_m_kept_on_the_device(vp):
    w = lattice(32, 128, 40, alpha=0.3)
    st = k3_state(w)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64, element_order=2)
    sim.step(40)
    got = sim.state_numpy(0)
    det0 = st["Mqq"] * st["Mpp"] - st["Mqp"] ** 2
    det1 = got["Mqq"] * got["Mpp"] - got["Mqp"] ** 2
    assert np.all(det0 > 0)
    assert np.max(np.abs(det1 - det0) / det0) < 1e-8
    assert np.max(np.abs(got["Mqq"] - st["Mqq"]) / st["Mqq"]) > 1e-2   # the moments moved
    sim.close()


def test_test_particles_in_a_prescribed_potential(vp):
    """The paper's test-particle potential V = 1 - cos(2 pi q / L), no self field: the
    moments feel V'' and the mean-force term -(1/2) Mqq V''' moves q*."""
    w = lattice(16, 64, 16, alpha=0.05)
    w.L = 10.0
    st = k3_state(w)
    st["Q"] = np.mod(st["Q"], w.L)
    ext = {"amp": 1.0, "mode": 1}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64, element_order=2,
                        self_field=False, external=ext)
    sim.step(30)
    check_run(sim, st, w, 30, ext=ext, self_field=False)
    sim.close()


@pytest.mark.parametrize("prec", ["fp32c", "fp32ts"])
def test_float32_state_matches_storage_reference(vp, prec):
    import fp32_reference as FR
    w = lattice(32, 256, 40, alpha=0.1)
    st = k3_state(w, np.float32)
    s64 = {k: v.astype(np.float64) for k, v in st.items()}
    nsteps = 20
    sim = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=32, element_order=2)
    sim.step(nsteps)
    hist = sim.history(0, 0, nsteps) + [sim.diagnostics(0)]
    got = sim.state_numpy(0)
    Wr, Hr, ref = FR.fp32_fused_reference_k3(s64, w, nsteps)
    errW = np.linalg.norm([h["W"] for h in hist] - Wr) / np.linalg.norm(Wr)
    errH = np.linalg.norm([h["H"] for h in hist] - Hr) / np.linalg.norm(Hr)
    assert errW < 1e-5 and errH < 1e-5, (errW, errH)
    for k, r in zip(K3, ref):
        x = np.asarray(got[k], dtype=np.float64)
        assert np.linalg.norm(x - r) <= 1e-5 * np.linalg.norm(r), k
    sim.close()


def test_full_size_two_stream(vp):
    """The two-stream workload at 2^20 particles, Ng 512, P2, with second moments: three
    fused steps in float64 against the oracle, every particle compared."""
    w = W.two_stream()
    st = w.state(moments=True)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=8, element_order=2)
    sim.set_tuning(threads=1024, ppt=4, acc_copies=4, graph_steps=3)
    sim.step(3)
    got = sim.state_numpy(0)
    ref, _, ref_hist = O.run_k3(st, w.L, w.ng, w.dt, 3)
    for k, r in zip(K3, ref):
        scale = max(1.0, float(np.max(np.abs(r))))
        assert np.max(np.abs(got[k] - r)) <= 1e-9 * scale, k
    d = sim.diagnostics(0)
    assert abs(d["W"] - ref_hist[-1]["W"]) <= 1e-9 * ref_hist[-1]["W"]
    sim.close()


def test_refused_configurations(vp):
    w = lattice(16, 64, 16)
    st = k3_state(w)
    for kw in (dict(element_order=1), dict(element_order=2, sort_every=4),
               dict(element_order=2, monopole_only=True)):
        with pytest.raises(vp.VPError) as e:
            vp.Simulation(st, w.L, w.ng, w.dt, "fp64", **kw)
        assert e.value.status == vp._lib.VP_ERR_ARG, kw
    with pytest.raises(vp.VPError):
        vp.Simulation(k3_state(w, np.float32), w.L, w.ng, w.dt, "fp32", element_order=2)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", element_order=2)
    with pytest.raises(vp.VPError):
        sim.set_tuning(threads=512, ppt=2, persistent=1)
    with pytest.raises(vp.VPError):
        sim.sort(0)
    sim.step(2)
    assert sim.diagnostics(0)["step"] == 2
    sim.close()
