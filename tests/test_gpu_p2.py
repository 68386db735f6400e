"""P2 elements (the degree-2 Lagrange space of eq. galerkin) on the HIP path against the
oracle's P2 functions.  The oracle assembles the P2 stiffness matrix and solves the bordered
system with the integral gauge, refined in extended precision; the kernels eliminate each
element's midpoint unknown and solve the P1 system that remains, so the two agree to the
kernels' float64 rounding: field values within 1e-12 of their scale at every mesh with the
scan solver (a NumPy model of the condensed solve in float64 is within 5e-15 of the oracle up
to Ng 1024) and max(1e-12, 1e-17 Ng^2) with the FFT solver, float64
trajectories 1e-10 (state, absolute) and 1e-10 (histories, relative to their scale).  Float32
state is held to the oracle's P2 sub-flows with the fused step's float32 storage points.
Edge cases: the smallest and largest meshes, a ragged tile tail, one particle, monopole-only
particles, a prescribed potential with and without the self field, the FFT solver, the
unfused primitive steps, an engine mixing P1 and P2 instances, every precision that P2
takes, and the configurations the library refuses."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("Q", "P", "qs", "ps", "psi")


def lattice(ng, nx, nv, alpha=0.05, seed=0):
    w = W.landau_linear(seed=seed, nx=nx, nv=nv, ng=ng)
    w.params["alpha"] = alpha
    return w


def field_tol(ng, solver="scan"):
    """The scan solve rounds like a prefix sum (a float64 model of it is within 1e-14 of the
    oracle up to Ng 1024); the FFT solve divides rounding of the high modes by eigenvalues
    that fall like 1/Ng^2 (a float64 NumPy model is 1.8e-12 off at Ng 1024, 1.1e-13 at 256)."""
    return 1e-12 if solver == "scan" else max(1e-12, 1e-17 * ng * ng)


def close(a, b, tol):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) <= tol * max(1e-300, float(np.max(np.abs(b))))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_run(st, L, ng, dt, nsteps, **kw):
    return O.run_p2(*(np.asarray(st[k], dtype=np.float64) for k in FIELDS), L, ng, dt, nsteps,
                    **kw)


def check_run(eng, st, L, ng, dt, nsteps, slot=0, **kw):
    got = eng.state_numpy(slot)
    hist = eng.history(slot, 0, nsteps) + [eng.diagnostics(slot)]
    ref_state, _, ref_hist = oracle_run(st, L, ng, dt, nsteps, **kw)
    for k, r in zip(FIELDS, ref_state):
        assert np.allclose(got[k], r, rtol=0, atol=1e-10), k
    for key in ("K", "W", "U", "H", "momentum", "e1_re", "e1_im"):
        g = np.array([h[key] for h in hist])
        r = np.array([h[key] for h in ref_hist])
        scale = max(1e-300, float(np.max(np.abs(r))))
        assert np.max(np.abs(g - r)) <= 1e-10 * scale or np.max(np.abs(g - r)) < 1e-14, key
    return hist, ref_hist


@pytest.mark.parametrize("ng,solver", [(8, "scan"), (64, "scan"), (64, "fft"), (1024, "scan"),
                                       (1024, "fft")])
def test_field_at_t0(vp, ng, solver):
    """The solved field of the initial state, node by node: b~ and Phi of the vertices and
    midpoints (integral gauge), E at the element midpoints, phi_h'' per element, and W."""
    w = lattice(ng, max(64, 4 * ng), 16)
    st = w.state()
    sim = vp.Simulation(st, w.L, ng, w.dt, "fp64", hist_cap=4, solver=solver, element_order=2)
    d = sim.diagnostics(0, grid=True)
    f = O.solve_field_p2(st["Q"], st["ps"], st["psi"], w.L, ng)
    tol = field_tol(ng, solver)
    assert d["bt"].shape == (2 * ng,) and d["Phi"].shape == (2 * ng,)
    assert close(d["bt"], np.concatenate([f["btv"], f["btm"]]), tol)
    assert close(d["Phi"], np.concatenate([f["Phv"], f["Phm"]]), tol)
    assert close(d["E"], f["E"], tol)
    assert close(d["g"], f["g"], tol)
    assert abs(d["W"] - f["W"]) <= tol * f["W"]
    h = w.L / ng
    # the integral gauge and the neutral load, by their definitions
    assert abs(h / 3 * d["Phi"][:ng].sum() + 2 * h / 3 * d["Phi"][ng:].sum()) < 1e-12 * np.abs(
        d["Phi"]).max() * w.L
    assert abs(d["bt"].sum()) < 1e-12 * np.sum(st["psi"])
    sim.close()


@pytest.mark.parametrize("solver,threads,ppt,copies,graph", [
    ("scan", 256, 1, 1, 3), ("fft", 1024, 4, 3, 6), ("scan", 512, 2, 8, 0),
    ("scan", 1024, 8, 2, 9)])
def test_trajectory_matches_oracle(vp, solver, threads, ppt, copies, graph):
    """Fused P2 steps, every launch shape: a ragged tail (n not a multiple of any tile)."""
    w = lattice(32, 128, 40, alpha=0.1)
    st = {k: v[:-37] for k, v in w.state().items()}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64, solver=solver, element_order=2)
    sim.set_tuning(threads=threads, ppt=ppt, acc_copies=copies, use_graph=1 if graph else 0,
                   graph_steps=max(1, graph))
    sim.step(20)
    check_run(sim, st, w.L, w.ng, w.dt, 20)
    sim.close()


@pytest.mark.parametrize("solver", ["scan", "fft"])
def test_largest_mesh_trajectory(vp, solver):
    """The largest mesh (Ng 1024: four vertices and four midpoints per solving thread, a
    2048-node deposit grid in LDS) through fused steps."""
    w = lattice(1024, 4096, 16, alpha=0.1)
    st = w.state()
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=16, solver=solver,
                        element_order=2)
    sim.set_tuning(threads=1024, ppt=2, acc_copies=4, graph_steps=3)
    sim.step(6)
    got = sim.state_numpy(0)
    ref, fld, _ = oracle_run(st, w.L, w.ng, w.dt, 6)
    for k, r in zip(FIELDS, ref):
        assert np.allclose(got[k], r, rtol=0, atol=1e-9), k
    d = sim.diagnostics(0, grid=True)
    # after six steps the field inherits the trajectories' difference (positions within 1e-9
    # of the oracle's), so it is held to that bar rather than to the same-bits field bar
    assert close(d["E"], fld["E"], 1e-9) and close(d["g"], fld["g"], 1e-9)
    sim.close()


def test_primitive_steps_equal_one_oracle_step(vp):
    """The unfused composition (gather_push, deposit, poisson, gather_push) with P2."""
    w = lattice(16, 64, 24, alpha=0.2)
    st = w.state()
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=8, element_order=2)
    for _ in range(3):
        sim.gather_push(0.5 * w.dt, w.dt)
        sim.deposit()
        sim.poisson()
        sim.gather_push(0.5 * w.dt, 0.0)
    got = sim.state_numpy(0)
    ref, fld, _ = oracle_run(st, w.L, w.ng, w.dt, 3)
    for k, r in zip(FIELDS, ref):
        assert np.allclose(got[k], r, rtol=0, atol=1e-12), k
    d = sim.diagnostics(0, grid=True)
    assert close(d["E"], fld["E"], 1e-12) and close(d["g"], fld["g"], 1e-12)
    sim.close()


def test_monopole_only_p2(vp):
    """Plain particle-in-cell with P2 elements: the dipoles stay zero."""
    w = lattice(32, 128, 32, alpha=0.1)
    st = w.state()
    st["qs"] = np.zeros_like(st["Q"])
    st["ps"] = np.zeros_like(st["Q"])
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=32, monopole_only=True,
                        element_order=2)
    sim.set_tuning(threads=512, ppt=2, acc_copies=2, graph_steps=3)
    sim.step(15)
    check_run(sim, st, w.L, w.ng, w.dt, 15)
    got = sim.state_numpy(0)
    assert not got["qs"].any() and not got["ps"].any()
    sim.close()


@pytest.mark.parametrize("self_field", [True, False])
def test_prescribed_potential_with_p2(vp, self_field):
    w = lattice(32, 128, 32, alpha=0.1)
    st = w.state()
    ext = {"amp": 0.3, "mode": 2}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=32, external=ext,
                        self_field=self_field, element_order=2)
    sim.set_tuning(threads=256, ppt=4, acc_copies=2, graph_steps=3)
    sim.step(12)
    hist, _ = check_run(sim, st, w.L, w.ng, w.dt, 12, ext=ext, self_field=self_field)
    assert max(abs(h["U"]) for h in hist) > 0.0
    if not self_field:
        assert all(h["W"] == 0.0 for h in hist)
    sim.close()


def test_one_particle_and_retire(vp):
    """A single decorated particle (its own field only): retire returns the state at the
    integer step, on the oracle's trajectory."""
    st = {"Q": np.array([1.3]), "P": np.array([0.4]), "qs": np.array([0.02]),
          "ps": np.array([-0.05]), "psi": np.array([1.0])}
    L, ng, dt = 5.0, 8, 0.05
    eng = vp.Engine("fp64", max_slots=1)
    eng.admit(0, st, L, ng, dt, hist_cap=16, element_order=2)
    eng.step(10)
    out = eng.retire(0)
    ref, _, _ = oracle_run(st, L, ng, dt, 10)
    for k, r in zip(FIELDS, ref):
        assert np.allclose(out[k].cpu().numpy(), r, rtol=0, atol=1e-12), k
    eng.close()


@pytest.mark.parametrize("persistent", [0, 1])
def test_engine_mixing_p1_and_p2(vp, persistent):
    """P1 and P2 instances of different meshes in one engine (one launch per kind of tile, or
    one persistent launch for all of them, in the kernel instance with P2 elements and
    general options): each on its own oracle trajectory."""
    specs = [dict(ng=64, order=1), dict(ng=32, order=2), dict(ng=16, order=2, mono=True),
             dict(ng=128, order=2, solver="fft"), dict(ng=32, order=1, ext={"amp": 0.2, "mode": 1})]
    eng = vp.Engine("fp64", max_slots=len(specs))
    sts = []
    for s, sp in enumerate(specs):
        w = lattice(sp["ng"], 4 * sp["ng"], 16, alpha=0.1, seed=s)
        st = w.state()
        if sp.get("mono"):
            st["qs"] = np.zeros_like(st["Q"])
            st["ps"] = np.zeros_like(st["Q"])
        sts.append((w, st))
        eng.admit(s, st, w.L, w.ng, w.dt, hist_cap=16, solver=sp.get("solver", "scan"),
                  monopole_only=sp.get("mono", False), external=sp.get("ext"),
                  element_order=sp["order"])
    eng.set_tuning(threads=512, ppt=2, acc_copies=2, graph_steps=3, persistent=persistent)
    eng.step(9)
    for s, (sp, (w, st)) in enumerate(zip(specs, sts)):
        if sp["order"] == 2:
            check_run(eng, st, w.L, w.ng, w.dt, 9, slot=s)
        else:
            got = eng.state_numpy(s)
            ext = sp.get("ext")
            ref, _, _ = O.run(*(st[k] for k in FIELDS), w.L, w.ng, w.dt, 9, ext=ext)
            for k, r in zip(FIELDS, ref):
                assert np.allclose(got[k], r, rtol=0, atol=1e-10), (s, k)
    eng.close()


@pytest.mark.parametrize("prec", ["fp32c", "fp32ts"])
def test_float32_state_matches_storage_reference(vp, prec):
    """P2 with float32 state (float64 particle arithmetic and accumulation) over 20 fused
    steps against the oracle's P2 sub-flows with the fused step's float32 storage points: W
    and H histories and the final state within 1e-5.  The departure from the float64 oracle
    run from the same bits is reported, not held: float32 rounding of positions moves the
    load through the basis slopes (up to 4/h for P2)."""
    import fp32_reference as FR
    w = W.two_stream(nx=256, nv=128, ng=64)
    st = w.state(np.float32)
    s64 = {k: v.astype(np.float64) for k, v in st.items()}
    nsteps = 20
    a = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=32, element_order=2)
    a.step(nsteps)
    ha = a.history(0, 0, nsteps) + [a.diagnostics(0)]
    got = a.state_numpy(0)
    a.close()
    Wr, Hr, (Q, P, qs, ps) = FR.fp32_fused_reference(s64, w, nsteps, order=2)
    errW = np.linalg.norm([h["W"] for h in ha] - Wr) / np.linalg.norm(Wr)
    errH = np.linalg.norm([h["H"] for h in ha] - Hr) / np.linalg.norm(Hr)
    _, _, ref = oracle_run(s64, w.L, w.ng, w.dt, nsteps)
    Wo = np.array([h["W"] for h in ref])
    dev = np.linalg.norm([h["W"] for h in ha] - Wo) / np.linalg.norm(Wo)
    print(f"\n[precision] P2 {prec}: W rel L2 vs float32-storage reference {errW:.3e}, H {errH:.3e}; "
          f"W vs float64 oracle {dev:.3e}")
    assert errW < 1e-5 and errH < 1e-5, (errW, errH)
    for k, r in (("Q", Q), ("P", P), ("qs", qs), ("ps", ps)):
        x = np.asarray(got[k], dtype=np.float64)
        assert np.linalg.norm(x - r) <= 1e-5 * np.linalg.norm(r), k


def test_full_size_two_stream(vp):
    """The two-stream workload at full size (2^20 particles, Ng 512) with P2: three fused
    steps against the oracle, every particle compared."""
    w = W.two_stream()
    st = w.state()
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=8, element_order=2)
    sim.set_tuning(threads=1024, ppt=4, acc_copies=4, graph_steps=3)
    sim.step(3)
    got = sim.state_numpy(0)
    ref, _, ref_hist = oracle_run(st, w.L, w.ng, w.dt, 3)
    for k, r in zip(FIELDS, ref):
        assert np.allclose(got[k], r, rtol=0, atol=1e-9), k
    d = sim.diagnostics(0)
    assert abs(d["W"] - ref_hist[-1]["W"]) <= field_tol(w.ng) * ref_hist[-1]["W"]
    sim.close()


def test_refused_configurations(vp):
    w = lattice(16, 64, 16)
    st = w.state()
    with pytest.raises(vp.VPError):
        vp.Simulation(st, w.L, w.ng, w.dt, "fp32", element_order=2)
    with pytest.raises(vp.VPError):
        vp.Simulation(st, w.L, w.ng, w.dt, "fp64", projection="nodal", element_order=2)
    with pytest.raises(vp.VPError):
        vp.Simulation(st, w.L, w.ng, w.dt, "fp64", element_order=3)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", element_order=2)
    with pytest.raises(vp.VPError):
        sim.set_tuning(threads=256, ppt=2, persistent=1)  # persistent steps: 512 or 1024
    assert sim.get_tuning()["persistent"] == 0
    sim.step(2)                                   # still steps after the refusal
    sim.close()


@pytest.mark.parametrize("threads,ppt,copies", [(1024, 4, 4), (512, 2, 2)])
def test_persistent_trajectory_matches_oracle(vp, threads, ppt, copies):
    """P2 instances in persistent launches (particles in registers between steps), a ragged
    tail, float64 against the oracle's P2 run (state 1e-10, histories 1e-10 of scale)."""
    w = lattice(32, 128, 40, alpha=0.1)
    st = {k: v[:-37] for k, v in w.state().items()}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64, element_order=2)
    sim.set_tuning(threads=threads, ppt=ppt, acc_copies=copies, persistent=1)
    assert sim.get_tuning()["persistent"] == 1
    sim.step(7)
    sim.step(13)                                  # two launches: the ring carries over
    check_run(sim, st, w.L, w.ng, w.dt, 20)
    sim.close()


def test_persistent_at_the_largest_grid(vp):
    """P2 at Ng = 1024 (a 2048-node load vector) in persistent launches: float64 against the
    oracle's P2 run, a ragged tail, two launches."""
    w = lattice(1024, 2048, 16, alpha=0.1, seed=3)
    st = {k: v[:-5] for k, v in w.state().items()}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=32, element_order=2)
    sim.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=1)
    sim.step(5)
    sim.step(4)
    check_run(sim, st, w.L, w.ng, w.dt, 9)
    sim.close()


def test_persistent_full_size_two_stream_fp32c(vp):
    """The `--element-order 2` workload at full size (2^20, Ng 512, fp32c) in persistent
    launches (1024 x 4, 4 copies), 31 steps against the P2 float32-storage reference:
    W and H histories and the final state within 1e-5."""
    from fp32_reference import fp32_fused_reference
    w = W.two_stream()
    st = w.state(np.float32)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=64, element_order=2)
    sim.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=1)
    n = 31
    sim.step(n)
    hist = sim.history(0, 0, n) + [sim.diagnostics(0)]
    s64 = {k: v.astype(np.float64) for k, v in st.items()}
    Wr, Hr, (Q, P, qs, ps) = fp32_fused_reference(s64, w, n, order=2)
    assert rel(np.array([h["W"] for h in hist]), Wr) < 1e-5
    assert rel(np.array([h["H"] for h in hist]), Hr) < 1e-5
    got = sim.state_numpy(0)
    for k, r in (("Q", Q), ("P", P), ("qs", qs), ("ps", ps)):
        assert rel(got[k], r) < 1e-5, k
    sim.close()
