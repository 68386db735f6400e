"""Parity at the benchmark sizes, in the launch shapes the benchmark's autotuner picks.

One fused step from the initial state, checked on the same input bits:
  * the particle update is the oracle's kick and drift applied to the device's own field
    (the materialised field of the initial state), computed in float64 from the stored
    float32 values in the kernel's operation order and stored in float32: bit-exact;
  * the neutralised load and field of the stepped state against the oracle's on the same
    (device) bits: relative L2 <= 1e-5;
  * the cell index of every particle of the stepped state: bit-exact.

Two-stream: N = 2^20, Ng = 512, fp32c, 512 threads x 4 particles per thread, 8 accumulator
copies.  Batched sweep: all 256 instances (sum N = 6.05e6), 512 x 8, 1 copy; sampled
instances are checked.  Nonlinear Landau (the precision study): N = 2^22, Ng = 256, in
float64, fp32c and fp32ts, 512 x 8, 8 copies.  The two-stream workload as plain
particle-in-cell particles, and with P2 elements (see its test for its bars).  (Over several steps, FP32 states computed with different rounding
sequences separate where a particle sits within an ulp of a node, so multi-step runs are
compared through the field-energy history in the other test files.)"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def first_fused_step_reference(st, f0, w, store=np.float32):
    """The first fused step (no pending half-kick yet): half-kick with the initial field,
    drift, all in float64 from the stored state, each stored value rounded once to the
    storage type."""
    Q, P, qs, ps = (st[k].astype(np.float64) for k in ("Q", "P", "qs", "ps"))
    P, qs = O.kick(Q, P, qs, ps, f0["E"], f0["g"], w.L, 0.5 * w.dt)
    Qn, psn = O.drift(Q, P, qs, ps, w.L, w.dt)
    return {"Q": Qn.astype(store), "P": P.astype(store), "qs": qs.astype(store),
            "ps": psn.astype(store)}


def check_slot(eng, slot, st, f0, w, store=np.float32, field_tol=1e-5):
    raw = {k: v.detach().cpu().numpy() for k, v in eng.state(slot).items()}  # P, q* pending
    ref = first_fused_step_reference(st, f0, w, store)
    for k in ("Q", "P", "qs", "ps"):
        assert raw[k].dtype == store, (slot, k)
        assert np.array_equal(raw[k], ref[k]), (slot, k)
    d = eng.diagnostics(slot, grid=True)
    fld = O.solve_field(raw["Q"].astype(np.float64), raw["ps"].astype(np.float64),
                        raw["psi"].astype(np.float64), w.L, w.ng)
    assert rel_l2(d["bt"], fld["bt"]) < field_tol, slot
    assert rel_l2(d["E"], fld["E"]) < field_tol, slot
    cells = eng.cell_index(slot).cpu().numpy()
    i, _ = O.cell_index(raw["Q"], w.L, w.ng)
    assert np.array_equal(cells, i.astype(np.int32)), slot


def test_two_stream_full_size_fused_step(vp):
    w = W.two_stream()
    st = w.state(np.float32)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=16)
    sim.set_tuning(threads=512, ppt=4, acc_copies=8, use_graph=1, graph_steps=3)
    f0 = sim.diagnostics(0, grid=True)
    sim.step(1)
    check_slot(sim, 0, st, f0, w)
    # and the graph path: three more steps replayed from a graph stay finite and counted
    sim.step(3)
    assert sim.diagnostics(0)["step"] == 4
    sim.close()


def test_batched_sweep_full_size_fused_step(vp):
    ws = W.landau_sweep()
    sts = [w.state(np.float32) for w in ws]
    eng = vp.Engine("fp32c", max_slots=len(ws))
    for s, (w, st) in enumerate(zip(ws, sts)):
        eng.admit(s, st, w.L, w.ng, w.dt, hist_cap=16)
    eng.set_tuning(threads=512, ppt=8, acc_copies=1, use_graph=1, graph_steps=3)
    sample = (0, 37, 101, 200, 255)
    f0 = {s: eng.diagnostics(s, grid=True) for s in sample}
    eng.step(1)
    for s in sample:
        check_slot(eng, s, sts[s], f0[s], ws[s])
    eng.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32ts"])
def test_landau_nonlinear_full_size_fused_step(vp, prec):
    """The precision study's workload at its full size (N = 2^22, Ng = 256) in the modes whose
    push arithmetic is float64: one fused step, bit-exact particle update on the device's
    own field, field of the stepped state against the oracle's (float64: summation order
    only, 1e-11; float32 storage: the stated 1e-5), cell indices bit-exact.  Launch shape
    512 threads x 8 particles per thread, 8 copies (1024 workgroups)."""
    w = W.landau_nonlinear()
    assert w.n == 1 << 22 and w.ng == 256
    st32 = w.state(np.float32)
    store = np.float64 if prec == "fp64" else np.float32
    st = {k: v.astype(store) for k, v in st32.items()}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=16)
    sim.set_tuning(threads=512, ppt=8, acc_copies=8, use_graph=1, graph_steps=3)
    f0 = sim.diagnostics(0, grid=True)
    sim.step(1)
    check_slot(sim, 0, st, f0, w, store, 1e-11 if prec == "fp64" else 1e-5)
    sim.close()


def test_monopole_two_stream_full_size_fused_step(vp):
    """The `--monopole` bench workload at full size: the two-stream lattice as plain
    particle-in-cell particles (p* = q* = 0), N = 2^20, fp32c, 512 x 4, 8 copies.  The
    monopole kernel instance never touches the dipole arrays, so the decorated reference
    with zero dipoles is its reference: bit-exact particle update, field within 1e-5."""
    w = W.two_stream()
    st = w.state(np.float32)
    st["qs"] = np.zeros_like(st["qs"])
    st["ps"] = np.zeros_like(st["ps"])
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=16, monopole_only=True)
    sim.set_tuning(threads=512, ppt=4, acc_copies=8, use_graph=1, graph_steps=3)
    f0 = sim.diagnostics(0, grid=True)
    sim.step(1)
    check_slot(sim, 0, st, f0, w)
    sim.close()


def within_one_ulp32(a, b):
    """Every float32 value of a is b's float64 value rounded to float32, give or take one
    float32 ulp (the reference's float64 result differs from the device's by a few float64
    ulps: one rounding to float32 can then land on a neighbour, never further)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mag = np.maximum(np.abs(a), np.abs(b)).astype(np.float32)
    return bool(np.all(np.abs(a - b) <= np.spacing(mag).astype(np.float64)))


def test_p2_two_stream_full_size_fp32c(vp):
    """The `--element-order 2` bench workload at full size and in the bench's precision and
    shape (N = 2^20, Ng 512, fp32c, 512 x 4, 4 copies), one fused step from the same float32
    bits.

    * The initial P2 field (midpoint E and phi_h'' per element) against the oracle's
      solve, relative to the largest value: 1e-9.  The oracle takes phi_h'' as second
      differences of the solved potential, which loses about five digits to cancellation
      at this mesh (3.7e-11 measured); the device uses the equivalent condensed form
      -(3 / 2h) times the neutralised midpoint load.
    * The particle update is the oracle's kick and drift applied to the device's own field:
      q* exactly (the same float64 products), Q, P and p* within one float32 ulp, because
      the device evaluates the linear element field as its midpoint value plus a slope term
      and the oracle as its left value plus the slope, which differ by float64 rounding.
    * The field energy of the stepped state against the oracle's P2 solve on the device's
      own stepped bits (relative 1e-5)."""
    w = W.two_stream()
    st = w.state(np.float32)
    h = w.L / w.ng
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=16, element_order=2)
    sim.set_tuning(threads=512, ppt=4, acc_copies=4, use_graph=1, graph_steps=3)
    Q0, P0, qs0, ps0, psi = (st[k].astype(np.float64) for k in ("Q", "P", "qs", "ps", "psi"))
    d0 = sim.diagnostics(0, grid=True)
    ora = O.solve_field_p2(Q0, ps0, psi, w.L, w.ng)
    for k in ("E", "g"):
        assert np.max(np.abs(d0[k] - ora[k])) <= 1e-9 * np.max(np.abs(ora[k])), k
    sim.step(1)
    raw = {k: v.detach().cpu().numpy() for k, v in sim.state(0).items()}  # P, q* pending
    own = {"E0": d0["E"] + 0.5 * h * d0["g"], "E1": -h * d0["g"], "g": d0["g"]}
    P1, qs1 = O.kick_p2(Q0, P0, qs0, ps0, own, w.L, 0.5 * w.dt)
    Q1, ps1 = O.drift(Q0, P1, qs1, ps0, w.L, w.dt)
    assert raw["qs"].dtype == np.float32
    assert np.array_equal(raw["qs"], qs1.astype(np.float32))
    for k, r in (("Q", Q1), ("P", P1), ("ps", ps1)):
        assert raw[k].dtype == np.float32, k
        assert within_one_ulp32(raw[k], r), k
    fld1 = O.solve_field_p2(raw["Q"].astype(np.float64), raw["ps"].astype(np.float64),
                            raw["psi"].astype(np.float64), w.L, w.ng)
    W1 = sim.diagnostics(0)["W"]
    assert abs(W1 - fld1["W"]) <= 1e-5 * fld1["W"]
    sim.close()


@pytest.mark.parametrize("copies", [4, 8])
def test_two_stream_full_size_persistent_steps(vp, copies):
    """The bench's default workload (N = 2^20, Ng 512, fp32c) in the persistent shapes its
    autotuner picks (1024 threads x 4 particles per thread, 256 workgroups, 4 or 8 copies).

    * One persistent launch of one step: the particle update is bit-exact against the
      oracle's kick and drift on the device's own initial field, the field of the stepped
      state within 1e-5 of the oracle's on the same bits, the cell indices bit-exact.
    * Then 30 more steps in one persistent launch: the field-energy and energy histories
      against the float32-storage reference of the fused step (the oracle's sub-flows in
      float64, stored in float32 where the kernel stores), relative L2 1e-5, and the final
      state against it (rel-L2 1e-5)."""
    from fp32_reference import fp32_fused_reference
    w = W.two_stream()
    st = w.state(np.float32)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32c", hist_cap=64)
    sim.set_tuning(threads=1024, ppt=4, acc_copies=copies, persistent=1)
    assert sim.get_tuning()["persistent"] == 1
    f0 = sim.diagnostics(0, grid=True)
    sim.step(1)
    check_slot(sim, 0, st, f0, w)
    more = 30
    sim.step(more)
    n = 1 + more
    hist = sim.history(0, 0, n) + [sim.diagnostics(0)]
    assert [h["step"] for h in hist] == list(range(n + 1))
    s64 = {k: v.astype(np.float64) for k, v in st.items()}
    Wr, Hr, (Q, P, qs, ps) = fp32_fused_reference(s64, w, n)
    assert rel_l2([h["W"] for h in hist], Wr) < 1e-5
    assert rel_l2([h["H"] for h in hist], Hr) < 1e-5
    got = sim.state_numpy(0)
    for k, r in (("Q", Q), ("P", P), ("qs", qs), ("ps", ps)):
        assert rel_l2(got[k], r) < 1e-5, k
    sim.close()


@pytest.mark.parametrize("persistent", [0, 1])
def test_two_stream_full_size_fp64_run_against_oracle(vp, persistent):
    """The two-stream workload at full size in float64 (N = 2^20, Ng 512), 33 steps against
    the oracle's run from the same bits: graph-replayed fused launches (512 threads x 4,
    8 copies, graphs of 3 steps, so every ring phase is replayed) or one persistent launch
    (1024 x 4, 4 copies).  The two sides differ in summation order only: state within
    1e-11 (absolute), W, K and H histories within 1e-10 (relative L2)."""
    w = W.two_stream()
    st = w.state(np.float64)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=64)
    if persistent:
        sim.set_tuning(threads=1024, ppt=4, acc_copies=4, persistent=1)
    else:
        sim.set_tuning(threads=512, ppt=4, acc_copies=8, use_graph=1, graph_steps=3)
    nsteps = 33
    sim.step(nsteps)
    hist = sim.history(0, 0, nsteps) + [sim.diagnostics(0)]
    got = sim.state_numpy(0)
    ref_state, _, ref_hist = O.run(*(st[k] for k in ("Q", "P", "qs", "ps", "psi")),
                                   w.L, w.ng, w.dt, nsteps)
    for k, r in zip(("Q", "P", "qs", "ps", "psi"), ref_state):
        assert np.max(np.abs(got[k] - r)) <= 1e-11, k
    for key in ("W", "K", "H"):
        assert rel_l2([h[key] for h in hist], [h[key] for h in ref_hist]) < 1e-10, key
    sim.close()
