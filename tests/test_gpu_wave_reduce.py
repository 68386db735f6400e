"""The wavefront-combined deposit (vp_tuning.wave_reduce = 1) against the oracle.

The combination applies to the compensated float32 mode (fp32ts), whose (hi, lo) pairs are
committed by a compare-and-swap per update; the modes that accumulate in float64 accept the
flag and keep their per-lane updates.  A state stored in cell order puts every lane of a
wavefront in one or two elements, so the segmented sums over runs of equal elements replace
most per-lane updates; a state in random order keeps the per-lane updates; a half-sorted
state mixes both within one launch.  Bars: the field of the stepped state against the
oracle's on the device's own bits (float64 and fp32c 1e-10, the two-sum pairs of fp32ts
1e-8), and fp32ts runs against the float32-storage reference (1e-5)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

FIELD_TOL = {"fp64": 1e-10, "fp32c": 1e-10, "fp32ts": 1e-8}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def arranged_state(w, how, store=np.float64):
    """The workload's state in cell order ("sorted"), in its random order ("random"), or
    its first half in cell order and the rest random ("half")."""
    st = {k: v.astype(store) for k, v in w.state(np.float64).items()}
    n = len(st["Q"])
    if how == "random":
        return st
    key = np.floor(st["Q"].astype(np.float64) * (w.ng / w.L))
    if how == "sorted":
        perm = np.argsort(key, kind="stable")
    else:
        h = n // 2
        perm = np.concatenate([np.argsort(key[:h], kind="stable"), np.arange(h, n)])
    return {k: v[perm].copy() for k, v in st.items()}


@pytest.mark.parametrize("how", ["sorted", "random", "half"])
@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32ts"])
@pytest.mark.parametrize("persistent", [0, 1])
def test_stepped_field_matches_oracle(vp, how, prec, persistent):
    """One step with the combined deposit: the deposited field of the stepped state against
    the oracle's solve of the same state bits; 16390 particles (a ragged last tile)."""
    w = W.landau_linear(seed=5, nx=149, nv=110, ng=64)
    w.params["alpha"] = 0.2
    store = np.float64 if prec == "fp64" else np.float32
    st = arranged_state(w, how, store)
    assert len(st["Q"]) == 16390
    sim = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=16)
    sim.set_tuning(threads=512, ppt=4, acc_copies=2, persistent=persistent, wave_reduce=1)
    assert sim.get_tuning()["wave_reduce"] == 1
    sim.step(1)
    d = sim.diagnostics(0, grid=True)
    got = sim.state_numpy(0)
    ref = O.solve_field(*(got[k].astype(np.float64) for k in ("Q", "ps", "psi")), w.L, w.ng)
    assert rel_l2(d["bt"], ref["bt"]) < FIELD_TOL[prec]
    assert rel_l2(d["E"], ref["E"]) < FIELD_TOL[prec]
    assert abs(d["W"] - ref["W"]) <= FIELD_TOL[prec] * ref["W"]
    sim.close()


@pytest.mark.parametrize("persistent", [0, 1])
def test_fp32ts_run_matches_storage_reference(vp, persistent):
    """31 fp32ts steps from a state in cell order (runs shrink as particles drift apart, so
    both the combined and the per-lane branch run) against the oracle's sub-flows with the
    fused step's float32 storage points: W and H histories and the final state within 1e-5."""
    from fp32_reference import fp32_fused_reference
    w = W.landau_linear(seed=6, nx=128, nv=96, ng=64)
    w.params["alpha"] = 0.2
    st = arranged_state(w, "sorted", np.float32)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32ts", hist_cap=64)
    sim.set_tuning(threads=1024, ppt=2, acc_copies=4, persistent=persistent, wave_reduce=1)
    nsteps = 31
    sim.step(nsteps)
    hist = sim.history(0, 0, nsteps) + [sim.diagnostics(0)]
    s64 = {k: v.astype(np.float64) for k, v in st.items()}
    Wr, Hr, (Q, P, qs, ps) = fp32_fused_reference(s64, w, nsteps)
    assert rel_l2([h["W"] for h in hist], Wr) < 1e-5
    assert rel_l2([h["H"] for h in hist], Hr) < 1e-5
    got = sim.state_numpy(0)
    for k, r in (("Q", Q), ("P", P), ("qs", qs), ("ps", ps)):
        assert rel_l2(got[k], r) < 1e-5, k


def test_sorted_stepping_with_combined_deposit(vp):
    """Periodic cell sorts keep the runs long; the diagnostics equal those of the unsorted
    per-lane fp32ts run to float32 storage precision (1e-5)."""
    w = W.landau_linear(seed=2, nx=256, nv=32, ng=128)
    w.params["alpha"] = 0.2
    st = w.state(np.float32)
    a = vp.Simulation(st, w.L, w.ng, w.dt, "fp32ts", sort_every=3, sort_chunk=512)
    b = vp.Simulation(st, w.L, w.ng, w.dt, "fp32ts")
    a.set_tuning(wave_reduce=1)
    a.step(10)
    b.step(10)
    da, db = a.diagnostics(0), b.diagnostics(0)
    for k in ("K", "W", "H", "momentum", "charge"):
        assert abs(da[k] - db[k]) <= 1e-5 * max(1.0, abs(db[k])), k


def test_p2_combined_deposit(vp):
    """P2 elements (three nodes per particle) with the combined fp32ts deposit, state in cell
    order: the stepped field against the oracle's P2 solve of the device's own bits (1e-8 of
    each array's scale)."""
    w = W.landau_linear(seed=7, nx=128, nv=64, ng=64)
    w.params["alpha"] = 0.2
    st = arranged_state(w, "sorted", np.float32)
    sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp32ts", hist_cap=16, element_order=2)
    sim.set_tuning(threads=512, ppt=4, acc_copies=2, wave_reduce=1)
    sim.step(1)
    d = sim.diagnostics(0, grid=True)
    got = {k: v.astype(np.float64) for k, v in sim.state_numpy(0).items()}
    ref = O.solve_field_p2(got["Q"], got["ps"], got["psi"], w.L, w.ng)
    for k in ("E", "g"):
        assert np.max(np.abs(d[k] - ref[k])) <= 1e-8 * np.max(np.abs(ref[k])), k


def test_wave_reduce_is_validated(vp):
    w = W.landau_linear(seed=1, nx=32, nv=16, ng=32)
    sim = vp.Simulation(w.state(), w.L, w.ng, w.dt, "fp64")
    with pytest.raises(vp.VPError):
        sim.set_tuning(wave_reduce=2)
    assert sim.get_tuning()["wave_reduce"] == 0
