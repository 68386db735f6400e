"""Checkpoint and resume through the C-ABI: a state read back after n steps (the read-back
applies the pending half-kick first) and admitted into a fresh engine continues as the
uninterrupted run does.

The resumed run deposits its first load with the admission kernel, the uninterrupted one
with the fused step, so the two loads differ in the order of their floating-point sums
only; in float64 the trajectories then agree to rounding (bar 1e-10 relative over the
linear-Landau horizon).  In float32 storage the read-back also rounds P and q* to float32
after the pending half-kick, where the uninterrupted run carries them in float64 into the
next half-kick, so the bar there is the stated float32 one (1e-5).  Also: two runs of one
input agree to summation-order rounding."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("Q", "P", "qs", "ps", "psi")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("fp32c", 1e-5)])
def test_resume_equals_uninterrupted(vp, prec, bar):
    w = W.landau_linear()
    st = w.state(np.float64 if prec == "fp64" else np.float32)
    n, m = 40, 60
    whole = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=n + m + 8)
    whole.step(n + m)
    ref = whole.state_numpy(0)
    w_ref = whole.diagnostics(0)["W"]
    whole.close()

    first = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=n + 8)
    first.step(n)
    saved = first.state_numpy(0)          # pending half-kick applied
    assert first.diagnostics(0)["step"] == n
    first.close()
    assert np.array_equal(saved["psi"], st["psi"])       # psi* is a Casimir: untouched
    resumed = vp.Simulation(saved, w.L, w.ng, w.dt, prec, hist_cap=m + 8)
    resumed.step(m)
    got = resumed.state_numpy(0)
    for k in FIELDS:
        assert got[k].dtype == ref[k].dtype, k
        assert rel_l2(got[k], ref[k]) <= bar, k
    assert abs(resumed.diagnostics(0)["W"] - w_ref) <= bar * w_ref
    resumed.close()


def test_two_identical_runs_agree_to_summation_order(vp):
    """Run-to-run reproducibility.  The deposit sums in float64 LDS and device atomics, whose
    order varies from run to run, so two runs of the same input agree to rounding, not
    bitwise: in float64 over 100 linear-Landau steps the states agree to 1e-12 relative."""
    w = W.landau_linear()
    st = w.state(np.float64)
    out = []
    for _ in range(2):
        sim = vp.Simulation(st, w.L, w.ng, w.dt, "fp64", hist_cap=128)
        sim.set_tuning(threads=512, ppt=1, acc_copies=4)
        sim.step(100)
        out.append((sim.state_numpy(0), sim.diagnostics(0)["W"]))
        sim.close()
    (a, wa), (b, wb) = out
    for k in FIELDS:
        assert rel_l2(a[k], b[k]) <= 1e-12, k
    assert abs(wa - wb) <= 1e-12 * wb
