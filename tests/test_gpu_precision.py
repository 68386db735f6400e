"""Precision modes on the nonlinear Landau workload (alpha = 0.5, k = 0.5, Ng = 256,
N = 2^22, dt = 0.05) against the stored FP64 oracle history (tests/golden/, written by
make_landau_nonlinear_history.py from the same FP32-rounded initial state).

The field-energy history is compared over t <= 20, before the turbulent phase amplifies
the rounding of any summation order (FP64 included) to O(1) differences."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "landau_nonlinear_oracle.npz")
STEPS = 400  # t = 20
# relative L2 of W over t <= 10 and 10 < t <= 20
BARS = {"fp64": (1e-10, 1e-8), "fp32c": (1e-6, 1e-4), "fp32ts": (1e-6, 1e-4),
        "fp32": (1e-5, 1e-4)}


@pytest.fixture(scope="module")
def reference():
    ref = np.load(GOLDEN, allow_pickle=False)
    keys = [str(k) for k in ref["keys"]]
    return {k: ref["hist"][:STEPS + 1, keys.index(k)] for k in keys}


@pytest.fixture(scope="module")
def state32():
    return W.landau_nonlinear().state(np.float32)


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32ts", "fp32"])
def test_precision_mode_against_fp64_oracle(vp, prec, reference, state32):
    w = W.landau_nonlinear()
    st = {k: (v.astype(np.float64) if prec == "fp64" else v) for k, v in state32.items()}
    sim = vp.Simulation(st, w.L, w.ng, w.dt, prec, hist_cap=STEPS + 8)
    sim.step(STEPS)
    hist = sim.history(0, 0, STEPS) + [sim.diagnostics(0)]
    Wg = np.array([h["W"] for h in hist])
    Wo = reference["W"]
    t = reference["t"]
    for (lo, hi), bar in zip(((-1.0, 10.0), (10.0, 20.0)), BARS[prec]):
        m = (t > lo) & (t <= hi)
        err = np.linalg.norm(Wg[m] - Wo[m]) / np.linalg.norm(Wo[m])
        assert err < bar, (prec, lo, hi, err)
    chg = np.array([h["charge"] for h in hist])
    assert np.max(np.abs(chg - reference["charge"][0])) < 1e-12 * reference["charge"][0]
    sim.close()
