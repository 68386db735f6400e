"""The seeded input recipes (CPU): reproducible, in range, and normalised as stated."""
import math

import numpy as np

import workloads as W


def test_random_markers_recipe():
    w = W.landau_strong()
    a = W.random_markers(w, 20000, seed=3)
    b = W.random_markers(w, 20000, seed=3)
    assert all(np.array_equal(a[k], b[k]) for k in ("Q", "P", "psi"))
    assert a["Q"].min() >= 0.0 and a["Q"].max() < w.L
    # weights (1 + A cos kx) L / n: total charge L up to the sampling error of sum cos kx
    assert abs(a["psi"].sum() - w.L) < 5 * w.params["alpha"] * w.L / math.sqrt(20000)
    assert abs(np.mean(a["P"])) < 0.05 and abs(np.std(a["P"]) - 1.0) < 0.02
    c = W.random_markers(w, 20000, seed=4)
    assert not np.array_equal(a["Q"], c["Q"])


def test_landau_strong_parameters():
    w = W.landau_strong(nx=128, nv=16)
    assert w.L == 12.0 and w.ng == 128 and w.dt == 0.2
    assert abs(w.params["k"] - 2 * math.pi / 12.0) < 1e-15 and w.params["alpha"] == 0.5
    st = w.state()
    assert st["Q"].shape == (128 * 16,)
    # the lattice carries the whole charge of f0 over v in [-6, 6]
    assert abs(st["psi"].sum() - w.L) < 1e-6 * w.L
