"""The decorated-particle initialisation (the paper's Algorithm 1) on the HIP path against
the oracle: the final assignment of every marker, the number of decorated particles and
their Q, P, psi* and q* are bit-exact (sums run in marker order on both sides); p* goes
through sin on each side and is held to 1e-13 of its scale.  Edge cases: one cluster, one
marker per cluster, no Lloyd iteration, duplicate markers (ties), a single velocity."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def landau_markers(m, seed, L=4 * math.pi):
    w = W.landau_linear()
    w.params["alpha"] = 0.3
    w.L = L
    w.params["k"] = 2 * math.pi / L
    st = W.random_markers(w, m, seed=seed)
    return st["Q"], st["P"], st["psi"], L


def compare(vp, q, p, w, k, L, iters, init):
    got = vp.cluster_markers(q, p, w, k, L, iters=iters, init_idx=init, return_assign=True)
    ref, a = O.cluster_markers(q, p, w, init, iters, L)
    ga = got["assign"].cpu().numpy()
    assert np.array_equal(ga, a.astype(np.int32))
    n = ref["Q"].shape[0]
    assert got["Q"].shape[0] == n
    for f in ("Q", "P", "psi", "qs"):
        assert np.array_equal(got[f].cpu().numpy(), ref[f]), f
    ps = got["ps"].cpu().numpy()
    scale = max(1e-300, np.abs(ref["ps"]).max())
    assert np.max(np.abs(ps - ref["ps"])) <= 1e-13 * scale
    return got, ref


@pytest.mark.parametrize("m,k,iters", [(20000, 2000, 5), (7777, 300, 12), (4096, 4096, 2),
                                       (5000, 1, 3), (3000, 50, 0)])
def test_matches_oracle(vp, m, k, iters):
    q, p, w, L = landau_markers(m, seed=m + k)
    init = np.random.default_rng(k).choice(m, k, replace=False)
    compare(vp, q, p, w, k, L, iters, init)


def test_duplicate_markers_and_single_velocity(vp):
    """Markers at identical places (equal distances: ties go to the lower centre and the
    lower marker) and all at one velocity (a zero-height grid in p)."""
    rng = np.random.default_rng(3)
    L = 5.0
    base = rng.uniform(0, L, 400)
    q = np.concatenate([base, base, base[:100]])
    p = np.full(q.size, 0.25)
    w = rng.uniform(0.5, 1.5, q.size)
    init = np.concatenate([np.arange(40), 400 + np.arange(40)])   # duplicate centres too
    compare(vp, q, p, w, init.size, L, 4, init)


def test_rejects_bad_arguments(vp):
    q, p, w, L = landau_markers(1000, seed=1)
    with pytest.raises(vp.VPError):
        vp.cluster_markers(q, p, w, 10, L, init_idx=np.array([0, 1, 2, 3, 4, 5, 6, 7, 8, 1000]))
    with pytest.raises(vp.VPError):
        vp.cluster_markers(q, p, w, 1001, L)
    with pytest.raises(vp.VPError):
        vp.cluster_markers(q, p, w, 10, -1.0)


def test_full_size_properties(vp):
    """2^20 markers into 2^16 clusters: the decorated particles equal the oracle's moments
    of the device's own assignment (bit-exact but p*), every marker's weight is carried
    (charge), and the total momentum is kept to rounding."""
    m, k = 1 << 20, 1 << 16
    q, p, w, L = landau_markers(m, seed=11)
    got = vp.cluster_markers(q, p, w, k, L, iters=8, seed=5, return_assign=True)
    a = got["assign"].cpu().numpy()
    assert a.min() >= 0 and a.max() < k
    ref = O.cluster_moments(q, p, w, a, k, L)
    for f in ("Q", "P", "psi", "qs"):
        assert np.array_equal(got[f].cpu().numpy(), ref[f]), f
    assert np.max(np.abs(got["ps"].cpu().numpy() - ref["ps"])) <= 1e-13 * np.abs(ref["ps"]).max()
    psi = got["psi"].cpu().numpy()
    assert abs(psi.sum() - w.sum()) < 1e-12 * w.sum()
    mom = np.sum(psi * got["P"].cpu().numpy() + got["qs"].cpu().numpy())
    assert abs(mom - np.sum(w * p)) < 1e-10 * np.sum(np.abs(w * p))


def test_decorated_particles_run_in_the_engine(vp):
    """Clusters of random markers are a valid initial state: the engine steps them and
    matches the oracle run from the same decorated particles (float64)."""
    m, k = 40000, 4000
    q, p, w, L = landau_markers(m, seed=21)
    dec = vp.cluster_markers(q, p, w, k, L, iters=6, seed=2)
    st = {f: dec[f].cpu().numpy() for f in ("Q", "P", "qs", "ps", "psi")}
    ng, dt, nsteps = 64, 0.1, 15
    sim = vp.Simulation(st, L, ng, dt, "fp64", hist_cap=32)
    sim.step(nsteps)
    got = sim.state_numpy(0)
    ref_state, _, _ = O.run(st["Q"], st["P"], st["qs"], st["ps"], st["psi"], L, ng, dt, nsteps)
    for f, r in zip(("Q", "P", "qs", "ps", "psi"), ref_state):
        assert np.allclose(got[f], r, rtol=0, atol=1e-10), f
    sim.close()


# ---------------------------------------------------------------- mini-batch k-means

def compare_minibatch(vp, q, p, w, k, L, init, batches):
    got = vp.cluster_markers(q, p, w, k, L, init_idx=init, batch_idx=batches, return_assign=True)
    ref, a, v = O.cluster_markers_minibatch(q, p, w, init, list(batches), L)
    assert np.array_equal(got["absorbed"].cpu().numpy(), v)
    assert np.array_equal(got["assign"].cpu().numpy(), a.astype(np.int32))
    assert got["Q"].shape[0] == ref["Q"].shape[0]
    for f in ("Q", "P", "psi", "qs"):
        assert np.array_equal(got[f].cpu().numpy(), ref[f]), f
    ps = got["ps"].cpu().numpy()
    assert np.max(np.abs(ps - ref["ps"])) <= 1e-13 * max(1e-300, np.abs(ref["ps"]).max())
    return got, ref


@pytest.mark.parametrize("m,k,batch,nbatch", [(20000, 500, 4000, 10), (7777, 300, 1000, 25),
                                              (5000, 1, 100, 3), (3000, 50, 3000, 1),
                                              (4096, 4096, 512, 4)])
def test_minibatch_matches_oracle(vp, m, k, batch, nbatch):
    """Mini-batch updates: the absorbed weights, the final assignment and the decorated
    particles bit-exact (p* to 1e-13), batches drawn with replacement (repeats count)."""
    q, p, w, L = landau_markers(m, seed=m + k + 1)
    rng = np.random.default_rng(k + batch)
    init = rng.choice(m, k, replace=False)
    batches = rng.integers(0, m, (nbatch, batch))
    compare_minibatch(vp, q, p, w, k, L, init, batches)


def test_minibatch_one_full_batch_equals_one_lloyd_iteration(vp):
    """A single batch of every marker once is one Lloyd iteration: the same clusters as the
    Lloyd entry point with one iteration."""
    q, p, w, L = landau_markers(6000, seed=4)
    init = np.random.default_rng(1).choice(6000, 200, replace=False)
    a = vp.cluster_markers(q, p, w, 200, L, init_idx=init, batch_idx=np.arange(6000)[None, :],
                           return_assign=True)
    b = vp.cluster_markers(q, p, w, 200, L, iters=1, init_idx=init, return_assign=True)
    assert np.array_equal(a["assign"].cpu().numpy(), b["assign"].cpu().numpy())
    for f in ("Q", "P", "psi", "qs", "ps"):
        assert np.array_equal(a[f].cpu().numpy(), b[f].cpu().numpy()), f


def test_minibatch_rejects_bad_batches(vp):
    q, p, w, L = landau_markers(1000, seed=2)
    init = np.arange(10)
    with pytest.raises(vp.VPError):      # an index outside [0, m)
        vp.cluster_markers(q, p, w, 10, L, init_idx=init,
                           batch_idx=np.array([[0, 5, 1000, 3]]))
    with pytest.raises(vp.VPError):
        vp.cluster_markers(q, p, w, 10, L, init_idx=init, batch_idx=np.array([[-1, 2]]))
    with pytest.raises(vp.VPError):      # batch > m
        vp.cluster_markers(q, p, w, 10, L, init_idx=init, batch=1001, nbatch=2)
    with pytest.raises(vp.VPError):      # no batch
        vp.cluster_markers(q, p, w, 10, L, init_idx=init, batch=10, nbatch=0)


def test_minibatch_full_size_properties(vp):
    """2^20 markers, 2^16 clusters, 12 batches of 2^17: the absorbed weights add up to the
    weight of every drawn index, the decorated particles are the oracle's moments of the
    device's own assignment (bit-exact but p*), and every marker's weight is carried."""
    m, k = 1 << 20, 1 << 16
    q, p, w, L = landau_markers(m, seed=12)
    rng = np.random.default_rng(9)
    batches = rng.integers(0, m, (12, 1 << 17))
    got = vp.cluster_markers(q, p, w, k, L, seed=3, batch_idx=batches, return_assign=True)
    v = got["absorbed"].cpu().numpy()
    drawn = w[batches.ravel()].sum()
    assert abs(v.sum() - drawn) < 1e-10 * drawn
    a = got["assign"].cpu().numpy()
    assert a.min() >= 0 and a.max() < k
    ref = O.cluster_moments(q, p, w, a, k, L)
    for f in ("Q", "P", "psi", "qs"):
        assert np.array_equal(got[f].cpu().numpy(), ref[f]), f
    assert np.max(np.abs(got["ps"].cpu().numpy() - ref["ps"])) <= 1e-13 * np.abs(ref["ps"]).max()
    assert abs(got["psi"].cpu().numpy().sum() - w.sum()) < 1e-12 * w.sum()


def test_minibatch_duplicates_ties_and_single_marker_batches(vp):
    """Mini-batch updates over duplicate markers (equal distances: ties to the lower centre),
    all at one velocity, with batches of a single marker and a batch that repeats one
    index: bit-exact against the oracle."""
    rng = np.random.default_rng(13)
    L = 5.0
    base = rng.uniform(0, L, 300)
    q = np.concatenate([base, base])
    p = np.full(q.size, -0.75)
    w = rng.uniform(0.5, 1.5, q.size)
    init = np.concatenate([np.arange(20), 300 + np.arange(20)])   # duplicate centres too
    singles = rng.integers(0, q.size, (7, 1))
    compare_minibatch(vp, q, p, w, init.size, L, init, singles)
    repeated = np.full((1, 64), 17)
    compare_minibatch(vp, q, p, w, init.size, L, init, repeated)
