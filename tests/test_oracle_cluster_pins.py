"""Pins of the initialisation oracle (Algorithm 1: k-means of markers, then each cluster's
decorated particle) against facts outside itself: brute force on tiny inputs, properties
of Lloyd's iteration, exactly recoverable clusters, and the identities the moment formulas
imply (charge, momentum and the first velocity moment are reproduced exactly; the first
position moment to third order in the cluster width; the periodic form of the spatial
moment across q = 0; a better load vector than monopoles at the centres)."""
import math

import numpy as np
import pytest

import oracle as O


def _markers(rng, m, L, pmax=3.0):
    q = rng.uniform(0, L, m)
    p = rng.uniform(-pmax, pmax, m)
    w = rng.uniform(0.5, 1.5, m)
    return q, p, w


def test_nearest_centre_brute_force_and_ties():
    rng = np.random.default_rng(0)
    q, p, _ = _markers(rng, 200, 5.0)
    cq, cp = rng.uniform(0, 5, 17), rng.uniform(-3, 3, 17)
    got = O.nearest_centre(q, p, cq, cp, chunk=7)
    for i in range(q.size):
        best, bi = math.inf, -1
        for c in range(cq.size):
            d = (q[i] - cq[c]) ** 2 + (p[i] - cp[c]) ** 2
            if d < best:
                best, bi = d, c
        assert got[i] == bi
    # a marker exactly between two centres goes to the lower index
    assert O.nearest_centre([1.0], [0.0], [0.0, 2.0], [0.0, 0.0])[0] == 0
    assert O.nearest_centre([1.0], [0.0], [2.0, 0.0], [0.0, 0.0])[0] == 0


def test_lloyd_objective_never_increases_and_reaches_a_fixed_point():
    rng = np.random.default_rng(1)
    q, p, w = _markers(rng, 3000, 8.0)
    init = rng.choice(q.size, 40, replace=False)
    prev = math.inf
    for it in range(0, 16):
        cq, cp, a = O.lloyd(q, p, w, init, it)
        obj = O.kmeans_objective(q, p, w, cq, cp, a)
        assert obj <= prev * (1 + 1e-12)
        prev = obj
    cq, cp, a = O.lloyd(q, p, w, init, 200)
    cq2, cp2, a2 = O.lloyd(q, p, w, init, 201)
    assert np.array_equal(a, a2) and np.array_equal(cq, cq2) and np.array_equal(cp, cp2)


def test_separated_blobs_are_recovered_exactly():
    rng = np.random.default_rng(2)
    centres = np.array([[1.0, -2.0], [4.0, 0.5], [7.5, 2.0], [2.5, 2.5], [6.0, -1.5]])
    lab = np.repeat(np.arange(5), 60)
    q = centres[lab, 0] + 0.05 * rng.standard_normal(lab.size)
    p = centres[lab, 1] + 0.05 * rng.standard_normal(lab.size)
    w = rng.uniform(0.5, 1.5, lab.size)
    perm = rng.permutation(lab.size)
    q, p, w, lab = q[perm], p[perm], w[perm], lab[perm]
    init = np.array([np.nonzero(lab == c)[0][0] for c in range(5)])
    cq, cp, a = O.lloyd(q, p, w, init, 10)
    assert np.array_equal(a, lab)
    for c in range(5):
        m = lab == c
        assert abs(cq[c] - np.sum(w[m] * q[m]) / np.sum(w[m])) < 1e-13
        assert abs(cp[c] - np.sum(w[m] * p[m]) / np.sum(w[m])) < 1e-13


def test_moments_reproduce_charge_momentum_and_mean_velocity():
    """psi*_a = sum of weights; P_a + q*_a / psi*_a = the cluster's mean velocity, so the
    total momentum sum(psi* P + q*) equals the markers' sum(psi P) (eq. moment-def)."""
    rng = np.random.default_rng(3)
    L = 6.0
    q, p, w = _markers(rng, 4000, L)
    init = rng.choice(q.size, 300, replace=False)
    dec, a = O.cluster_markers(q, p, w, init, 8, L)
    assert abs(dec["psi"].sum() - w.sum()) < 1e-12 * w.sum()
    mom_markers = np.sum(w * p)
    mom_dec = np.sum(dec["psi"] * dec["P"] + dec["qs"])
    assert abs(mom_dec - mom_markers) < 1e-11 * np.sum(np.abs(w * p))
    for j, c in enumerate(dec["cluster"]):
        m = a == c
        zp = np.sum(w[m] * p[m]) / np.sum(w[m])
        assert abs(dec["P"][j] + dec["qs"][j] / dec["psi"][j] - zp) < 1e-12 * (1 + abs(zp))
        # the centre is the member nearest the weighted mean
        zq = np.sum(w[m] * q[m]) / np.sum(w[m])
        d2 = (q[m] - zq) ** 2 + (p[m] - zp) ** 2
        assert dec["Q"][j] == q[m][np.argmin(d2)] and dec["P"][j] == p[m][np.argmin(d2)]


def test_position_moment_to_third_order_in_cluster_width():
    """With the periodic c, Q_a - p*_a / psi*_a is the weighted mean position up to the
    sine's cubic term, (2 pi / L)^2 / 6 times the third moment about Q_a: scaling the
    cluster's positions by 1/2 (same centre member) divides the error by 8."""
    rng = np.random.default_rng(4)
    L = 10.0
    u = rng.uniform(-1, 1, 50)
    p = rng.uniform(-1, 1, 50)
    w = rng.uniform(0.5, 1.5, 50)
    errs = []
    for width in (0.1, 0.05, 0.025):
        q = 3.0 + width * u
        dec = O.cluster_moments(q, p, w, np.zeros(50, dtype=int), 1, L)
        zq = np.sum(w * q) / np.sum(w)
        d = dec["Q"][0] - q
        predicted = (2 * math.pi / L) ** 2 / 6 * np.sum(w * d ** 3) / np.sum(w)
        err = dec["Q"][0] - dec["ps"][0] / dec["psi"][0] - zq
        assert abs(err - predicted) < 0.05 * abs(predicted) + 1e-15, (width, err, predicted)
        errs.append(abs(err))
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0, errs


def test_spatial_moment_is_periodic_across_zero():
    """A cluster straddling q = 0 gets the small displacement of its members through the
    periodic boundary, not the domain length."""
    L = 4.0
    q = np.array([0.05, L - 0.05, 0.02])
    p = np.zeros(3)
    w = np.ones(3)
    dec = O.cluster_moments(q, p, w, np.zeros(3, dtype=int), 1, L)
    # unwrapped positions 0.05, -0.05, 0.02 around the centre chosen among them
    unwrapped = np.array([0.05, -0.05, 0.02])
    qa = dec["Q"][0] if dec["Q"][0] < L / 2 else dec["Q"][0] - L
    approx = np.sum(w * (qa - unwrapped))
    assert abs(dec["ps"][0] - approx) < 1e-3      # the sine's cubic term: ~4e-4 here
    assert abs(dec["ps"][0]) < 0.2


def test_decorated_load_beats_monopoles_at_the_centres():
    """For clusters much narrower than an element, the P1 load vector of the decorated
    particles is much closer to that of the markers than the load of monopoles of the same
    weights at the same centres: the dipole moves each cluster's charge to its mean, exactly
    while the cluster sits inside one element (P1 hats are linear there).  For clusters as
    wide as an element the gain goes away."""
    rng = np.random.default_rng(5)
    L, m = 2 * math.pi, 8000
    x = rng.uniform(0, L, m)
    v = rng.standard_normal(m)
    w = (1 + 0.3 * np.cos(x)) * L / m
    init = rng.choice(m, 4000, replace=False)        # clusters about 0.1 wide
    dec, _ = O.cluster_markers(x, v, w, init, 6, L)
    ratios = []
    for ng in (4, 8, 16):
        b_mark = O.deposit(x, np.zeros(m), w, L, ng)
        b_dec = O.deposit(dec["Q"], dec["ps"], dec["psi"], L, ng)
        b_mono = O.deposit(dec["Q"], np.zeros_like(dec["Q"]), dec["psi"], L, ng)
        ratios.append(np.linalg.norm(b_dec - b_mark) / np.linalg.norm(b_mono - b_mark))
    assert ratios[0] < 0.1 and ratios[0] < ratios[1] < ratios[2] < 0.5, ratios


# ---------------------------------------------------------------- mini-batch k-means

def test_minibatch_one_full_batch_is_one_lloyd_iteration():
    """From zero absorbed weight, a batch of every marker once moves each centre to the
    weighted mean of its markers: exactly Lloyd's update."""
    rng = np.random.default_rng(6)
    q, p, w = _markers(rng, 3000, 7.0)
    init = rng.choice(q.size, 60, replace=False)
    cq, cp, v = O.minibatch(q, p, w, init, [np.arange(q.size)])
    lq, lp, _ = O.lloyd(q, p, w, init, 1)
    assert np.array_equal(cq, lq) and np.array_equal(cp, lp)
    a = O.nearest_centre(q, p, q[init], p[init])
    assert np.allclose(v, np.bincount(a, weights=w, minlength=60), rtol=1e-15, atol=0)


def test_minibatch_centres_are_running_weighted_means():
    """After any sequence of batches (repeated indices included) every centre that received
    members equals the weighted mean of all the batch members it received, at the time
    they were assigned; the others keep their starting markers; the absorbed weights add up
    to the weight of every drawn index."""
    rng = np.random.default_rng(7)
    q, p, w = _markers(rng, 2000, 5.0)
    k = 40
    init = rng.choice(q.size, k, replace=False)
    batches = [rng.integers(0, q.size, 300) for _ in range(12)]
    cq, cp, v, seen = O.minibatch(q, p, w, init, batches, record=True)
    allb = np.concatenate(batches)
    alla = np.concatenate(seen)
    assert abs(v.sum() - w[allb].sum()) < 1e-12 * w[allb].sum()
    for c in range(k):
        m = alla == c
        if not m.any():
            assert cq[c] == q[init[c]] and cp[c] == p[init[c]] and v[c] == 0.0
            continue
        W = w[allb][m].sum()
        assert abs(cq[c] - np.sum(w[allb][m] * q[allb][m]) / W) < 1e-12 * 5.0
        assert abs(cp[c] - np.sum(w[allb][m] * p[allb][m]) / W) < 1e-12 * 3.0
        assert abs(v[c] - W) < 1e-12 * W
    # the final assignment of Algorithm 1 takes every marker to its nearest final centre
    # (brute force over the centres for a sample of markers)
    _, a, v2 = O.cluster_markers_minibatch(q, p, w, init, batches, 5.0)
    assert np.array_equal(v2, v)
    for i in rng.choice(q.size, 60, replace=False):
        d2 = [(q[i] - cq[c]) ** 2 + (p[i] - cp[c]) ** 2 for c in range(k)]
        assert a[i] == int(np.argmin(d2))


def test_minibatch_recovers_separated_blobs():
    rng = np.random.default_rng(8)
    centres = np.array([[1.0, -2.0], [4.0, 0.5], [7.5, 2.0], [2.5, 2.5], [6.0, -1.5]])
    lab = np.repeat(np.arange(5), 80)
    q = centres[lab, 0] + 0.05 * rng.standard_normal(lab.size)
    p = centres[lab, 1] + 0.05 * rng.standard_normal(lab.size)
    w = rng.uniform(0.5, 1.5, lab.size)
    perm = rng.permutation(lab.size)
    q, p, w, lab = q[perm], p[perm], w[perm], lab[perm]
    init = np.array([np.nonzero(lab == c)[0][0] for c in range(5)])
    batches = [rng.integers(0, lab.size, 40) for _ in range(20)]
    dec, a, _ = O.cluster_markers_minibatch(q, p, w, init, batches, 10.0)
    assert np.array_equal(a, lab)
    assert np.array_equal(dec["psi"], np.bincount(lab, weights=w))


def test_minibatch_objective_is_close_to_lloyds():
    """The paper allows mini-batch k-means for large runs on the ground that the results are
    nearly the same: on Landau markers (40 per cluster) 30 batches of a fifth of the markers
    land within 15% of the within-cluster sum of squares of 10 Lloyd iterations."""
    import workloads as W
    w_ = W.landau_linear()
    w_.params["alpha"] = 0.3
    w_.L = 4 * math.pi
    w_.params["k"] = 2 * math.pi / w_.L
    st = W.random_markers(w_, 20000, seed=3)
    q, p, w = st["Q"], st["P"], st["psi"]
    rng = np.random.default_rng(0)
    init = rng.choice(q.size, 500, replace=False)
    cq, cp, a = O.lloyd(q, p, w, init, 10)
    lloyd_obj = O.kmeans_objective(q, p, w, cq, cp, a)
    batches = [rng.integers(0, q.size, 4000) for _ in range(30)]
    mq, mp, _ = O.minibatch(q, p, w, init, batches)
    mb_obj = O.kmeans_objective(q, p, w, mq, mp, O.nearest_centre(q, p, mq, mp))
    start_obj = O.kmeans_objective(q, p, w, q[init], p[init], O.nearest_centre(q, p, q[init], p[init]))
    assert mb_obj < 1.15 * lloyd_obj and mb_obj < 0.7 * start_obj, (mb_obj, lloyd_obj, start_obj)
