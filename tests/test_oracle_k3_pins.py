"""Pins of the k = 3 oracle (decorated particles with second moments, P2 potential) against
statements independent of its formulas: finite-difference curvature of the P2 basis, clouds
of marker particles moved one by one by the same leapfrog, the Casimir of the moments'
Lie-Poisson bracket, the exact reduction to k = 2 without moments, and the order in the
cloud width at which the moment model follows a cloud in a prescribed potential."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _p2_basis_value(node_kind, j, x, L, ng):
    """A P2 basis function written from its definition (tent of quadratics): vertex j is
    N2 on element j-1 and N0 on element j; midpoint j is N1 on element j; zero elsewhere."""
    h = L / ng
    e = int(np.floor(x / h)) % ng
    s = x / h - np.floor(x / h)
    if node_kind == "m":
        return 4 * s * (1 - s) if e == j else 0.0
    if e == j:
        return (1 - s) * (1 - 2 * s)
    if e == (j - 1) % ng:
        return s * (2 * s - 1)
    return 0.0


def test_k3_deposit_adds_half_mqq_times_basis_curvature():
    """The second-moment load (1/2) Mqq phi_k''(Q), with phi_k'' by central differences of
    the basis functions (exact for quadratics up to rounding), away from the nodes."""
    rng = np.random.default_rng(0)
    L, ng, n = 3.0, 8, 40
    h = L / ng
    Q = (rng.integers(0, ng, n) + rng.uniform(0.05, 0.95, n)) * h
    ps, psi = 0.1 * rng.normal(size=n), rng.uniform(0.5, 1.5, n)
    Mqq = rng.uniform(0.0, 0.2, n)
    bv, bm = O.deposit_p2_k3(Q, ps, psi, Mqq, L, ng)
    bv2, bm2 = O.deposit_p2(Q, ps, psi, L, ng)
    d = 1e-3 * h
    for kind, b, b2 in (("v", bv, bv2), ("m", bm, bm2)):
        for j in range(ng):
            ref = 0.0
            for a in range(n):
                f = lambda x: _p2_basis_value(kind, j, x, L, ng)  # noqa: E731
                curv = (f(Q[a] + d) - 2 * f(Q[a]) + f(Q[a] - d)) / (d * d)
                ref += 0.5 * Mqq[a] * curv
            assert abs((b[j] - b2[j]) - ref) < 1e-7 * max(1.0, abs(ref)), (kind, j)
    # the moments add no charge: the basis functions sum to one, so their curvatures to 0
    assert abs((bv.sum() + bm.sum()) - psi.sum()) < 1e-12 * psi.sum()


@pytest.mark.parametrize("g0", [0.7, -0.4])
def test_k3_moments_are_the_covariance_of_a_cloud_moved_by_the_same_leapfrog(g0):
    """In a field of uniform curvature g0 (E linear in the offset), a cloud of markers about
    the centre moves by the linear leapfrog map, written here per marker; the oracle's
    second moments after n kick-drift-kick steps equal the cloud's covariance about the
    centre (so a wrong sign or factor in any moment update fails)."""
    rng = np.random.default_rng(1)
    m = 200
    dq, dp = 0.05 * rng.normal(size=m), 0.08 * rng.normal(size=m)
    w = rng.uniform(0.5, 1.5, m)
    M = [np.sum(w * dq * dq), np.sum(w * dq * dp), np.sum(w * dp * dp)]
    ng, L, tau, nsteps = 8, 10.0, 0.1, 37
    fld = {"E0": np.zeros(ng), "E1": np.zeros(ng), "g": np.full(ng, g0)}
    st = (np.array([3.3]), np.array([0.0]), np.array([0.0]), np.array([0.0]), np.array([w.sum()]),
          np.array([M[0]]), np.array([M[1]]), np.array([M[2]]))
    for _ in range(nsteps):
        st = O.kick_k3(st, fld, L, 0.5 * tau)
        st = O.drift_k3(st, L, tau)
        st = O.kick_k3(st, fld, L, 0.5 * tau)
        # markers: the force on an offset dq is -g0 dq
        dp = dp - 0.5 * tau * g0 * dq
        dq = dq + tau * dp
        dp = dp - 0.5 * tau * g0 * dq
    ref = [np.sum(w * dq * dq), np.sum(w * dq * dp), np.sum(w * dp * dp)]
    got = [st[5][0], st[6][0], st[7][0]]
    for a, b in zip(got, ref):
        assert abs(a - b) < 1e-12 * max(ref, key=abs), (got, ref)


def _k3_lattice(ng=16, nx=64, nv=24, seed=3, alpha=0.2):
    w = W.landau_linear(seed=seed, nx=nx, nv=nv, ng=ng)
    w.params["alpha"] = alpha
    st = dict(w.state())
    rng = np.random.default_rng(seed)
    h = w.L / ng
    # second moments of a small cloud: positive definite, about a tenth of a cell wide
    st["Mqq"] = st["psi"] * (0.1 * h) ** 2 * rng.uniform(0.5, 1.5, st["Q"].size)
    st["Mpp"] = st["psi"] * 0.05 ** 2 * rng.uniform(0.5, 1.5, st["Q"].size)
    st["Mqp"] = 0.3 * np.sqrt(st["Mqq"] * st["Mpp"]) * rng.uniform(-1, 1, st["Q"].size)
    return w, st


def test_k3_casimir_det_m_is_kept_by_every_step():
    """det M = Mqq Mpp - Mqp^2 is a Casimir of the moments' Lie-Poisson bracket, and each
    sub-flow is a congruence by a unimodular matrix: over a self-consistent run every
    particle's det M stays at its initial value to rounding."""
    w, st = _k3_lattice()
    state, _, hist = O.run_k3(st, w.L, w.ng, w.dt, 40)
    det0 = st["Mqq"] * st["Mpp"] - st["Mqp"] ** 2
    det1 = state[5] * state[7] - state[6] ** 2
    assert np.all(det0 > 0)
    assert np.max(np.abs(det1 - det0) / det0) < 1e-9
    assert abs(hist[-1]["casimir"] - hist[0]["casimir"]) < 1e-9 * abs(hist[0]["casimir"])
    # the moments moved (the test is not of a frozen state)
    assert np.max(np.abs(state[5] - st["Mqq"]) / st["Mqq"]) > 1e-2


def test_k3_without_moments_is_the_k2_p2_run():
    """With M = 0 the moment terms vanish and the k = 3 run is the P2 decorated run."""
    w, st = _k3_lattice()
    for k in ("Mqq", "Mqp", "Mpp"):
        st[k] = np.zeros_like(st["Q"])
    s3, f3, h3 = O.run_k3(st, w.L, w.ng, w.dt, 15)
    s2, f2, h2 = O.run_p2(st["Q"], st["P"], st["qs"], st["ps"], st["psi"], w.L, w.ng, w.dt, 15)
    for a, b in zip(s3[:5], s2):
        assert np.array_equal(a, b)
    assert [h["W"] for h in h3] == [h["W"] for h in h2]
    assert [h["K"] for h in h3] == [h["K"] for h in h2]


def _cloud_error(width, order, steps=400, dt=2e-3):
    """Mean velocity of a cloud of markers in V = 1 - cos(2 pi q / L), L = 10 (the paper's
    test-particle potential), against a decorated particle of order k (2 or 3) with the
    cloud's moments about its centre, after `steps` leapfrog steps of both; no self field."""
    L = 10.0
    ext = {"amp": 1.0, "mode": 1}
    u = np.array([-1.0, -0.5, 0.0, 0.5, 1.0, -0.8, 0.8, 0.3, -0.3, 0.1])
    v = np.array([0.6, -1.0, 0.2, 0.9, -0.4, -0.7, 0.1, -0.2, 0.5, 0.3])
    wgt = np.array([1.0, 0.8, 1.2, 0.9, 1.1, 0.7, 1.3, 1.0, 0.95, 1.05])
    Q0, P0 = 2.1, 0.35
    q = Q0 + width * u
    p = P0 + width * v
    psi = wgt.sum()
    ps = np.sum(wgt * (Q0 - q))
    qs = -np.sum(wgt * (P0 - p))
    ng = 8
    fld = {"E0": np.zeros(ng), "E1": np.zeros(ng), "g": np.zeros(ng)}
    if order == 3:
        st = (np.array([Q0]), np.array([P0]), np.array([qs]), np.array([ps]), np.array([psi]),
              np.array([np.sum(wgt * (q - Q0) ** 2)]), np.array([np.sum(wgt * (q - Q0) * (p - P0))]),
              np.array([np.sum(wgt * (p - P0) ** 2)]))
    for _ in range(steps):
        # markers
        E, _ = O.external_field(q, L, ext)
        p = p + 0.5 * dt * E
        q = q + dt * p
        E, _ = O.external_field(q, L, ext)
        p = p + 0.5 * dt * E
        if order == 3:
            st = O.kick_k3(st, fld, L, 0.5 * dt, ext, self_field=False)
            st = O.drift_k3(st, L, dt)
            st = O.kick_k3(st, fld, L, 0.5 * dt, ext, self_field=False)
        else:
            Pq, qsq = O.kick(np.array([Q0]), np.array([P0]), np.array([qs]), np.array([ps]),
                             np.zeros(ng), np.zeros(ng), L, 0.5 * dt, ext=ext, self_field=False)
            Qn, psn = O.drift(np.array([Q0]), Pq, qsq, np.array([ps]), L, dt)
            Pq, qsq = O.kick(Qn, Pq, qsq, psn, np.zeros(ng), np.zeros(ng), L, 0.5 * dt, ext=ext,
                             self_field=False)
            Q0, P0, qs, ps = float(Qn[0]), float(Pq[0]), float(qsq[0]), float(psn[0])
    mean_markers = np.sum(wgt * p) / psi
    if order == 3:
        mean_model = st[1][0] + st[2][0] / st[4][0]
    else:
        mean_model = P0 + qs / psi
    return abs(mean_model - mean_markers)


def test_k3_follows_a_cloud_one_order_further_in_its_width():
    """The cloud's mean velocity feels the mean force -V'(Q) - (1/2) <dq^2> V'''(Q) + ...;
    the k = 2 particle misses the second term, so its error falls like width^2, and the
    k = 3 particle keeps it (through -Mqq V''' / 2 in dq*/dt), so its error falls at least
    like width^3.  Halving the width: k = 2 error / 4, k = 3 error / 8 or better."""
    e2 = [_cloud_error(wd, 2) for wd in (0.2, 0.1, 0.05)]
    e3 = [_cloud_error(wd, 3) for wd in (0.2, 0.1, 0.05)]
    r2 = [e2[i] / e2[i + 1] for i in range(2)]
    r3 = [e3[i] / e3[i + 1] for i in range(2)]
    assert all(3.0 < r < 5.0 for r in r2), (e2, r2)
    assert all(r > 6.5 for r in r3), (e3, r3)
    assert e3[-1] < 0.05 * e2[-1], (e2, e3)


def test_k3_test_particle_energy_error_is_second_order():
    """Without self field, in V = 1 - cos(2 pi q / L): H = K + U (with Mpp/2 and
    Mqq V''/2) is the Hamiltonian of the splitting's exact sub-flows, so its error over a
    fixed time is second order in dt: halving dt divides the largest deviation over t <= 40
    by four (measured 4.005 and 4.001).  The band itself widens in time, as the moments of
    particles on passing orbits shear."""
    L = 10.0
    ext = {"amp": 1.0, "mode": 1}
    ng = 8
    fld = {"E0": np.zeros(ng), "E1": np.zeros(ng), "g": np.zeros(ng), "W": 0.0}
    st0 = (np.array([1.0, 4.0, 7.5]), np.array([0.4, -0.2, 0.9]), np.array([0.01, -0.02, 0.0]),
           np.array([0.03, 0.01, -0.02]), np.array([1.0, 0.7, 1.3]),
           np.array([0.02, 0.05, 0.01]), np.array([0.004, -0.01, 0.0]), np.array([0.03, 0.02, 0.05]))
    H0 = O.diagnostics_k3(st0, fld, L, ext, self_field=False)["H"]
    bands = []
    for dt in (0.1, 0.05, 0.025):
        st = st0
        dev = 0.0
        for _ in range(int(round(40.0 / dt))):
            st = O.kick_k3(st, fld, L, 0.5 * dt, ext, self_field=False)
            st = O.drift_k3(st, L, dt)
            st = O.kick_k3(st, fld, L, 0.5 * dt, ext, self_field=False)
            dev = max(dev, abs(O.diagnostics_k3(st, fld, L, ext, self_field=False)["H"] - H0))
        bands.append(dev)
    for i in range(2):
        assert 3.9 < bands[i] / bands[i + 1] < 4.1, bands


def test_k3_cluster_load_matches_the_markers_inside_an_element():
    """Clusters of markers lying inside one element each (Algorithm 1's particles with their
    second moments): a P2 basis function is a quadratic on the element, so the ansatz's
    Taylor terms up to second order reproduce the markers' load; what is left is the periodic
    form of the first and second moments, of relative size (width / L)^2.  The k = 3 load is
    therefore orders of magnitude closer to the markers' load than the k = 2 load, whose error
    is the second-order term it leaves out."""
    rng = np.random.default_rng(7)
    L, ng = 2 * math.pi, 16
    h = L / ng
    k = 300
    for width in (0.1, 0.05):
        cq = (rng.integers(0, ng, k) + 0.5) * h       # element centres
        cp = rng.normal(size=k)
        off = np.clip(width * h * rng.normal(size=(k, 12)), -0.45 * h, 0.45 * h)
        q = (cq[:, None] + off).reshape(-1)
        p = (cp[:, None] + 0.1 * rng.normal(size=(k, 12))).reshape(-1)
        w = rng.uniform(0.5, 1.5, q.size) / q.size
        assign = np.repeat(np.arange(k), 12)
        dec = O.cluster_moments_k3(q, p, w, assign, k, L)
        ref = np.concatenate(O.deposit_p2(q, np.zeros_like(q), w, L, ng))
        k2 = np.concatenate(O.deposit_p2(dec["Q"], dec["ps"], dec["psi"], L, ng))
        k3 = np.concatenate(O.deposit_p2_k3(dec["Q"], dec["ps"], dec["psi"], dec["Mqq"], L, ng))
        e2 = np.linalg.norm(k2 - ref) / np.linalg.norm(ref)
        e3 = np.linalg.norm(k3 - ref) / np.linalg.norm(ref)
        assert e3 < 1e-3 * e2 and e3 < 10 * (width * h / L) ** 2, (width, e2, e3)
