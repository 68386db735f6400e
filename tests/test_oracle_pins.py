"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own formula: each compares the oracle with an
independent statement (brute-force hat-function sums, dense assembled stiffness matrices,
the paper's closed-form single-source solutions, exact sub-flow solutions, the Vlasov
dispersion relation) chosen so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

import physics_helpers as PH


# ---------------------------------------------------------------- brute-force helpers
def _wrap_dist(x, xj, L):
    """x - xj reduced to (-L/2, L/2]."""
    r = (x - xj) % L
    return np.where(r > L / 2, r - L, r)


def _hat(x, j, L, ng):
    """Periodic P1 hat phi_j(x) written from its definition (tent of half-width h)."""
    h = L / ng
    r = _wrap_dist(x, j * h, L)
    return np.maximum(0.0, 1.0 - np.abs(r) / h)


def _hat_slope(x, j, L, ng):
    """phi_j'(x): +1/h on the rising side, -1/h on the falling side, 0 outside."""
    h = L / ng
    r = _wrap_dist(x, j * h, L)
    inside = np.abs(r) < h
    return np.where(inside, np.where(r < 0, 1.0 / h, -1.0 / h), 0.0)


def _stiffness(L, ng):
    """Periodic P1 stiffness matrix assembled element by element (eq. lin-sys):
    each element [q_e, q_{e+1}] adds (1/h) [[1, -1], [-1, 1]] on nodes (e, e+1 mod Ng)."""
    h = L / ng
    A = np.zeros((ng, ng))
    for e in range(ng):
        a, b = e, (e + 1) % ng
        A[a, a] += 1 / h
        A[b, b] += 1 / h
        A[a, b] -= 1 / h
        A[b, a] -= 1 / h
    return A


def _rand_particles(rng, n, L, ng, avoid_nodes=True):
    Q = rng.uniform(0, L, n)
    if avoid_nodes:
        h = L / ng
        s = (Q / h) % 1.0
        Q = np.where((s < 1e-6) | (s > 1 - 1e-6), Q + 0.37 * h, Q) % L
    return Q, rng.normal(size=n), rng.normal(size=n) * 0.1, rng.normal(size=n) * 0.05, rng.uniform(0.1, 1.0, n)


# ---------------------------------------------------------------- cell index (C1 rules)
def test_cell_index_half_open_and_clamp():
    L, ng = 2.0, 8
    h = L / ng
    nodes = np.arange(ng) * h
    i, s = O.cell_index(nodes, L, ng)
    assert np.array_equal(i, np.arange(ng))           # on a node -> element to the right
    assert np.all(s == 0.0)
    i, s = O.cell_index(np.array([np.nextafter(L, 0.0)]), L, ng)
    assert i[0] == ng - 1 and 0.0 <= s[0] <= 1.0
    i, s = O.cell_index(np.array([np.float32(L * 0.999999)]).astype(np.float32), L, ng)
    assert i[0] == ng - 1


# ---------------------------------------------------------------- deposit
@pytest.mark.parametrize("ng,n,seed", [(4, 7, 0), (8, 40, 1), (16, 64, 2)])
def test_deposit_brute_force(ng, n, seed):
    """T-D1: eq. rhs-assembly evaluated hat by hat, particle by particle."""
    rng = np.random.default_rng(seed)
    L = 3.7
    Q, _, _, ps, psi = _rand_particles(rng, n, L, ng)
    b_ref = np.zeros(ng)
    for j in range(ng):
        for a in range(n):
            b_ref[j] += psi[a] * _hat(Q[a], j, L, ng) - ps[a] * _hat_slope(Q[a], j, L, ng)
    b = O.deposit(Q, ps, psi, L, ng)
    assert np.max(np.abs(b - b_ref)) <= 1e-13 * max(1.0, np.sum(np.abs(psi)) + np.sum(np.abs(ps)) * ng / L)


def test_deposit_charge_and_linearity():
    """T-D2: the hats sum to one and their slopes to zero, so sum_j b_j = sum_a psi*_a;
    b is linear in (psi*, p*)."""
    rng = np.random.default_rng(3)
    L, ng = 5.0, 32
    Q, _, _, ps, psi = _rand_particles(rng, 500, L, ng)
    b = O.deposit(Q, ps, psi, L, ng)
    assert abs(b.sum() - psi.sum()) <= 1e-13 * psi.sum()
    b1 = O.deposit(Q, ps, np.zeros_like(psi), L, ng)
    b2 = O.deposit(Q, np.zeros_like(ps), psi, L, ng)
    assert np.allclose(b, b1 + b2, rtol=0, atol=1e-13)
    assert abs(b1.sum()) < 1e-12
    b3 = O.deposit(Q, 2.5 * ps, -0.5 * psi, L, ng)
    assert np.allclose(b3, 2.5 * b1 - 0.5 * b2, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- Poisson solve
@pytest.mark.parametrize("ng", [8, 16, 64])
def test_solve_matches_dense_pseudo_inverse(ng):
    """T-S1: A Phi = b~ with 1^T Phi = 0, against the pseudo-inverse of the assembled A."""
    rng = np.random.default_rng(ng)
    L = 2 * math.pi * 1.3
    bt = O.neutralize(rng.normal(size=ng))
    A = _stiffness(L, ng)
    ref = np.linalg.pinv(A) @ bt
    Phi = O.poisson_solve(bt, L)
    assert np.max(np.abs(Phi - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert abs(Phi.sum()) < 1e-12
    assert np.allclose(A @ Phi, bt, atol=1e-11)
    # the stiffness kernel: constant vectors
    assert np.allclose(A @ np.ones(ng), 0.0, atol=1e-12)


def test_solve_green_function_closed_form():
    """T-S2: A^+ = h G with G(d) = (Ng^2 - 1)/(12 Ng) - d (Ng - d)/(2 Ng), d the circular
    node distance (derived for the periodic P1 stiffness); so E = -D G b~ is free of h."""
    for ng in (8, 33, 64):
        for L in (1.0, 7.5):
            h = L / ng
            d = np.abs(np.arange(ng)[:, None] - np.arange(ng)[None, :])
            d = np.minimum(d, ng - d)
            G = (ng * ng - 1) / (12.0 * ng) - d * (ng - d) / (2.0 * ng)
            A = _stiffness(L, ng)
            assert np.allclose(np.linalg.pinv(A), h * G, atol=1e-12 * h * ng)
            rng = np.random.default_rng(ng)
            bt = O.neutralize(rng.normal(size=ng))
            assert np.allclose(O.poisson_solve(bt, L), h * G @ bt, atol=1e-12 * h * ng)


@pytest.mark.parametrize("Qfrac", [0.123, 0.5, 0.999, 0.0])
def test_single_monopole_matches_theorem1(Qfrac):
    """T-S3: Theorem 1 (eq. solution) for a monopole.  In 1D the P1 Galerkin solution is
    exact at the nodes up to the gauge, so Phi_j = phi_M(q_j) - mean_k phi_M(q_k)."""
    L, ng = 6.0, 24
    h = L / ng
    Q = (7 + Qfrac) * h
    psi = 0.8
    b = O.deposit(np.array([Q]), np.array([0.0]), np.array([psi]), L, ng)
    Phi = O.poisson_solve(O.neutralize(b), L)
    q = np.arange(ng) * h
    r = (q - Q) % L
    r = np.where(r > L / 2, r - L, r)
    phiM = psi * (r * r / (2 * L) - np.abs(r) / 2 + L / 12)
    assert np.allclose(Phi, phiM - phiM.mean(), atol=1e-13)
    # the continuum solution itself has zero mean (its L/12 constant)
    xx = np.linspace(0, L, 200001)[:-1]
    rr = (xx - Q) % L
    rr = np.where(rr > L / 2, rr - L, rr)
    assert abs(np.mean(psi * (rr * rr / (2 * L) - np.abs(rr) / 2 + L / 12))) < 1e-6


@pytest.mark.parametrize("Qfrac", [0.1, 0.5, 0.93])
def test_single_dipole_matches_explicit_discrete_solution(Qfrac):
    """T-S4: the paper's explicit P1 dipole solution (proof of Theorem 2): slope p*/L off
    the element e_Q, end values +-p*(L - h)/(2L) on e_Q, independent of Q inside e_Q.
    This fixes the sign of the dipole load and the solve together."""
    L, ng = 5.0, 20
    h = L / ng
    iQ = 13
    Q = (iQ + Qfrac) * h
    ps = 0.37
    b = O.deposit(np.array([Q]), np.array([ps]), np.array([0.0]), L, ng)
    Phi = O.poisson_solve(O.neutralize(b), L)
    ref = np.empty(ng)
    for m in range(ng):
        ref[(iQ + 1 + m) % ng] = ps * (-(L - h) / (2 * L) + m * h / L)
    assert np.allclose(Phi, ref, atol=1e-14)
    assert abs(Phi[iQ] - ps * (L - h) / (2 * L)) < 1e-14
    # C0 = p*(b - a)/(2L): the constant gap between continuum and discrete solutions
    a_, b_ = Q - iQ * h, (iQ + 1) * h - Q
    q = np.arange(ng) * h
    r = (q - Q) % L
    r = np.where(r > L / 2, r - L, r)
    phiD = ps * (r / L - 0.5 * np.sign(r))
    off = np.array([j for j in range(ng) if j not in (iQ, (iQ + 1) % ng)])
    gap = phiD[off] - Phi[off]
    assert np.allclose(gap, ps * (b_ - a_) / (2 * L), atol=1e-13)


def test_field_energy_identities():
    """T-F1: (1/2) Phi^T A Phi = (1/2) b~^T Phi = (1/2) sum_e h E_e^2, E_amp = sqrt(2W/L)."""
    rng = np.random.default_rng(7)
    L, ng = 4.0, 32
    Q, P, qs, ps, psi = _rand_particles(rng, 300, L, ng)
    f = O.solve_field(Q, ps, psi, L, ng)
    A = _stiffness(L, ng)
    W1 = 0.5 * f["Phi"] @ A @ f["Phi"]
    W2 = 0.5 * f["bt"] @ f["Phi"]
    assert abs(W1 - f["W"]) < 1e-12 * abs(W1) and abs(W2 - f["W"]) < 1e-12 * abs(W1)
    d = O.diagnostics(P, qs, psi, f, L)
    assert abs(d["e_amp"] - math.sqrt(np.sum(f["E"] ** 2) * (L / ng) / L)) < 1e-14


def test_gather_is_adjoint_of_deposit():
    """T-G1: W is quadratic in (psi*, p*), so central differences are exact up to
    rounding: dW/dp*_a = E[i_a] = -phi_h'(Q_a), dW/dpsi*_a = phi_h(Q_a)."""
    rng = np.random.default_rng(11)
    L, ng = 3.0, 16
    Q, P, qs, ps, psi = _rand_particles(rng, 12, L, ng)
    f = O.solve_field(Q, ps, psi, L, ng)
    i, s = O.cell_index(Q, L, ng)
    eps = 1e-3
    for a in range(len(Q)):
        dp = np.zeros_like(ps)
        dp[a] = eps
        Wp = O.solve_field(Q, ps + dp, psi, L, ng)["W"]
        Wm = O.solve_field(Q, ps - dp, psi, L, ng)["W"]
        assert abs((Wp - Wm) / (2 * eps) - f["E"][i[a]]) < 1e-9
        Wp = O.solve_field(Q, ps, psi + dp, L, ng)["W"]
        Wm = O.solve_field(Q, ps, psi - dp, L, ng)["W"]
        phi_at = (1 - s[a]) * f["Phi"][i[a]] + s[a] * f["Phi"][(i[a] + 1) % ng]
        assert abs((Wp - Wm) / (2 * eps) - phi_at) < 1e-9


def test_projected_curvature_identity():
    """T-G2: lumped projection gives g_e = -(b~_e + b~_{e+1}) / (2h) (stiffness identity
    E_{e+1} - E_{e-1} = b~_e + b~_{e+1})."""
    rng = np.random.default_rng(5)
    L, ng = 7.0, 64
    Q, _, _, ps, psi = _rand_particles(rng, 800, L, ng)
    f = O.solve_field(Q, ps, psi, L, ng)
    h = L / ng
    ref = -(f["bt"] + np.roll(f["bt"], -1)) / (2 * h)
    assert np.allclose(f["g"], ref, atol=1e-12 * np.max(np.abs(ref)))
    # continuum limit: phi'' = -(rho - n0), so g tracks minus the nodal charge density
    assert np.corrcoef(f["g"], -f["bt"])[0, 1] > 0.5


# ---------------------------------------------------------------- push (exact sub-flows)
def test_uniform_field_free_fall_is_exact():
    """T-P1: in a uniform prescribed field E0 with zero curvature, KDK reproduces the
    closed form of eq. sw_prescribed_potential: Q = Q0 + P0 t + E0 t^2/2, P = P0 + E0 t,
    q* constant, p* = p*0 - q*0 t."""
    L, ng, dt, n = 1e6, 4, 0.01, 137
    E0 = 0.3
    E = np.full(ng, E0)
    g = np.zeros(ng)
    Q0, P0, q0, p0 = np.array([1000.0]), np.array([0.7]), np.array([0.2]), np.array([-0.4])
    Q, P, qs, ps = Q0.copy(), P0.copy(), q0.copy(), p0.copy()
    for _ in range(n):
        P, qs = O.kick(Q, P, qs, ps, E, g, L, dt / 2)
        Q, ps = O.drift(Q, P, qs, ps, L, dt)
        P, qs = O.kick(Q, P, qs, ps, E, g, L, dt / 2)
    t = n * dt
    assert abs(Q[0] - (Q0[0] + P0[0] * t + E0 * t * t / 2)) < 1e-9
    assert abs(P[0] - (P0[0] + E0 * t)) < 1e-12
    assert qs[0] == q0[0]
    assert abs(ps[0] - (p0[0] - q0[0] * t)) < 1e-12


@pytest.mark.parametrize("g0", [0.8, -0.3])
def test_uniform_curvature_shape_oscillator(g0):
    """T-P2: with uniform curvature g0 the shape pair obeys p*'' = -g0 p*; the KDK map is
    the Stormer-Verlet map whose n-th power has the closed form with cos(theta) =
    1 - dt^2 g0 / 2, and it converges to the exact cos/sin (cosh/sinh) at O(dt^2)."""
    L, ng = 100.0, 4
    E = np.zeros(ng)
    g = np.full(ng, g0)
    p0, q0 = 0.3, -0.2
    T = 2.0
    errs = []
    for nsteps in (100, 200, 400):
        dt = T / nsteps
        Q, P = np.array([10.0]), np.array([0.0])
        qs, ps = np.array([q0]), np.array([p0])
        for _ in range(nsteps):
            P, qs = O.kick(Q, P, qs, ps, E, g, L, dt / 2)
            Q, ps = O.drift(Q, P, qs, ps, L, dt)
            P, qs = O.kick(Q, P, qs, ps, E, g, L, dt / 2)
        # discrete closed form: M = K D K with K = [[1,0],[dt g/2, 1]] on (p*, q*) kick
        K = np.array([[1.0, 0.0], [dt * g0 / 2, 1.0]])
        D = np.array([[1.0, -dt], [0.0, 1.0]])
        M = K @ D @ K
        ref = np.linalg.matrix_power(M, nsteps) @ np.array([p0, q0])
        assert abs(ps[0] - ref[0]) < 1e-12 and abs(qs[0] - ref[1]) < 1e-12
        w = math.sqrt(abs(g0))
        if g0 > 0:
            pe = p0 * math.cos(w * T) - q0 / w * math.sin(w * T)
        else:
            pe = p0 * math.cosh(w * T) - q0 / w * math.sinh(w * T)
        errs.append(abs(ps[0] - pe))
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5      # second order


def test_reversibility():
    """T-P4: KDK is time-symmetric and the kick depends only on (Q, p*); flipping
    (P, q*) after n steps and running n more returns the initial state."""
    w = W.landau_linear(nx=32, nv=32, ng=32)
    st = w.state()
    state = tuple(st[k].copy() for k in ("Q", "P", "qs", "ps", "psi"))
    L, ng, dt = w.L, w.ng, w.dt
    fld = O.solve_field(state[0], state[3], state[4], L, ng)
    for _ in range(40):
        state, fld = O.step(state, fld, L, ng, dt)
    Q, P, qs, ps, psi = state
    state = (Q, -P, -qs, ps, psi)
    fld = O.solve_field(Q, ps, psi, L, ng)
    for _ in range(40):
        state, fld = O.step(state, fld, L, ng, dt)
    Q, P, qs, ps, psi = state
    dQ = np.abs(Q - st["Q"])
    dQ = np.minimum(dQ, L - dQ)
    assert dQ.max() < 1e-11
    assert np.abs(-P - st["P"]).max() < 1e-11
    assert np.abs(-qs - st["qs"]).max() < 1e-13
    assert np.abs(ps - st["ps"]).max() < 1e-13


def test_pic_special_case_and_casimir():
    """T-C2 and T-C1: with p* = q* = 0 the shape stays zero (plain P1 PIC); psi* never
    changes; the neutralised load sums to zero."""
    w = W.landau_linear(nx=32, nv=32, ng=32)
    st = w.state()
    zero = np.zeros_like(st["Q"])
    state, fld, hist = O.run(st["Q"], st["P"], zero, zero, st["psi"], w.L, w.ng, w.dt, 30)
    assert np.all(state[2] == 0.0) and np.all(state[3] == 0.0)
    assert np.array_equal(state[4], st["psi"])
    assert abs(fld["bt"].sum()) < 1e-13 * np.abs(fld["b"]).max() * w.ng
    assert all(abs(h["charge"] - hist[0]["charge"]) == 0.0 for h in hist)


def test_energy_behaviour_linear_landau():
    """T-C1: in the PIC special case (p* = q* = 0) H_h stays within a small bound with no
    trend.  With dipoles, the change of H_h over the run does not shrink with dt: it comes
    from the P1 dipole load -p* phi_j'(Q), which jumps between node pairs whenever a
    particle crosses a node (the semi-discrete H_h is discontinuous in Q), not from the
    time integrator.  Both facts are checked; the size is bounded for the linear run."""
    w = W.landau_linear()
    st = w.state()
    zero = np.zeros_like(st["Q"])
    _, _, hist = O.run(st["Q"], st["P"], zero, zero, st["psi"], w.L, w.ng, w.dt, 200)
    H = np.array([h["H"] for h in hist])
    assert np.max(np.abs(H - H[0])) / abs(H[0]) < 1e-3
    ends = []
    for dt, n in ((0.1, 200), (0.05, 400)):
        _, _, hist = O.run(st["Q"], st["P"], st["qs"], st["ps"], st["psi"], w.L, w.ng, dt, n)
        H = np.array([h["H"] for h in hist])
        assert np.max(np.abs(H - H[0])) / abs(H[0]) < 0.02
        ends.append(H[-1] - H[0])
    assert abs(ends[0] - ends[1]) < 0.1 * abs(ends[0])


# ---------------------------------------------------------------- sort
def test_sort_perm_is_stable_chunked_permutation():
    rng = np.random.default_rng(0)
    cells = rng.integers(0, 7, size=1000)
    for chunk in (1, 3, 64, 1000, 4096):
        perm = O.sort_perm(cells, chunk)
        assert np.array_equal(np.sort(perm), np.arange(1000))
        for c0 in range(0, 1000, chunk):
            seg = perm[c0:c0 + chunk]
            assert seg.min() >= c0 and seg.max() < c0 + chunk
            keys = cells[seg]
            assert np.all(np.diff(keys) >= 0)
            same = np.diff(keys) == 0
            assert np.all(np.diff(seg)[same] > 0)          # ties keep original order


# ---------------------------------------------------------------- physics: Landau rate
def test_landau_root_value():
    om = PH.landau_root(0.5)
    assert abs(om.real - 1.4157) < 1e-3 and abs(om.imag + 0.1534) < 1e-3


def test_linear_landau_rate_matches_dispersion_root():
    """T-L1: the damped mode-1 field of the linear Landau run (k = 0.5, alpha = 0.01,
    N = 4096, Ng = 64, dt = 0.1) matches the root of the dispersion relation:
    gamma = -0.1534 (mean over seeds within 0.01), omega = 1.4157 (within 2%)."""
    om = PH.landau_root(0.5)
    fits = []
    for seed in (0, 1, 2):
        w = W.landau_linear(seed=seed)
        st = w.state()
        _, _, hist = O.run(st["Q"], st["P"], st["qs"], st["ps"], st["psi"], w.L, w.ng, w.dt, 200)
        z = np.array([complex(h["e1_re"], h["e1_im"]) for h in hist])
        fits.append(PH.fit_damped_mode(np.arange(z.size) * w.dt, z, 2.0, 12.0))
    g = np.array([f[0] for f in fits])
    wr = np.array([f[1] for f in fits])
    assert abs(g.mean() - om.imag) < 0.01, fits
    assert np.all(np.abs(g - om.imag) < 0.02), fits
    assert np.all(np.abs(wr - om.real) < 0.02 * om.real), fits


def test_two_stream_root_value():
    """The two-stream configuration (k = 0.2, beams +-2.4, T = 1) is linearly unstable
    with a purely growing root."""
    om = PH.two_stream_root(0.2, 2.4)
    assert abs(om.real) < 1e-8 and 0.2 < om.imag < 0.25


def test_two_stream_growth_matches_dispersion_root():
    """T-L2 on a small lattice: the two-stream configuration (k = 0.2, alpha = 1e-3, beams
    +-2.4, T = 1, Ng = 64, 128 x 128 decorated particles, dt = 0.05) grows its mode-1 field
    at the rate of the unstable root (gamma = 0.2258): a least-squares line through
    log |E1| over t in [12, 26], after the stable beam modes have faded and before
    saturation, within 3%.  A wrong sign in the kick or in the deposit's dipole term
    turns the instability off."""
    om = PH.two_stream_root(0.2, 2.4)
    w = W.two_stream(nx=128, nv=128, ng=64)
    st = w.state()
    _, _, hist = O.run(st["Q"], st["P"], st["qs"], st["ps"], st["psi"], w.L, w.ng, w.dt, 540)
    t = np.arange(len(hist)) * w.dt
    a = np.array([abs(complex(h["e1_re"], h["e1_im"])) for h in hist])
    g = PH.fit_growth(t, a, 12.0, 26.0)
    assert abs(g - om.imag) < 0.03 * om.imag, (g, om.imag)


# ---------------------------------------------------------------- projection readings of phi_h''
def _mass_by_quadrature(L, ng):
    """M_ij = integral of phi_i phi_j over the periodic domain, by 4-point Gauss-Legendre on
    every element with the brute-force hats (exact for the quadratic integrands)."""
    h = L / ng
    xg, wg = np.polynomial.legendre.leggauss(4)
    M = np.zeros((ng, ng))
    for e in range(ng):
        x = e * h + 0.5 * h * (xg + 1.0)
        w = 0.5 * h * wg
        hats = np.array([_hat(x, j, L, ng) for j in range(ng)])
        M += (hats * w) @ hats.T
    return M


@pytest.mark.parametrize("ng", [8, 32])
def test_nodal_projections_match_assembled_mass_matrix(ng):
    """The consistent projection solves M g = -b~ with M assembled from the hats by
    quadrature; the lumped one uses M's row sums.  Both must match the oracle's
    (Fourier-diagonalised / scaled) forms."""
    rng = np.random.default_rng(ng)
    L = 3.3
    Q, _, _, ps, psi = _rand_particles(rng, 200, L, ng)
    f = O.solve_field(Q, ps, psi, L, ng)
    M = _mass_by_quadrature(L, ng)
    gc = np.linalg.solve(M, -f["bt"])
    gl = -f["bt"] / M.sum(axis=1)
    assert np.allclose(O.nodal_curvature(f["bt"], L, "consistent"), gc, rtol=0,
                       atol=1e-11 * np.abs(gc).max())
    assert np.allclose(O.nodal_curvature(f["bt"], L, "nodal"), gl, rtol=0,
                       atol=1e-12 * np.abs(gl).max())
    # the weak second derivative of phi_h against each hat is -b~_j: -(phi_h', phi_j')
    h = L / ng
    Phi = f["Phi"]
    slope = -f["E"]                                      # phi_h' per element
    weak = np.array([-sum(slope[e] * (_hat_slope((e + 0.5) * h, j, L, ng)) * h
                          for e in range(ng)) for j in range(ng)])
    assert np.allclose(weak, -f["bt"], rtol=0, atol=1e-11 * np.abs(f["bt"]).max())
    assert np.allclose(Phi.sum(), 0.0, atol=1e-12 * np.abs(Phi).max())


def test_element_projection_is_element_average_of_lumped_nodal():
    """The default (element-constant) reading equals the average over each element's two
    nodes of the lumped nodal reading (both are lumped projections; derived identity)."""
    rng = np.random.default_rng(9)
    L, ng = 5.0, 64
    Q, _, _, ps, psi = _rand_particles(rng, 500, L, ng)
    f = O.solve_field(Q, ps, psi, L, ng)
    gn = O.nodal_curvature(f["bt"], L, "nodal")
    assert np.allclose(f["g"], 0.5 * (gn + np.roll(gn, -1)), rtol=0,
                       atol=1e-12 * np.abs(gn).max())


def test_curvature_at_is_p1_interpolant():
    """For the nodal readings phi_h''(Q) is the P1 function sum_j g_j phi_j(Q) (brute-force
    hats); for the element reading it is the value of the element holding Q."""
    rng = np.random.default_rng(2)
    L, ng = 2.5, 16
    g = rng.normal(size=ng)
    Q = rng.uniform(0, L, 300)
    brute = np.array([sum(g[j] * _hat(q, j, L, ng) for j in range(ng)) for q in Q])
    for proj in ("nodal", "consistent"):
        assert np.allclose(O.curvature_at(Q, g, L, proj), brute, rtol=0, atol=1e-13)
    i = np.floor(Q / (L / ng)).astype(int)
    assert np.array_equal(O.curvature_at(Q, g, L, "elem"), g[i])


@pytest.mark.parametrize("proj", ["elem", "nodal", "consistent"])
def test_projected_curvature_converges_to_minus_density(proj):
    """phi'' = -(rho - n0): for rho = 1 + a cos(kx) carried by a fine uniform set of
    monopoles, every reading of phi_h'' at the mesh points tends to -a cos(kx) at second
    order in h (element readings at the element midpoints)."""
    L, a = 2 * np.pi, 0.3
    errs = []
    for ng in (16, 32, 64):
        n = 4096 * 8
        x = (np.arange(n) + 0.5) * L / n
        psi = (1.0 + a * np.cos(x)) * L / n
        f = O.solve_field(x, np.zeros(n), psi, L, ng, proj)
        h = L / ng
        pts = (np.arange(ng) + (0.5 if proj == "elem" else 0.0)) * h
        errs.append(np.abs(f["g"] + a * np.cos(pts)).max())
    assert errs[0] < 0.05 * a
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5, errs


def test_projection_enters_only_through_the_shape_kick():
    """The curvature multiplies p* in q*'s kick and nothing else: one step from the same
    state gives bitwise the same positions under every reading (the first half-kick and the
    drift of Q use E only), and different q*."""
    w = W.landau_linear(nx=32, nv=32, ng=32)
    st = w.state()
    out = {}
    for proj in O.PROJECTIONS:
        state, _, _ = O.run(st["Q"], st["P"], st["qs"], st["ps"], st["psi"], w.L, w.ng, w.dt,
                            1, projection=proj)
        out[proj] = state
    for proj in ("nodal", "consistent"):
        assert np.array_equal(out["elem"][0], out[proj][0])
        assert not np.array_equal(out["elem"][2], out[proj][2])


# ---------------------------------------------------------------- convergence (Theorem 2)
def _periodic_green(x, Q, L):
    """Zero-mean periodic solution of -phi'' = delta(x - Q) - 1/L:
    G(r) = r^2 / (2L) - r/2 + L/12, r = (x - Q) mod L."""
    r = (x - Q) % L
    return r * r / (2 * L) - r / 2 + L / 12


def _periodic_dipole(x, Q, L):
    """Zero-mean periodic solution of -phi'' = delta'(x - Q): dG/dr = r/L - 1/2."""
    r = (x - Q) % L
    return r / L - 0.5


def _l2_error_p1(Phi, exact, Q, L):
    """|| exact - P1 interpolant of Phi ||_L2 by 6-point Gauss-Legendre on each element,
    the element holding Q split at Q (the exact solution has a kink or jump there)."""
    ng = Phi.shape[0]
    h = L / ng
    xg, wg = np.polynomial.legendre.leggauss(6)
    tot = 0.0
    for e in range(ng):
        a, b = e * h, (e + 1) * h
        cuts = [a, Q, b] if a < Q < b else [a, b]
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            x = 0.5 * (hi - lo) * (xg + 1.0) + lo
            w = 0.5 * (hi - lo) * wg
            s = (x - a) / h
            ph = (1 - s) * Phi[e] + s * Phi[(e + 1) % ng]
            tot += np.sum(w * (exact(x) - ph) ** 2)
    return math.sqrt(tot)


def test_point_source_convergence_rates():
    """T-S5 (Theorem 2): for one monopole the L2 error of the Galerkin potential falls as
    h^(3/2), for one dipole as h^(1/2) (the exact potential has a kink, resp. a jump, at
    the particle).  Q sits at the same relative place in its element on every mesh."""
    L = 1.0
    rates = {}
    for kind in ("monopole", "dipole"):
        hs, errs = [], []
        for ng in (16, 32, 64, 128, 256, 512, 1024):
            h = L / ng
            Q = L / 4 + 0.3 * h
            psi, ps = (1.0, 0.0) if kind == "monopole" else (0.0, 1.0)
            f = O.solve_field(np.array([Q]), np.array([ps]), np.array([psi]), L, ng)
            exact = (lambda x: _periodic_green(x, Q, L)) if kind == "monopole" else \
                (lambda x: _periodic_dipole(x, Q, L))
            hs.append(h)
            errs.append(_l2_error_p1(f["Phi"], exact, Q, L))
        rates[kind] = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert abs(rates["monopole"] - 1.5) < 0.1, rates
    assert abs(rates["dipole"] - 0.5) < 0.05, rates


# ---------------------------------------------------------------- decorated particle in a potential
def _pendulum_field(Q, kappa):
    """V(q) = 1 - cos(kappa q): E = -V'(Q), curvature g = V''(Q)."""
    return -kappa * np.sin(kappa * Q), kappa * kappa * np.cos(kappa * Q)


def _kdk_prescribed(state, kappa, L, dt, n):
    Q, P, qs, ps, psi = (np.array(a, dtype=np.float64) for a in state)
    for _ in range(n):
        P, qs = O.kick_values(P, qs, ps, *_pendulum_field(Q, kappa), 0.5 * dt)
        Q, ps = O.drift(Q, P, qs, ps, L, dt)
        P, qs = O.kick_values(P, qs, ps, *_pendulum_field(Q, kappa), 0.5 * dt)
    return Q, P, qs, ps, psi


def test_shape_variables_are_the_tangent_of_the_central_motion():
    """T-P3 (eq. sw_prescribed_potential): (p*, -q*) evolves as the linearisation of the
    (Q, P) map along its trajectory, so two central trajectories started eps (p*, -q*)
    apart separate by eps (p*_n, -q*_n) + O(eps^2).  A wrong sign or factor in the q* kick
    or in the p* drift breaks it."""
    L = 10.0
    kappa = 2 * np.pi / L
    base = ([2.0, 5.5, 8.0], [0.4, -0.7, 1.1], [0.1, -0.2, 0.05], [0.3, 0.1, -0.25],
            [1.0, 1.0, 1.0])
    dt, n = 0.05, 400
    Q, P, qs, ps, _ = _kdk_prescribed(base, kappa, L, dt, n)
    res = []
    for eps in (1e-4, 1e-5):
        Qe, Pe, _, _, _ = _kdk_prescribed(
            (np.add(base[0], eps * np.array(base[3])), np.subtract(base[1], eps * np.array(base[2])),
             base[2], base[3], base[4]), kappa, L, dt, n)
        dQ = _wrap_dist(Qe, Q, L) / eps
        dP = (Pe - P) / eps
        res.append(max(np.abs(dQ - ps).max(), np.abs(dP + qs).max()))
    assert res[0] < 1e-3 * max(np.abs(ps).max(), np.abs(qs).max()), res
    assert res[1] < res[0] / 5, res                      # first order in eps


def test_test_particle_hamiltonian_is_bounded_at_second_order():
    """T-P5: three decorated particles in V = 1 - cos(kappa q), L = 10 (the paper's
    test-particle example, eq. swpic_test_particle): H_SWPIC under the splitting stays
    within an O(dt^2) band with no secular drift."""
    L = 10.0
    kappa = 2 * np.pi / L

    def H(st):
        Q, P, qs, ps, psi = st
        return float(np.sum(0.5 * psi * P * P + P * qs + psi * (1 - np.cos(kappa * Q))
                            - ps * kappa * np.sin(kappa * Q)))

    st0 = ([2.0, 5.0, 8.0], [0.5, -0.3, 1.0], [0.1, -0.05, 0.02], [0.05, 0.1, -0.03],
           [10.0, 10.0, 10.0])
    H0 = H(tuple(np.array(a) for a in st0))
    bands = []
    for dt in (0.1, 0.05):
        n = int(round(200.0 / dt))
        st = tuple(np.array(a, dtype=np.float64) for a in st0)
        dev = []
        for _ in range(n // 20):
            st = _kdk_prescribed(st, kappa, L, dt, 20)
            dev.append(H(st) - H0)
        dev = np.abs(np.array(dev))
        bands.append(dev.max())
        q = dev.size // 4
        quarters = [dev[k * q:(k + 1) * q].max() for k in range(4)]
        assert max(quarters) < 1.3 * min(quarters), quarters      # no secular growth
    assert bands[0] < 1e-3 * abs(H0)
    assert 3.6 < bands[0] / bands[1] < 4.4, bands                # second order in dt


def test_bump_on_tail_root_value():
    """The bump-on-tail configuration of the served mix (k = 0.3; the velocity profile is
    0.9 N(0, 1) + 0.1 N(4.5, 1/4)) is unstable: the root of the Vlasov dispersion relation
    has omega = 1.0012 + 0.1981i.  A check that the unit-density normalisation of the two
    Maxwellians is read correctly (the density of the bump sets the growth rate)."""
    om = PH.bump_on_tail_root(0.3)
    assert abs(om.real - 1.0012) < 2e-3 and abs(om.imag - 0.1981) < 2e-3, om


# ---------------------------------------------------------------- prescribed potential
def test_run_without_self_field_is_the_test_particle_system():
    """O.run with a prescribed potential and no self field is exactly the splitting of
    eq. swpic_test_particle (the hand-written field of the test above, bitwise), and its
    H = K + U is the paper's H_SWPIC."""
    L = 10.0
    kappa = 2 * np.pi / L
    st0 = ([2.0, 5.0, 8.0], [0.5, -0.3, 1.0], [0.1, -0.05, 0.02], [0.05, 0.1, -0.03],
           [10.0, 10.0, 10.0])
    dt, n = 0.05, 200
    ref = _kdk_prescribed(st0, kappa, L, dt, n)
    got, _, hist = O.run(*(np.array(a) for a in st0), L, 16, dt, n,
                         ext={"amp": 1.0, "mode": 1}, self_field=False)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    Q, P, qs, ps, psi = ref
    h_swpic = float(np.sum(0.5 * psi * P * P + P * qs + psi * (1 - np.cos(kappa * Q))
                           - ps * kappa * np.sin(kappa * Q)))
    assert abs(hist[-1]["H"] - h_swpic) < 1e-12 * abs(h_swpic)
    assert hist[-1]["W"] == 0.0 and hist[-1]["e_amp"] == 0.0


def test_external_energy_gradients_are_the_external_field():
    """dU/dp*_a = -V'(Q_a) = E_ext(Q_a) and dU/dQ_a = psi*_a V'(Q_a) - p*_a V''(Q_a),
    by central differences (U is smooth)."""
    rng = np.random.default_rng(8)
    L, ext = 7.0, {"amp": 0.7, "mode": 2}
    Q = rng.uniform(0, L, 5)
    ps = rng.normal(size=5) * 0.1
    psi = rng.uniform(0.5, 1.5, 5)
    E, g = O.external_field(Q, L, ext)
    eps = 1e-6
    for a in range(5):
        d = np.zeros(5)
        d[a] = eps
        dU_dps = (O.external_energy(Q, ps + d, psi, L, ext)
                  - O.external_energy(Q, ps - d, psi, L, ext)) / (2 * eps)
        dU_dQ = (O.external_energy(Q + d, ps, psi, L, ext)
                 - O.external_energy(Q - d, ps, psi, L, ext)) / (2 * eps)
        assert abs(dU_dps - E[a]) < 1e-8
        assert abs(dU_dQ - (psi[a] * (-E[a]) - ps[a] * g[a])) < 1e-7


def test_energy_with_self_field_and_potential_is_bounded():
    """Landau plasma in an added potential (self field on): H = K + U + W stays within a
    band over 100 steps: 2e-4 in the PIC special case, 5e-3 with dipoles (whose P1 load
    jumps at node crossings, R7); the potential does work (U of order H)."""
    w = W.landau_linear(nx=64, nv=64, ng=64)
    st = w.state()
    ext = {"amp": 0.05, "mode": 1}
    z = np.zeros_like(st["Q"])
    for dip, bound in ((True, 5e-3), (False, 2e-4)):
        qs, ps = (st["qs"], st["ps"]) if dip else (z, z)
        _, _, hist = O.run(st["Q"], st["P"], qs, ps, st["psi"], w.L, w.ng, w.dt, 100, ext=ext)
        H = np.array([h["H"] for h in hist])
        U = np.array([h["U"] for h in hist])
        assert np.max(np.abs(U)) > 0.05 * abs(H[0])
        assert np.max(np.abs(H - H[0])) / abs(H[0]) < bound, dip


# ---------------------------------------------------------------- P2 elements
def _p2_fn(x, kind, j, L, ng):
    """Periodic P2 basis function from its definition: the vertex function of node j is
    (1 - s)(1 - 2s) on element j and s(2s - 1) on element j - 1; the midpoint function of
    element j is 4 s (1 - s) on element j; zero elsewhere."""
    h = L / ng
    x = np.asarray(x, dtype=np.float64) % L
    e = np.floor(x / h).astype(int) % ng
    s = x / h - np.floor(x / h)
    if kind == "v":
        return np.where(e == j, (1 - s) * (1 - 2 * s),
                        np.where(e == (j - 1) % ng, s * (2 * s - 1), 0.0))
    return np.where(e == j, 4 * s * (1 - s), 0.0)


def _p2_slope(x, kind, j, L, ng, d=1e-7):
    return (_p2_fn(x + d, kind, j, L, ng) - _p2_fn(x - d, kind, j, L, ng)) / (2 * d)


def test_p2_deposit_brute_force():
    rng = np.random.default_rng(21)
    L, ng = 3.0, 6
    Q, _, _, ps, psi = _rand_particles(rng, 40, L, ng)
    bv, bm = O.deposit_p2(Q, ps, psi, L, ng)
    for j in range(ng):
        rv = sum(psi[a] * _p2_fn(Q[a], "v", j, L, ng) - ps[a] * _p2_slope(Q[a], "v", j, L, ng)
                 for a in range(Q.size))
        rm = sum(psi[a] * _p2_fn(Q[a], "m", j, L, ng) - ps[a] * _p2_slope(Q[a], "m", j, L, ng)
                 for a in range(Q.size))
        assert abs(bv[j] - rv) < 1e-6 and abs(bm[j] - rm) < 1e-6
    assert abs(bv.sum() + bm.sum() - psi.sum()) < 1e-12 * psi.sum()   # the basis sums to one


def test_p2_stiffness_by_quadrature():
    """A_kl = integral of phi_k' phi_l' (3-point Gauss-Legendre per element on slopes of the
    brute-force basis) equals the assembled element matrices."""
    L, ng = 2.0, 5
    h = L / ng
    xg, wg = np.polynomial.legendre.leggauss(3)
    fns = [("v", j) for j in range(ng)] + [("m", j) for j in range(ng)]
    A = O.p2_stiffness(L, ng)
    order = lambda kind, j: 2 * j + (0 if kind == "v" else 1)  # noqa: E731
    for ka, ja in fns:
        for kb, jb in fns:
            tot = 0.0
            for e in range(ng):
                x = e * h + 0.5 * h * (xg + 1)
                tot += np.sum(0.5 * h * wg * _p2_slope(x, ka, ja, L, ng) * _p2_slope(x, kb, jb, L, ng))
            assert abs(A[order(ka, ja), order(kb, jb)] - tot) < 1e-5 / h


def test_p2_monopole_is_exact_at_vertices_and_energy_identity():
    """Theorem 1 for degree 2: one monopole's Galerkin potential equals the continuous
    periodic solution at the vertices up to the gauge constant; and W = (1/2) Phi^T A Phi
    equals (1/2) integral of E^2 with E from the basis."""
    L, ng = 1.0, 16
    h = L / ng
    for Q in (0.31 * L, 0.5 * L + 0.2 * h):
        f = O.solve_field_p2(np.array([Q]), np.zeros(1), np.ones(1), L, ng)
        v = np.arange(ng) * h
        r = (v - Q) % L
        G = r * r / (2 * L) - r / 2 + L / 12
        d = f["Phv"] - G
        assert np.ptp(d) < 1e-12
        xg, wg = np.polynomial.legendre.leggauss(4)
        s = 0.5 * (xg + 1)
        WE = 0.5 * sum(np.sum(0.5 * wg * h * (f["E0"][e] + s * f["E1"][e]) ** 2) for e in range(ng))
        assert abs(WE - f["W"]) < 1e-12 * f["W"]


def test_p2_smooth_solution_converges_at_third_order():
    """For the load of rho - n0 = a cos(kx) (by quadrature against the basis) the P2
    potential approaches (a / k^2) cos(kx) in L2 as h^3, and its exact second derivative
    tracks -a cos(kx) at second order."""
    L, a = 2 * np.pi, 0.4
    errs, gerrs = [], []
    for ng in (8, 16, 32):
        h = L / ng
        xg, wg = np.polynomial.legendre.leggauss(6)
        bv, bm = np.zeros(ng), np.zeros(ng)
        for e in range(ng):
            x = e * h + 0.5 * h * (xg + 1)
            s = 0.5 * (xg + 1)
            N, _ = O.p2_basis(s)
            rho = a * np.cos(x)
            bv[e] += np.sum(0.5 * h * wg * rho * N[0])
            bv[(e + 1) % ng] += np.sum(0.5 * h * wg * rho * N[2])
            bm[e] += np.sum(0.5 * h * wg * rho * N[1])
        Phv, Phm = O.poisson_solve_p2(bv, bm, L)
        err2 = 0.0
        for e in range(ng):
            x = e * h + 0.5 * h * (xg + 1)
            s = 0.5 * (xg + 1)
            N, _ = O.p2_basis(s)
            ph = Phv[e] * N[0] + Phm[e] * N[1] + Phv[(e + 1) % ng] * N[2]
            err2 += np.sum(0.5 * h * wg * (ph - a * np.cos(x)) ** 2)
        errs.append(math.sqrt(err2))
        # phi_h'' (exact for P2, constant per element) tracks phi'' = -a cos(x)
        _, _, g = O.field_p2(Phv, Phm, L)
        xm = (np.arange(ng) + 0.5) * h
        gerrs.append(np.max(np.abs(g + a * np.cos(xm))))
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0, errs
    assert gerrs[2] < 0.01 * a and gerrs[1] / gerrs[2] > 3.5, gerrs


def test_p2_field_energy_of_the_landau_lattice_converges():
    """With several particles per element across x, the P2 field energy of the linear
    Landau state approaches (1/2)(alpha/k)^2 L/2; with one particle column per element the
    midpoint unknowns resolve the particles' discreteness and the energy is far off."""
    exact = 0.5 * (0.01 / 0.5) ** 2 * (4 * np.pi) / 2
    w = W.landau_linear(nx=1024, nv=64, ng=64)
    st = w.state()
    f = O.solve_field_p2(st["Q"], st["ps"], st["psi"], w.L, w.ng)
    assert abs(f["W"] - exact) < 1e-3 * exact
    w = W.landau_linear(nx=64, nv=64, ng=64)
    st = w.state()
    assert O.solve_field_p2(st["Q"], st["ps"], st["psi"], w.L, w.ng)["W"] > 5 * exact


def test_p2_without_self_field_is_the_element_free_test_particle_flow():
    """With no field of their own the particles see only the prescribed potential, so the
    P2 run and the P1 run agree exactly (the mesh takes no part in the kicks), and a
    particle at rest at the potential's minimum with no dipoles stays there."""
    rng = np.random.default_rng(12)
    L, ng, n = 10.0, 16, 40
    Q = rng.uniform(0, L, n)
    P = rng.normal(0, 0.5, n)
    qs = rng.normal(0, 0.05, n)
    ps = rng.normal(0, 0.05, n)
    psi = rng.uniform(0.5, 1.5, n)
    Q[0], P[0], qs[0], ps[0] = 0.0, 0.0, 0.0, 0.0
    ext = {"amp": 0.7, "mode": 2}
    a, _, ha = O.run_p2(Q, P, qs, ps, psi, L, ng, 0.05, 30, ext=ext, self_field=False)
    b, _, hb = O.run(Q, P, qs, ps, psi, L, ng, 0.05, 30, ext=ext, self_field=False)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert [h["H"] for h in ha] == [h["H"] for h in hb]
    assert all(h["W"] == 0.0 for h in ha)
    assert a[0][0] == 0.0 and a[1][0] == 0.0
    # with the self field the P2 field does act (a different trajectory from P1)
    c, _, _ = O.run_p2(Q, P, qs, ps, psi, L, ng, 0.05, 30, ext=ext)
    assert not np.allclose(c[1], b[1])


# ---------------------------------------------------------------- momentum and FP32 storage
def test_momentum_is_the_velocity_moment_of_the_ansatz():
    """diagnostics()['momentum'] is the integral of p f over phase space for the ansatz of
    eq. sw_f_ansatz: the monopole psi* delta_Z gives psi* P, the spatial dipole
    p* d_q delta_Z gives nothing, and the momentum dipole -q* d_p delta_Z gives +q*.  Two
    independent values fix it:
      (1) lattice cells of an asymmetric profile (bump on tail) with velocity jitter: the
          cell moments make psi* P + q* the integral of v f0 over each cell, so the total is
          int X dx * int v V(v) dv, here by adaptive quadrature of the profile;
      (2) decorated particles made from markers by Algorithm 1: the total is the markers'
          sum w p.
    The jitter puts each centre off its cell's mean velocity, so q* carries a sizeable share:
    dropping it or flipping its sign misses both values by far more than the tolerance."""
    from scipy.integrate import quad
    from workloads import lattice as LT
    k, alpha = 0.3, 0.04
    L = 2 * math.pi / k
    vmin, vmax, ng = -8.0, 10.0, 32
    X, V = LT.bump_on_tail_profile(alpha, k)
    st = LT.make_lattice(L, 32, 72, vmin, vmax, (X, V), seed=5, jx=1.0, jv=1.0)
    fld = O.solve_field(st["Q"], st["ps"], st["psi"], L, ng)
    mom = O.diagnostics(st["P"], st["qs"], st["psi"], fld, L)["momentum"]
    ix = quad(X, 0.0, L, epsabs=0, epsrel=1e-13, limit=200)[0]
    iv = quad(lambda v: v * V(v), vmin, vmax, epsabs=0, epsrel=1e-13, limit=400)[0]
    ref = ix * iv
    tol = 1e-11 * abs(ref)
    assert abs(mom - ref) < tol, (mom, ref)
    assert abs(np.sum(st["qs"])) > 1e4 * tol  # q* matters at this tolerance

    rng = np.random.default_rng(11)
    m, kc = 6000, 500
    q = rng.uniform(0.0, L, m)
    p = np.where(rng.uniform(size=m) < 0.8, rng.normal(0.0, 1.0, m), rng.normal(4.5, 0.5, m))
    wm = rng.uniform(0.5, 1.5, m) * (L / m)
    init = rng.choice(m, kc, replace=False)
    dec, _ = O.cluster_markers(q, p, wm, init, 6, L)
    fld = O.solve_field(dec["Q"], dec["ps"], dec["psi"], L, ng)
    mom = O.diagnostics(dec["P"], dec["qs"], dec["psi"], fld, L)["momentum"]
    ref = float(np.sum(wm * p))
    tol = 1e-12 * float(np.sum(np.abs(wm * p)))
    assert abs(mom - ref) < tol, (mom, ref)
    assert abs(np.sum(dec["qs"])) > 1e4 * tol


def test_fp32_storage_departs_from_fp64_on_linear_landau():
    """Rounding the state to float32 at a GPU path's storage points, every step otherwise
    computed in float64 from the stored values (tests/fp32_reference.py), moves the linear
    Landau W history (4096 particles, Ng 64, dt 0.1, 200 steps, from the same float32 initial
    bits) away from the float64 run.  A particle whose rounded position crosses a node one step
    earlier or later shifts the dipole load by 2 p* / h there (the P1 slope jumps at a node),
    and these shifts accumulate.  Measured relative L2 over the 201 samples (seeds 0, 1, 2):
    0.083, 0.059, 0.058 at the primitive path's storage points, 0.018, 0.015, 0.052 at the
    fused step's; within the first 50 steps 4e-6 to 4e-4.  So float32 storage does not meet
    the 1e-4 history target against the float64 oracle, whatever the accumulation; the GPU's
    float32 runs are held to these references instead, and their departure from the float64
    oracle to the departure pinned here."""
    import fp32_reference as FR
    for seed in (0, 1, 2):
        w = W.landau_linear(seed=seed)
        s64 = {k: v.astype(np.float64) for k, v in w.state(np.float32).items()}
        _, _, ref = O.run(s64["Q"], s64["P"], s64["qs"], s64["ps"], s64["psi"], w.L, w.ng,
                          w.dt, w.nsteps)
        Wo = np.array([h["W"] for h in ref])
        for fn in (FR.fp32_storage_reference, FR.fp32_fused_reference):
            Wx = fn(s64, w, w.nsteps)[0]
            err = np.linalg.norm(Wx - Wo) / np.linalg.norm(Wo)
            early = np.linalg.norm(Wx[:51] - Wo[:51]) / np.linalg.norm(Wo[:51])
            assert 5e-3 < err < 0.15, (seed, fn.__name__, err)
            assert early < 1e-3, (seed, fn.__name__, early)
