"""Plain FP64 CPU oracle for the decorated-particle (Scovel-Weinstein, k = 2) cycle.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference the HIP
path is checked against.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product path never does.  It shares no code with the
HIP library: it imports NumPy and nothing else.

Everything below is written from the paper (arXiv 2605.21794, "A Structure-Preserving
Decorated Particle Method for the Vlasov-Poisson System"), Section 5 "Discretization in
space and time", in the normalised 1D1V setting e = m = eps0 = 1 on the periodic
domain [0, L).

Readings taken where the paper is silent:
  * finite elements are P1 (degree k = 1) on a uniform periodic mesh of Ng elements,
    h = L / Ng, element e = [e h, (e+1) h), nodes q_j = j h, node Ng == node 0;
  * a particle sitting exactly on a node belongs to the element on its right;
  * the second derivative phi_h'' needed by the dipole equation (eq. sw-evolution) is
    taken from the lumped-mass L2 projection of the element-constant field E_h onto
    P1, then differentiated on each element (the paper's projection step for phi_h'').
    Two other readings of that step are available behind the `projection` argument:
    the L2 projection onto P1 of phi_h'' itself, taken in the weak sense
    ((phi_h'', phi_j) = -(phi_h', phi_j') = -b~_j), with the lumped ("nodal") or the
    consistent ("consistent") mass matrix, evaluated at Q by P1 interpolation;
  * the paper's leapfrog (the standard PIC one) is read as the kick-drift-kick Strang splitting of
    H_h = H_kin + H_field, each sub-flow solved exactly (derived from the 1D bracket,
    eq. lp1d): the kick freezes (Q, p*) and moves (P, q*), the drift freezes (P, q*)
    and moves (Q, p*).

Functions and the passages they follow:
  cell_index          -- locating Q in the mesh (P1 local support; half-open elements)
  deposit             -- eq. rhs-assembly (monopole + dipole load vector b)
  neutralize          -- eq. neutrality / zero-mean background (b - mean(b))
  poisson_solve       -- eq. lin-sys with the gauge 1^T Phi = 0
  element_field       -- E_e = -phi_h' on each element (field read from the basis)
  projected_curvature -- phi_h'' via the lumped L2 projection (reading above)
  mass_eigenvalues,
  nodal_curvature     -- the two other projections of phi_h'' (readings above)
  curvature_at        -- phi_h''(Q_a) from any of the three projections
  kick_values, kick,
  drift               -- exact sub-flows of eq. sw-evolution split as above
  external_field,
  external_energy     -- a prescribed potential V(q) = A (1 - cos(kappa q)) added to the
                         field (eq. sw_prescribed_potential, eq. swpic_test_particle), and
                         its part of the Hamiltonian; `self_field=False` drops the particles'
                         own field (charge e = 0, the paper's test-particle example)
  diagnostics         -- eq. Hh (discrete Hamiltonian), eq. Eamp, charge, momentum
  deposit_p2 ... run_p2 -- the same cycle with P2 elements (degree-2 Lagrange basis,
                         assembled stiffness, bordered solve refined in extended precision,
                         exact phi_h''), from their definitions
  sort_perm           -- chunked stable counting sort by cell (a layout step of the
                         GPU path; its meaning is fixed here, not by the paper)
  run                 -- the whole cycle, one field solve per step

parity unpinned: the choice among the three projections for phi_h'' (no printed value in
the paper discriminates between them); each projection itself, and every other function, is
pinned by the tests in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "inv_h", "cell_index", "deposit", "neutralize", "poisson_eigenvalues",
    "poisson_solve", "element_field", "projected_curvature", "mass_eigenvalues",
    "nodal_curvature", "curvature_at", "solve_field", "kick_values", "kick", "drift", "wrap",
    "diagnostics", "sort_perm", "step", "run", "PROJECTIONS", "external_field",
    "external_energy", "p2_basis", "deposit_p2", "p2_node_weights", "neutralize_p2",
    "p2_stiffness", "poisson_solve_p2", "field_p2", "solve_field_p2", "field_from_load_p2",
    "kick_p2", "step_p2",
    "run_p2",
]

# Readings of the projection step for phi_h'': element-constant from the lumped projection
# of E (the default), or a P1 function from the lumped / consistent projection of phi_h''.
PROJECTIONS = ("elem", "nodal", "consistent")


def inv_h(L: float, ng: int) -> float:
    """1/h = Ng / L, one FP64 division (uniform periodic mesh, Section 5)."""
    return float(ng) / float(L)


def cell_index(Q, L: float, ng: int):
    """Element index i and local coordinate s of each position.

    x = Q * (Ng / L) in FP64 (FP32 inputs are promoted exactly); i = floor(x) clamped to
    [0, Ng-1] (a position rounding onto L lands in the last element); s = x - i clipped
    to [0, 1].  Elements are half-open, so a particle on node j is in element j.
    """
    x = np.asarray(Q, dtype=np.float64) * inv_h(L, ng)
    i = np.floor(x).astype(np.int64)
    i = np.minimum(np.maximum(i, 0), ng - 1)
    s = np.clip(x - i, 0.0, 1.0)
    return i, s


def deposit(Q, ps, psi, L: float, ng: int):
    """Load vector b_j = sum_a [psi*_a phi_j(Q_a) - p*_a phi_j'(Q_a)] (eq. rhs-assembly).

    On element i the two P1 hats that do not vanish are phi_i = 1 - s and
    phi_{i+1} = s, with slopes -1/h and +1/h.  So particle a adds
    psi*(1 - s) + p*/h to node i and psi* s - p*/h to node i+1 (mod Ng).
    The result still contains the full monopole charge: sum_j b_j = sum_a psi*_a.
    """
    ps = np.asarray(ps, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    i, s = cell_index(Q, L, ng)
    ih = inv_h(L, ng)
    w_left = psi * (1.0 - s) + ps * ih
    w_right = psi * s - ps * ih
    b = np.bincount(i, weights=w_left, minlength=ng)
    b = b + np.bincount((i + 1) % ng, weights=w_right, minlength=ng)
    return b


def neutralize(b):
    """Subtract the uniform background (eq. neutrality: n0 L = sum psi*).

    The background's load on node j is n0 * integral(phi_j) = n0 h, and
    n0 h = (sum_a psi*_a) / Ng = mean(b) because the hats sum to one.  The paper notes the
    background drops out against zero-mean test functions; removing the mean makes the
    load consistent with the singular stiffness matrix.
    """
    b = np.asarray(b, dtype=np.float64)
    return b - b.mean()


def poisson_eigenvalues(L: float, ng: int):
    """Eigenvalues of the periodic P1 stiffness matrix A = (1/h) circ(-1, 2, -1).

    A is circulant, so its eigenvectors are the discrete Fourier modes and
    lambda_m = (2/h) (1 - cos(2 pi m / Ng)); lambda_0 = 0 spans the kernel {1}.
    """
    h = float(L) / ng
    m = np.arange(ng)
    return (2.0 / h) * (1.0 - np.cos(2.0 * np.pi * m / ng))


def poisson_solve(bt, L: float):
    """Phi with A Phi = b~ and 1^T Phi = 0 (eq. lin-sys with the zero-mean gauge).

    The circulant A is diagonal in the Fourier basis; the gauge removes mode 0.  The FFT
    is a library primitive standing in for that diagonalisation.
    """
    bt = np.asarray(bt, dtype=np.float64)
    ng = bt.shape[0]
    lam = poisson_eigenvalues(L, ng)
    bh = np.fft.fft(bt)
    ph = np.zeros_like(bh)
    ph[1:] = bh[1:] / lam[1:]
    return np.fft.ifft(ph).real


def element_field(Phi, L: float):
    """E_e = -phi_h' on element e = -(Phi_{e+1} - Phi_e) / h (field from the basis)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    ng = Phi.shape[0]
    return -(np.roll(Phi, -1) - Phi) * inv_h(L, ng)


def projected_curvature(E, L: float):
    """phi_h'' per element from the lumped L2 projection of E_h onto P1.

    The lumped projection of an element-constant function onto P1 on a uniform mesh is
    the nodal average E_n_j = (E_{j-1} + E_j) / 2.  Projected phi_h' is -E_n, so on
    element e: phi_h'' = g_e = -(E_n_{e+1} - E_n_e) / h.
    """
    E = np.asarray(E, dtype=np.float64)
    ng = E.shape[0]
    En = 0.5 * (np.roll(E, 1) + E)
    return -(np.roll(En, -1) - En) * inv_h(L, ng)


def mass_eigenvalues(L: float, ng: int):
    """Eigenvalues of the periodic P1 mass matrix M_ij = integral(phi_i phi_j).

    On a uniform periodic mesh M = (h/6) circ(1, 4, 1), circulant, so
    mu_m = (h/3) (2 + cos(2 pi m / Ng)), all positive.
    """
    h = float(L) / ng
    m = np.arange(ng)
    return (h / 3.0) * (2.0 + np.cos(2.0 * np.pi * m / ng))


def nodal_curvature(bt, L: float, projection: str):
    """phi_h'' as a P1 function g = sum_j g_j phi_j: the L2 projection of the weak second
    derivative of phi_h, (phi_h'', phi_j) = -(phi_h', phi_j') = -(A Phi)_j = -b~_j.

    projection "nodal": lumped mass (M replaced by its row sums, h on the diagonal), so
    h g_j = -b~_j; "consistent": M g = -b~ with the full mass matrix, solved in the Fourier
    basis of the circulant M.
    """
    bt = np.asarray(bt, dtype=np.float64)
    ng = bt.shape[0]
    if projection == "nodal":
        return -bt * inv_h(L, ng)
    if projection == "consistent":
        return np.fft.ifft(-np.fft.fft(bt) / mass_eigenvalues(L, ng)).real
    raise ValueError(f"not a nodal projection: {projection!r}")


def curvature_at(Q, g, L: float, projection: str):
    """phi_h''(Q_a): the element value g[i] for the element-constant projection; the P1
    interpolant (1 - s) g_i + s g_{i+1} for the nodal and consistent ones."""
    g = np.asarray(g, dtype=np.float64)
    ng = g.shape[0]
    i, s = cell_index(Q, L, ng)
    if projection == "elem":
        return g[i]
    if projection in ("nodal", "consistent"):
        return (1.0 - s) * g[i] + s * g[(i + 1) % ng]
    raise ValueError(f"unknown projection {projection!r}")


def solve_field(Q, ps, psi, L: float, ng: int, projection: str = "elem"):
    """Deposit, neutralise, solve; returns dict with b, bt, Phi, E, g, W, projection."""
    b = deposit(Q, ps, psi, L, ng)
    bt = neutralize(b)
    Phi = poisson_solve(bt, L)
    E = element_field(Phi, L)
    if projection == "elem":
        g = projected_curvature(E, L)
    else:
        g = nodal_curvature(bt, L, projection)
    h = float(L) / ng
    W = 0.5 * h * np.sum(E * E)
    return {"b": b, "bt": bt, "Phi": Phi, "E": E, "g": g, "W": W, "projection": projection}


def kick_values(P, qs, ps, Ea, ga, tau: float):
    """Exact flow of the field part of the Hamiltonian for time tau, given each particle's
    field value Ea = -phi'(Q_a) and curvature ga = phi''(Q_a).  Q and p* are frozen (so are
    Ea and ga), hence
        P  <- P  + tau * Ea              (dP/dt  = -phi'(Q)),
        q* <- q* + tau * p* * ga         (dq*/dt =  p* phi''(Q)),
    with the products evaluated left to right (eq. sw-evolution; with a prescribed
    potential V in place of phi, eq. sw_prescribed_potential).
    """
    P = np.asarray(P, dtype=np.float64) + tau * np.asarray(Ea, dtype=np.float64)
    qs = np.asarray(qs, dtype=np.float64) + tau * np.asarray(ps, dtype=np.float64) * ga
    return P, qs


def external_field(Q, L: float, ext):
    """Field and curvature of the prescribed potential V(q) = A (1 - cos(kappa q)),
    kappa = 2 pi m / L (ext = {"amp": A, "mode": m}): E = -V'(Q) = -(A kappa) sin(kappa Q),
    phi'' = V''(Q) = (A kappa^2) cos(kappa Q)."""
    Q = np.asarray(Q, dtype=np.float64)
    k = 2.0 * np.pi * ext["mode"] / L
    ak = ext["amp"] * k
    akk = ak * k
    return -(ak * np.sin(k * Q)), akk * np.cos(k * Q)


def external_energy(Q, ps, psi, L: float, ext):
    """The prescribed potential's part of H_SWPIC: sum psi* V(Q) - p* V'(Q)."""
    Q = np.asarray(Q, dtype=np.float64)
    k = 2.0 * np.pi * ext["mode"] / L
    a = float(ext["amp"])
    ak = a * k
    return float(np.sum(np.asarray(psi) * (a * (1.0 - np.cos(k * Q)))
                        - np.asarray(ps) * (ak * np.sin(k * Q))))


def kick(Q, P, qs, ps, E, g, L: float, tau: float, projection: str = "elem", ext=None,
         self_field: bool = True):
    """Exact flow of the field part of the Hamiltonian for time tau with the mesh field:
    Ea = E[i_a] read from the basis, ga = phi_h''(Q_a) from the projection; without the
    self field these are zero; a prescribed potential adds its field and curvature."""
    ng = np.asarray(E).shape[0]
    i, _ = cell_index(Q, L, ng)
    Ea = np.asarray(E)[i]
    ga = curvature_at(Q, g, L, projection)
    if not self_field:
        Ea = np.zeros_like(Ea)
        ga = np.zeros_like(ga)
    if ext is not None:
        ee, ge = external_field(Q, L, ext)
        Ea = Ea + ee
        ga = ga + ge
    return kick_values(P, qs, ps, Ea, ga, tau)


def wrap(Qn, L: float):
    """Bring Q + dt P back into [0, L): add L if negative, then subtract L if >= L.

    Valid when |dt P| < L (checked by the caller)."""
    Qn = np.asarray(Qn, dtype=np.float64).copy()
    Qn = np.where(Qn < 0.0, Qn + L, Qn)
    Qn = np.where(Qn >= L, Qn - L, Qn)
    return Qn


def drift(Q, P, qs, ps, L: float, tau: float):
    """Exact flow of H_kin = sum (psi* P^2 / 2 + q* P) for time tau.

    P and q* are frozen, so Q <- Q + tau P (periodic wrap) and p* <- p* - tau q*.
    """
    Qn = wrap(np.asarray(Q, dtype=np.float64) + tau * np.asarray(P, dtype=np.float64), L)
    psn = np.asarray(ps, dtype=np.float64) - tau * np.asarray(qs, dtype=np.float64)
    return Qn, psn


def diagnostics(P, qs, psi, fld, L: float, Q=None, ps=None, ext=None, self_field: bool = True):
    """FP64 invariants: K, W, U, H (eq. Hh), charge, momentum, E_amp (eq. Eamp), E mode 1.

    K = sum psi* P^2 / 2 + q* P; W = (1/2) Phi^T A Phi = (1/2) sum_e h E_e^2 (zero without
    the self field); U = the prescribed potential's energy (zero without one); H = K + U + W;
    momentum = sum (psi* P + q*) (first p-moment of the ansatz); charge = sum psi*;
    E_amp = sqrt((1/L) int E^2) = sqrt(2 W / L);
    E1 = (1/Ng) sum_e E_e exp(-2 pi i e / Ng).
    """
    P = np.asarray(P, dtype=np.float64)
    qs = np.asarray(qs, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    E = fld["E"] if self_field else np.zeros_like(fld["E"])
    ng = E.shape[0]
    K = float(np.sum(0.5 * psi * P * P + qs * P))
    W = float(fld["W"]) if self_field else 0.0
    U = external_energy(Q, ps, psi, L, ext) if ext is not None else 0.0
    e1 = np.sum(E * np.exp(-2j * np.pi * np.arange(ng) / ng)) / ng
    return {
        "K": K, "W": W, "U": U, "H": K + U + W,
        "charge": float(np.sum(psi)),
        "momentum": float(np.sum(psi * P + qs)),
        "e_amp": float(np.sqrt(2.0 * W / L)),
        "e1_re": float(e1.real), "e1_im": float(e1.imag),
    }


def sort_perm(cells, chunk: int):
    """Chunked stable sort permutation: within each chunk of `chunk` particles, order by
    cell index, ties kept in original order.  perm[k] is the source index of slot k."""
    cells = np.asarray(cells)
    n = cells.shape[0]
    out = np.empty(n, dtype=np.int64)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        out[c0:c1] = c0 + np.argsort(cells[c0:c1], kind="stable")
    return out


def step(state, fld, L: float, ng: int, dt: float, ext=None, self_field: bool = True):
    """One kick(dt/2) - drift(dt) - [deposit, solve] - kick(dt/2) step."""
    Q, P, qs, ps, psi = state
    proj = fld.get("projection", "elem")
    P, qs = kick(Q, P, qs, ps, fld["E"], fld["g"], L, 0.5 * dt, proj, ext, self_field)
    Q, ps = drift(Q, P, qs, ps, L, dt)
    fld = solve_field(Q, ps, psi, L, ng, proj)
    P, qs = kick(Q, P, qs, ps, fld["E"], fld["g"], L, 0.5 * dt, proj, ext, self_field)
    return (Q, P, qs, ps, psi), fld


def run(Q, P, qs, ps, psi, L: float, ng: int, dt: float, nsteps: int, record=True,
        projection: str = "elem", ext=None, self_field: bool = True):
    """Run nsteps KDK steps from the given state.  Returns (state, field, history),
    where history is a list of diagnostics dicts at t = 0, dt, ..., nsteps dt.
    ext = {"amp": A, "mode": m} adds the potential A (1 - cos(2 pi m q / L));
    self_field=False drops the particles' own field (charge e = 0)."""
    state = tuple(np.asarray(a, dtype=np.float64).copy() for a in (Q, P, qs, ps, psi))
    fld = solve_field(state[0], state[3], state[4], L, ng, projection)

    def diag(st):
        return diagnostics(st[1], st[2], st[4], fld, L, st[0], st[3], ext, self_field)
    hist = [diag(state)] if record else []
    for _ in range(nsteps):
        state, fld = step(state, fld, L, ng, dt, ext, self_field)
        if record:
            hist.append(diag(state))
    return state, fld, hist


# ---------------------------------------------------------------- P2 elements
# Degree-2 Lagrange elements on the same uniform periodic mesh (the paper's finite elements
# of degree k, here k = 2): on element e, local coordinate s in [0, 1), the three basis
# functions are N0 = (1 - s)(1 - 2s) at vertex e, N1 = 4 s (1 - s) at the midpoint and
# N2 = s (2s - 1) at vertex e+1.  Unknowns: Ng vertex values and Ng midpoint values.
# Everything below follows the definitions: the load vector of eq. rhs-assembly against
# these functions, the stiffness matrix assembled element by element, a solve of the
# assembled system with the zero-mean gauge, the field -phi_h' read from the basis, and
# phi_h'' read from the basis too (it exists for P2, so no projection is needed).

def p2_basis(s):
    """(N0, N1, N2) and their s-derivatives at local coordinate s."""
    s = np.asarray(s, dtype=np.float64)
    N = ((1.0 - s) * (1.0 - 2.0 * s), 4.0 * s * (1.0 - s), s * (2.0 * s - 1.0))
    dN = (4.0 * s - 3.0, 4.0 - 8.0 * s, 4.0 * s - 1.0)
    return N, dN


def deposit_p2(Q, ps, psi, L: float, ng: int):
    """P2 load vector: b_k = sum_a psi*_a phi_k(Q_a) - p*_a phi_k'(Q_a); returns (vertex
    loads, midpoint loads), Ng each."""
    ps = np.asarray(ps, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    i, s = cell_index(Q, L, ng)
    ih = inv_h(L, ng)
    N, dN = p2_basis(s)
    bv = np.bincount(i, weights=psi * N[0] - ps * (dN[0] * ih), minlength=ng)
    bv = bv + np.bincount((i + 1) % ng, weights=psi * N[2] - ps * (dN[2] * ih), minlength=ng)
    bm = np.bincount(i, weights=psi * N[1] - ps * (dN[1] * ih), minlength=ng)
    return bv, bm


def p2_node_weights(L: float, ng: int):
    """Integrals of the basis functions: h/3 for a vertex function, 2h/3 for a midpoint."""
    h = float(L) / ng
    return h / 3.0, 2.0 * h / 3.0


def neutralize_p2(bv, bm, L: float, ng: int):
    """Subtract the uniform background n0 = sum(b) / L against each basis function."""
    wv, wm = p2_node_weights(L, ng)
    n0 = (np.sum(bv) + np.sum(bm)) / float(L)
    return np.asarray(bv) - n0 * wv, np.asarray(bm) - n0 * wm


def _p2_assembled(ng: int):
    """3h times the assembled periodic P2 stiffness matrix over the unknowns ordered
    (v_0, m_0, v_1, m_1, ...): the element matrices [[7, -8, 1], [-8, 16, -8], [1, -8, 7]]
    added element by element.  Its entries are small integers, exact in any float type."""
    n = 2 * ng
    K = np.array([[7.0, -8.0, 1.0], [-8.0, 16.0, -8.0], [1.0, -8.0, 7.0]])
    A = np.zeros((n, n))
    for e in range(ng):
        idx = (2 * e, 2 * e + 1, (2 * e + 2) % n)
        for a in range(3):
            for b in range(3):
                A[idx[a], idx[b]] += K[a, b]
    return A


def p2_stiffness(L: float, ng: int):
    """Assembled periodic P2 stiffness matrix over the unknowns ordered
    (v_0, m_0, v_1, m_1, ...): element matrix (1/3h) [[7, -8, 1], [-8, 16, -8], [1, -8, 7]]."""
    h = float(L) / ng
    return _p2_assembled(ng) / (3.0 * h)


_P2_SYSTEMS = {}


def _p2_bordered(ng: int):
    """The bordered matrix [[3h A, c], [c^T, 0]] of the P2 system with the integral gauge,
    c = the basis functions' integrals in units of h/3 (1 at a vertex, 2 at a midpoint): all
    entries integers, so the float64 and extended-precision copies are the exact matrix
    (cached per mesh size)."""
    if ng not in _P2_SYSTEMS:
        c = np.tile([1.0, 2.0], ng)
        B = np.zeros((2 * ng + 1, 2 * ng + 1))
        B[:2 * ng, :2 * ng] = _p2_assembled(ng)
        B[:2 * ng, 2 * ng] = c
        B[2 * ng, :2 * ng] = c
        _P2_SYSTEMS[ng] = (B, B.astype(np.longdouble))
    return _P2_SYSTEMS[ng]


def poisson_solve_p2(btv, btm, L: float, refine: int = 3):
    """A Phi = b~ with the gauge integral(phi_h) = 0 (sum_k w_k Phi_k = 0), as the bordered
    system [[3h A, c], [c^T, 0]] [Phi; mu] = [3h b~; 0] whose matrix has integer entries
    (_p2_bordered).  Gaussian elimination with partial pivoting (np.linalg.solve), then
    `refine` steps of iterative refinement whose residuals are formed in extended precision
    (np.longdouble; Wilkinson's mixed-precision refinement).  The condition number grows like
    Ng^2; since the matrix is exact, refinement brings Phi to the rounding of the extended
    type, and phi_h'' read from second differences of Phi keeps its float64 digits.
    Returns (vertex, midpoint) Phi in extended precision."""
    btv = np.asarray(btv, dtype=np.float64)
    ng = btv.shape[0]
    B, Bx = _p2_bordered(ng)
    h3 = np.longdouble(3.0) * (np.longdouble(L) / np.longdouble(ng))
    rhs = np.zeros(2 * ng + 1, dtype=np.longdouble)
    rhs[0:2 * ng:2] = btv.astype(np.longdouble) * h3
    rhs[1:2 * ng:2] = np.asarray(btm, dtype=np.float64).astype(np.longdouble) * h3
    x = np.linalg.solve(B, rhs.astype(np.float64)).astype(np.longdouble)
    for _ in range(refine):
        r = rhs - Bx @ x
        x = x + np.linalg.solve(B, r.astype(np.float64)).astype(np.longdouble)
    return x[0:2 * ng:2], x[1:2 * ng:2]


def field_p2(Phv, Phm, L: float, average: bool = False):
    """On element e: E(s) = -phi_h'(s) = E0_e + s E1_e from the basis derivatives, and
    phi_h'' = g_e (constant on the element); with average=True the element average
    E0 + E1 / 2 alone.  Evaluated in the precision of Phi (extended for the output of
    poisson_solve_p2), returned in float64."""
    Phv = np.asarray(Phv)
    Phm = np.asarray(Phm)
    if Phv.dtype != np.longdouble:
        Phv = Phv.astype(np.float64)
        Phm = Phm.astype(np.float64)
    ng = Phv.shape[0]
    ih = Phv.dtype.type(ng) / Phv.dtype.type(L)
    Pn = np.roll(Phv, -1)
    # -phi' = -(Phi_e N0'(s) + Phi_m N1'(s) + Phi_{e+1} N2'(s)) / h
    E0 = -(-3.0 * Phv + 4.0 * Phm - 1.0 * Pn) * ih
    E1 = -(4.0 * Phv - 8.0 * Phm + 4.0 * Pn) * ih
    g = (4.0 * Phv - 8.0 * Phm + 4.0 * Pn) * ih * ih
    if average:
        return (E0 + 0.5 * E1).astype(np.float64)
    return E0.astype(np.float64), E1.astype(np.float64), g.astype(np.float64)


def solve_field_p2(Q, ps, psi, L: float, ng: int):
    """P2 counterpart of solve_field: dict with bv, bm (loads), btv, btm, Phv, Phm, E0, E1,
    g, the element-average field E (= E0 + E1 / 2) and W = (1/2) Phi^T A Phi."""
    bv, bm = deposit_p2(Q, ps, psi, L, ng)
    return field_from_load_p2(bv, bm, L, ng)


def field_from_load_p2(bv, bm, L: float, ng: int):
    """The steps of solve_field_p2 after the deposit: neutralise, solve, read the field."""
    btv, btm = neutralize_p2(bv, bm, L, ng)
    Phv, Phm = poisson_solve_p2(btv, btm, L)
    E0, E1, g = field_p2(Phv, Phm, L)
    # the element average of E (its value at the midpoint), from the extended-precision Phi
    Eavg = field_p2(Phv, Phm, L, average=True)
    phi = np.empty(2 * ng, dtype=np.longdouble)
    phi[0::2] = Phv
    phi[1::2] = Phm
    h3 = np.longdouble(3.0) * (np.longdouble(L) / np.longdouble(ng))
    W = float(0.5 * (phi @ (_p2_bordered(ng)[1][:2 * ng, :2 * ng] @ phi)) / h3)
    return {"bv": bv, "bm": bm, "btv": btv, "btm": btm, "Phv": Phv.astype(np.float64),
            "Phm": Phm.astype(np.float64), "E0": E0, "E1": E1, "g": g, "E": Eavg,
            "W": W, "order": 2}


def kick_p2(Q, P, qs, ps, fld, L: float, tau: float, ext=None, self_field: bool = True):
    """Exact flow of the field part with the P2 field: E(Q) from the basis, phi_h''(Q);
    without the self field these are zero, and a prescribed potential adds its own (as in
    kick)."""
    ng = fld["E0"].shape[0]
    i, s = cell_index(Q, L, ng)
    Ea = fld["E0"][i] + s * fld["E1"][i]
    ga = fld["g"][i]
    if not self_field:
        Ea = np.zeros_like(Ea)
        ga = np.zeros_like(ga)
    if ext is not None:
        ee, ge = external_field(Q, L, ext)
        Ea = Ea + ee
        ga = ga + ge
    return kick_values(P, qs, ps, Ea, ga, tau)


def step_p2(state, fld, L: float, ng: int, dt: float, ext=None, self_field: bool = True):
    """One KDK step with P2 elements (as step(): half-kick, drift, solve, half-kick)."""
    Q, P, qs, ps, psi = state
    P, qs = kick_p2(Q, P, qs, ps, fld, L, 0.5 * dt, ext, self_field)
    Q, ps = drift(Q, P, qs, ps, L, dt)
    fld = solve_field_p2(Q, ps, psi, L, ng)
    P, qs = kick_p2(Q, P, qs, ps, fld, L, 0.5 * dt, ext, self_field)
    return (Q, P, qs, ps, psi), fld


def run_p2(Q, P, qs, ps, psi, L: float, ng: int, dt: float, nsteps: int, ext=None,
           self_field: bool = True):
    """KDK run with P2 elements; history as run() (E1 and E_amp from the element-average
    field and W); ext and self_field as in run()."""
    state = tuple(np.asarray(a, dtype=np.float64).copy() for a in (Q, P, qs, ps, psi))
    fld = solve_field_p2(state[0], state[3], state[4], L, ng)

    def diag(st):
        return diagnostics(st[1], st[2], st[4], fld, L, st[0], st[3], ext, self_field)
    hist = [diag(state)]
    for _ in range(nsteps):
        state, fld = step_p2(state, fld, L, ng, dt, ext, self_field)
        hist.append(diag(state))
    return state, fld, hist
