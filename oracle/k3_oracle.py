"""Plain FP64 CPU oracle for decorated particles with second moments (k = 3).

TEST INFRASTRUCTURE ONLY, like the rest of this package: imported by the tests, never by
the HIP product path.  NumPy only; the P2 finite-element pieces come from vp_oracle.

The paper's ansatz (eq. sw_f_ansatz) adds, for k > 2, the centred moments
M_l (2 <= l <= k-1) of each particle as (-1)^l / l! M_l^{mu...} d^l delta_Z, and gives their
Poisson bracket as the Lie-Poisson bracket of the quotient algebra s_k = s / I_k (Section
"Scovel-Weinstein enhancement of PIC"); it does not write the resulting equations out.  For
k = 3 in 1D1V, s_3 is the space of quadratic phase-space polynomials, closed under the
canonical bracket, and a particle carries M = (Mqq, Mqp, Mpp), a symmetric 2 x 2 matrix, in
the ansatz term (1/2)(Mqq d_q^2 + 2 Mqp d_q d_p + Mpp d_p^2) delta_Z.  Written out (the
derivation is in the design notes of this repository):

  * pairing: <M, s> = (1/2) tr(M S) for s(z) = (1/2) z^T S z;
  * Hamiltonian: H = sum_a [psi* P^2/2 + q* P + Mpp/2] + (field energy), where the load of
    eq. rhs-assembly gains (1/2) Mqq phi_j''(Q), and a prescribed potential V adds
    psi* V(Q) - p* V'(Q) + (1/2) Mqq V''(Q);
  * dH/dM is the quadratic s_H with S_H = Hess h(Z) = diag(phi''(Q), 1) (h = p^2/2 + phi),
    and the Lie-Poisson bracket with the canonical bracket of the paper's eq. for
    {h1, h2}_can gives
        dMqq/dt = 2 Mqp,   dMqp/dt = Mpp - phi'' Mqq,   dMpp/dt = -2 phi'' Mqp,
    the covariance equations of the linearised flow (M -> A M A^T);
  * the (Q, P, q*, p*) equations of eq. sw-evolution are unchanged except
        dq*/dt = p* phi''(Q) - (1/2) Mqq phi'''(Q),
    where phi''' vanishes inside every element for P1 and P2 potentials (only a prescribed
    potential contributes it).

Splitting (as for k = 2, each sub-flow exact with its frozen variables):
  kick  (field part; Q, p*, Mqq frozen):  P += tau E, q* += tau (p* g - Mqq V'''/2),
        Mqp -= tau g Mqq, Mpp += -2 tau g Mqp + tau^2 g^2 Mqq     (M -> A M A^T, A = [[1, 0],
        [-tau g, 1]]);
  drift (kinetic part; P, q*, Mpp frozen): Q += tau P, p* -= tau q*,
        Mqq += 2 tau Mqp + tau^2 Mpp, Mqp += tau Mpp              (A = [[1, tau], [0, 1]]).
Both are congruences by unimodular matrices, so det M = Mqq Mpp - Mqp^2 (the Casimir of
the Lie-Poisson bracket on s_3*) is kept by every step.

Readings (where the paper is silent):
  * the potential is P2 (element_order 2): phi_h'' then exists on each element and the
    load term (1/2) Mqq phi_j''(Q) is a function; with P1 it would be point masses at the
    nodes, which no projection turns into a consistent Hamiltonian;
  * initial second moments of a cluster on the torus (cluster_moments_k3): centred about the
    central marker, with the periodic squared distance (L/pi)^2 sin^2(pi (Q - x)/L) for qq and
    the periodic displacement (L/2pi) sin(2pi (Q - x)/L) of the first moment in qp.

parity unpinned: the torus form of the initial second moments (second bullet above); every
function here is pinned by tests/test_oracle_k3_pins.py.
"""
from __future__ import annotations

import math

import numpy as np

from . import vp_oracle as V

__all__ = ["deposit_p2_k3", "solve_field_p2_k3", "kick_k3", "drift_k3", "diagnostics_k3",
           "step_k3", "run_k3", "cluster_moments_k3", "K3_FIELDS"]

K3_FIELDS = ("Q", "P", "qs", "ps", "psi", "Mqq", "Mqp", "Mpp")


def deposit_p2_k3(Q, ps, psi, Mqq, L: float, ng: int):
    """P2 load with the second-moment term: b_k = sum_a psi*_a phi_k(Q_a) - p*_a phi_k'(Q_a)
    + (1/2) Mqq_a phi_k''(Q_a).  On an element the basis' second derivatives are 4, -8, 4
    (left vertex, midpoint, right vertex) over h^2.  Returns (vertex loads, midpoint loads)."""
    bv, bm = V.deposit_p2(Q, ps, psi, L, ng)
    Mqq = np.asarray(Mqq, dtype=np.float64)
    i, _ = V.cell_index(Q, L, ng)
    ih = V.inv_h(L, ng)
    c = 0.5 * Mqq * (ih * ih)
    bv = bv + np.bincount(i, weights=4.0 * c, minlength=ng)
    bv = bv + np.bincount((i + 1) % ng, weights=4.0 * c, minlength=ng)
    bm = bm + np.bincount(i, weights=-8.0 * c, minlength=ng)
    return bv, bm


def solve_field_p2_k3(Q, ps, psi, Mqq, L: float, ng: int):
    """The P2 field (as vp_oracle.solve_field_p2) of the load with second moments."""
    bv, bm = deposit_p2_k3(Q, ps, psi, Mqq, L, ng)
    return V.field_from_load_p2(bv, bm, L, ng)


def _ext_third(Q, L: float, ext):
    """V'''(Q) of the prescribed potential V = A (1 - cos(kappa q)), kappa = 2 pi m / L."""
    kap = 2.0 * math.pi * float(ext["mode"]) / L
    return -float(ext["amp"]) * kap ** 3 * np.sin(kap * np.asarray(Q, dtype=np.float64))


def _fields_at(Q, fld, L: float, ext, self_field: bool):
    """E, phi'' and phi''' at the particles: the P2 self field (E linear and phi''
    constant on each element, phi''' zero) plus a prescribed potential's."""
    ng = fld["E0"].shape[0]
    i, s = V.cell_index(Q, L, ng)
    if self_field:
        Ea = fld["E0"][i] + s * fld["E1"][i]
        ga = fld["g"][i]
    else:
        Ea = np.zeros(np.shape(Q))
        ga = np.zeros(np.shape(Q))
    g3 = np.zeros(np.shape(Q))
    if ext is not None:
        ee, ge = V.external_field(Q, L, ext)
        Ea = Ea + ee
        ga = ga + ge
        g3 = _ext_third(Q, L, ext)
    return Ea, ga, g3


def kick_k3(state, fld, L: float, tau: float, ext=None, self_field: bool = True):
    """Exact flow of the field part for time tau (Q, p*, Mqq frozen)."""
    Q, P, qs, ps, psi, Mqq, Mqp, Mpp = state
    Ea, ga, g3 = _fields_at(Q, fld, L, ext, self_field)
    P = P + tau * Ea
    # the k = 2 kick's terms in its operation order, then the moments' mean-force term
    qs = qs + tau * ps * ga - (0.5 * tau) * Mqq * g3
    Mpp = Mpp - 2.0 * tau * ga * Mqp + (tau * ga) * (tau * ga) * Mqq
    Mqp = Mqp - tau * ga * Mqq
    return (Q, P, qs, ps, psi, Mqq, Mqp, Mpp)


def drift_k3(state, L: float, tau: float):
    """Exact flow of the kinetic part for time tau (P, q*, Mpp frozen)."""
    Q, P, qs, ps, psi, Mqq, Mqp, Mpp = state
    Q, ps = V.drift(Q, P, qs, ps, L, tau)
    Mqq = Mqq + 2.0 * tau * Mqp + tau * tau * Mpp
    Mqp = Mqp + tau * Mpp
    return (Q, P, qs, ps, psi, Mqq, Mqp, Mpp)


def diagnostics_k3(state, fld, L: float, ext=None, self_field: bool = True):
    """K = sum psi* P^2/2 + q* P + Mpp/2; W; U = prescribed potential's energy, with
    (1/2) Mqq V''(Q); H = K + U + W; charge; momentum sum(psi* P + q*) (the second moments
    carry none); casimir = sum of det M."""
    Q, P, qs, ps, psi, Mqq, Mqp, Mpp = state
    K = float(np.sum(0.5 * psi * P * P + qs * P + 0.5 * Mpp))
    W = float(fld["W"]) if self_field else 0.0
    U = 0.0
    if ext is not None:
        _, ge = V.external_field(Q, L, ext)
        U = V.external_energy(Q, ps, psi, L, ext) + float(np.sum(0.5 * Mqq * ge))
    return {"K": K, "W": W, "U": U, "H": K + U + W, "charge": float(np.sum(psi)),
            "momentum": float(np.sum(psi * P + qs)),
            "casimir": float(np.sum(Mqq * Mpp - Mqp * Mqp))}


def step_k3(state, fld, L: float, ng: int, dt: float, ext=None, self_field: bool = True):
    """One kick(dt/2) - drift(dt) - [deposit, solve] - kick(dt/2) step."""
    state = kick_k3(state, fld, L, 0.5 * dt, ext, self_field)
    state = drift_k3(state, L, dt)
    fld = solve_field_p2_k3(state[0], state[3], state[4], state[5], L, ng)
    state = kick_k3(state, fld, L, 0.5 * dt, ext, self_field)
    return state, fld


def run_k3(state: dict, L: float, ng: int, dt: float, nsteps: int, ext=None,
           self_field: bool = True):
    """Run nsteps steps from a state dict with the K3_FIELDS; returns (state tuple, field,
    history of diagnostics at t = 0, dt, ..., nsteps dt)."""
    st = tuple(np.asarray(state[k], dtype=np.float64).copy() for k in K3_FIELDS)
    fld = solve_field_p2_k3(st[0], st[3], st[4], st[5], L, ng)
    hist = [diagnostics_k3(st, fld, L, ext, self_field)]
    for _ in range(nsteps):
        st, fld = step_k3(st, fld, L, ng, dt, ext, self_field)
        hist.append(diagnostics_k3(st, fld, L, ext, self_field))
    return st, fld, hist


def cluster_moments_k3(q, p, w, assign, k: int, L: float):
    """Algorithm 1's decorated particle of every non-empty cluster (as
    cluster_oracle.cluster_moments), with its centred second moments about the central
    marker: Mqq = sum w (L/pi)^2 sin^2(pi (Q - x)/L), Mqp = sum w c (P - v) with the first
    moment's periodic displacement c = (L/2pi) sin(2pi (Q - x)/L), Mpp = sum w (P - v)^2."""
    from .cluster_oracle import cluster_moments
    dec = cluster_moments(q, p, w, assign, k, L)
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    a = np.asarray(assign)
    slot = np.full(k, -1)
    slot[dec["cluster"]] = np.arange(dec["cluster"].shape[0])
    s = slot[a]
    dq = (L / math.pi) * np.sin(math.pi * (dec["Q"][s] - q) / L)
    c = (L / (2.0 * math.pi)) * np.sin(2.0 * math.pi * (dec["Q"][s] - q) / L)
    dp = dec["P"][s] - p
    n = dec["cluster"].shape[0]
    dec["Mqq"] = np.bincount(s, weights=w * dq * dq, minlength=n)
    dec["Mqp"] = np.bincount(s, weights=w * c * dp, minlength=n)
    dec["Mpp"] = np.bincount(s, weights=w * dp * dp, minlength=n)
    return dec
