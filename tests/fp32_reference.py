"""References for FP32-state runs: the oracle's sub-flows with the same float32 storage
points as a GPU path (every sub-step computes in float64 from the stored values and stores
float32 results).  Test helper; calls only the oracle.

Two paths store at different points:
  * the primitive path (gather_push(dt/2, dt), deposit, poisson, gather_push(dt/2, 0)) stores
    Q, P, q*, p* after the first half-kick and the drift, and P, q* again after the second
    half-kick;
  * the fused step keeps P and q* in float64 from the pending half-kick of one step through
    the first half-kick of the next, and stores Q, P, q*, p* once per step, after the drift.
"""
import numpy as np

import oracle as O


def _r32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def fp32_storage_reference(s64, w, nsteps):
    """The primitive path's storage points.  Returns (W history, (Q, P, q*, p*))."""
    Q, P, qs, ps, psi = (np.asarray(s64[k], dtype=np.float64).copy()
                         for k in ("Q", "P", "qs", "ps", "psi"))
    fld = O.solve_field(Q, ps, psi, w.L, w.ng)
    Ws = [fld["W"]]
    for _ in range(nsteps):
        P, qs = O.kick(Q, P, qs, ps, fld["E"], fld["g"], w.L, 0.5 * w.dt)
        Q, ps = O.drift(Q, P, qs, ps, w.L, w.dt)
        Q, P, qs, ps = _r32(Q), _r32(P), _r32(qs), _r32(ps)
        fld = O.solve_field(Q, ps, psi, w.L, w.ng)
        P, qs = O.kick(Q, P, qs, ps, fld["E"], fld["g"], w.L, 0.5 * w.dt)
        P, qs = _r32(P), _r32(qs)
        Ws.append(fld["W"])
    return np.array(Ws), (Q, P, qs, ps)


def _solve(Q, ps, psi, w, order):
    if order == 2:
        return O.solve_field_p2(Q, ps, psi, w.L, w.ng)
    return O.solve_field(Q, ps, psi, w.L, w.ng)


def _kick(Q, P, qs, ps, fld, w, order):
    if order == 2:
        return O.kick_p2(Q, P, qs, ps, fld, w.L, 0.5 * w.dt)
    return O.kick(Q, P, qs, ps, fld["E"], fld["g"], w.L, 0.5 * w.dt)


def fp32_fused_reference(s64, w, nsteps, order: int = 1):
    """The fused step's storage points (P1 elements, or P2 with order=2).  Step n computes,
    in float64 from the stored values: the half-kick still owed from step n-1 (none at n = 0)
    with the field of the stored positions, the half-kick of step n with the same field, and
    the drift; then it stores Q, P, q*, p* as float32.  The last step's owed half-kick is
    applied in float64 at the end (a read-back of the device state applies it the same way
    and stores float32).  Returns (W history, H history, (Q, P, q*, p*)); H at step n uses
    the unrounded P, q* after the owed half-kick, as the fused step's kinetic sums do."""
    Q, P, qs, ps, psi = (np.asarray(s64[k], dtype=np.float64).copy()
                         for k in ("Q", "P", "qs", "ps", "psi"))
    fld = _solve(Q, ps, psi, w, order)
    Ws, Hs = [], []
    for n in range(nsteps + 1):
        if n > 0:
            P, qs = _kick(Q, P, qs, ps, fld, w, order)
        Ws.append(fld["W"])
        Hs.append(O.diagnostics(P, qs, psi, fld, w.L)["H"])
        if n == nsteps:
            break
        P, qs = _kick(Q, P, qs, ps, fld, w, order)
        Q, ps = O.drift(Q, P, qs, ps, w.L, w.dt)
        Q, P, qs, ps = _r32(Q), _r32(P), _r32(qs), _r32(ps)
        fld = _solve(Q, ps, psi, w, order)
    P, qs = _r32(P), _r32(qs)
    return np.array(Ws), np.array(Hs), (Q, P, qs, ps)


def fp32_fused_reference_k3(s64, w, nsteps):
    """The fused step's storage points for particles with second moments (k = 3, P2
    elements): as fp32_fused_reference, with the moments rounded to float32 where the
    state is stored.  Returns (W history, H history, final state tuple of eight arrays)."""
    st = tuple(np.asarray(s64[k], dtype=np.float64).copy() for k in O.K3_FIELDS)
    fld = O.solve_field_p2_k3(st[0], st[3], st[4], st[5], w.L, w.ng)
    Ws, Hs = [], []
    for n in range(nsteps + 1):
        if n > 0:
            st = O.kick_k3(st, fld, w.L, 0.5 * w.dt)
        Ws.append(fld["W"])
        Hs.append(O.diagnostics_k3(st, fld, w.L)["H"])
        if n == nsteps:
            break
        st = O.kick_k3(st, fld, w.L, 0.5 * w.dt)
        st = O.drift_k3(st, w.L, w.dt)
        st = tuple(_r32(a) if k != 4 else a for k, a in enumerate(st))
        fld = O.solve_field_p2_k3(st[0], st[3], st[4], st[5], w.L, w.ng)
    st = tuple(_r32(a) if k in (1, 2, 6, 7) else a for k, a in enumerate(st))
    return np.array(Ws), np.array(Hs), st
