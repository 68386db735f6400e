"""Reference for FP32-state runs: the oracle's sub-flows with the same float32 storage
points as the GPU path (every sub-step computes in float64 from the stored values and stores
float32 results).  Test helper; calls only the oracle."""
import numpy as np

import oracle as O


def fp32_storage_reference(s64, w, nsteps):
    """The primitive path's arithmetic written with the oracle's sub-flows: every sub-step
    computes in float64 from the stored values and stores float32 results."""
    r32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    Q, P, qs, ps, psi = (s64[k].copy() for k in ("Q", "P", "qs", "ps", "psi"))
    fld = O.solve_field(Q, ps, psi, w.L, w.ng)
    Ws = [fld["W"]]
    for _ in range(nsteps):
        P, qs = O.kick(Q, P, qs, ps, fld["E"], fld["g"], w.L, 0.5 * w.dt)
        Q, ps = O.drift(Q, P, qs, ps, w.L, w.dt)
        Q, P, qs, ps = r32(Q), r32(P), r32(qs), r32(ps)
        fld = O.solve_field(Q, ps, psi, w.L, w.ng)
        P, qs = O.kick(Q, P, qs, ps, fld["E"], fld["g"], w.L, 0.5 * w.dt)
        P, qs = r32(P), r32(qs)
        Ws.append(fld["W"])
    return np.array(Ws), (Q, P, qs, ps)
