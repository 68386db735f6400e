"""Plain FP64 CPU oracle for the decorated-particle initialisation (the paper's Algorithm 1,
"Decorated Particle Initialization", with the periodic moments of its torus subsection).

TEST INFRASTRUCTURE ONLY, like the rest of this package: imported by the tests, never by
the product path.  NumPy only; shares no code with the HIP library.

What is computed (readings where the paper leaves a choice are marked):
  * k-means in the phase-space coordinates (q, p) of the markers, by Lloyd's iteration:
    assign every marker to its nearest centre (Euclidean distance in (q, p), not wrapped
    in q: the paper clusters plain phase-space coordinates), ties to the lowest centre
    index; move every centre to the weighted mean of its markers (reading: the marker
    weights psi-bar are the k-means sample weights); a centre with no markers stays.
    The starting centres are given markers (their indices are an input), and a fixed
    number of iterations is run, followed by a final assignment.
  * per non-empty cluster S_a, in cluster order:
      psi*_a = sum of the weights (eq. psi-star);
      Z_a = weighted mean of the members;
      A0 = the member nearest Z_a (ties to the lowest marker index); (Q_a, P_a) = its
      coordinates;
      p*_a = sum_A psi_A (L / 2 pi) sin(2 pi (Q_a - Q_A) / L)  (periodic c);
      q*_a = -sum_A psi_A (P_a - P_A)                             (eq. moment-def).
Every sum runs over the members in increasing marker index (np.bincount adds in input
order), so a GPU implementation that sums in the same order agrees bit for bit except
where it evaluates sin.

The paper allows MiniBatch k-means in place of Lloyd's iteration for large runs.  The
variant here is the weighted, batched form of Sculley's mini-batch k-means ("Web-scale
k-means clustering", WWW 2010): per batch of markers (indices given as input; the random
draw is the caller's), assign each to its nearest current centre, then move every centre
that received members to the weighted mean of all the batch members it has ever received,
its previous value standing in for the earlier ones:
    v_c <- v_c + W_c,   centre_c <- (centre_c v_c(old) + S_c) / v_c(new),
with W_c, S_c the weight and the weighted coordinate sums of its members in this batch
(batch order).  No reassignment of starved centres and no stopping test (readings).
"""
from __future__ import annotations

import numpy as np

__all__ = ["nearest_centre", "lloyd", "cluster_moments", "cluster_markers", "kmeans_objective",
           "minibatch", "cluster_markers_minibatch"]


def nearest_centre(q, p, cq, cp, chunk: int = 2048):
    """Index of the nearest centre of every marker: argmin over centres of
    (q - cq)^2 + (p - cp)^2, first (lowest) index on ties.  Brute force, in chunks."""
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    cq = np.asarray(cq, dtype=np.float64)
    cp = np.asarray(cp, dtype=np.float64)
    out = np.empty(q.shape[0], dtype=np.int64)
    for s in range(0, q.shape[0], chunk):
        dq = q[s:s + chunk, None] - cq[None, :]
        dp = p[s:s + chunk, None] - cp[None, :]
        out[s:s + chunk] = np.argmin(dq * dq + dp * dp, axis=1)
    return out


def kmeans_objective(q, p, w, cq, cp, assign):
    """Weighted within-cluster sum of squares, the quantity Lloyd's iteration lowers."""
    a = np.asarray(assign)
    dq = np.asarray(q) - np.asarray(cq)[a]
    dp = np.asarray(p) - np.asarray(cp)[a]
    return float(np.sum(np.asarray(w) * (dq * dq + dp * dp)))


def lloyd(q, p, w, init_idx, iters: int):
    """Centres after `iters` Lloyd iterations from the markers init_idx, and the final
    assignment to them."""
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    init_idx = np.asarray(init_idx)
    k = init_idx.shape[0]
    cq = q[init_idx].copy()
    cp = p[init_idx].copy()
    for _ in range(iters):
        a = nearest_centre(q, p, cq, cp)
        cnt = np.bincount(a, minlength=k)
        W = np.bincount(a, weights=w, minlength=k)
        SQ = np.bincount(a, weights=w * q, minlength=k)
        SP = np.bincount(a, weights=w * p, minlength=k)
        live = cnt > 0
        cq[live] = SQ[live] / W[live]
        cp[live] = SP[live] / W[live]
    return cq, cp, nearest_centre(q, p, cq, cp)


def cluster_moments(q, p, w, assign, k: int, L: float):
    """Algorithm 1's decorated particle of every non-empty cluster, in cluster order:
    dict of Q, P, qs, ps, psi arrays (and `cluster`, the cluster index of each)."""
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    a = np.asarray(assign)
    cnt = np.bincount(a, minlength=k)
    W = np.bincount(a, weights=w, minlength=k)
    zq = np.bincount(a, weights=w * q, minlength=k)
    zp = np.bincount(a, weights=w * p, minlength=k)
    live = np.nonzero(cnt > 0)[0]
    zq = zq[live] / W[live]
    zp = zp[live] / W[live]
    Qa = np.empty(live.shape[0])
    Pa = np.empty(live.shape[0])
    members = np.argsort(a, kind="stable")          # markers grouped by cluster, index order
    starts = np.concatenate(([0], np.cumsum(cnt)))
    for j, c in enumerate(live):
        m = members[starts[c]:starts[c + 1]]
        d2 = (q[m] - zq[j]) * (q[m] - zq[j]) + (p[m] - zp[j]) * (p[m] - zp[j])
        a0 = m[np.argmin(d2)]
        Qa[j] = q[a0]
        Pa[j] = p[a0]
    slot = np.full(k, -1)
    slot[live] = np.arange(live.shape[0])
    s = slot[a]
    two_pi = 2.0 * np.pi
    c_term = w * ((L / two_pi) * np.sin(two_pi * (Qa[s] - q) / L))
    ps = np.bincount(s, weights=c_term, minlength=live.shape[0])
    qs = -np.bincount(s, weights=w * (Pa[s] - p), minlength=live.shape[0])
    return {"Q": Qa, "P": Pa, "qs": qs, "ps": ps, "psi": W[live], "cluster": live}


def cluster_markers(q, p, w, init_idx, iters: int, L: float):
    """Algorithm 1: k-means of the markers, then the decorated particle of each cluster.
    Returns (decorated state dict, final assignment)."""
    cq, cp, a = lloyd(q, p, w, init_idx, iters)
    return cluster_moments(q, p, w, a, np.asarray(init_idx).shape[0], L), a


def minibatch(q, p, w, init_idx, batches, record: bool = False):
    """Mini-batch k-means from the markers init_idx, one update per batch (each batch an
    array of marker indices; a repeated index counts once per occurrence).  Returns the
    centres and the weight v each has absorbed, and with record=True also the assignment
    of every batch (a list of arrays)."""
    q = np.asarray(q, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    init_idx = np.asarray(init_idx)
    k = init_idx.shape[0]
    cq = q[init_idx].copy()
    cp = p[init_idx].copy()
    v = np.zeros(k)
    seen = []
    for B in batches:
        B = np.asarray(B)
        qb, pb, wb = q[B], p[B], w[B]
        a = nearest_centre(qb, pb, cq, cp)
        cnt = np.bincount(a, minlength=k)
        W = np.bincount(a, weights=wb, minlength=k)
        SQ = np.bincount(a, weights=wb * qb, minlength=k)
        SP = np.bincount(a, weights=wb * pb, minlength=k)
        live = cnt > 0
        vn = v[live] + W[live]
        cq[live] = (cq[live] * v[live] + SQ[live]) / vn
        cp[live] = (cp[live] * v[live] + SP[live]) / vn
        v[live] = vn
        if record:
            seen.append(a)
    return (cq, cp, v, seen) if record else (cq, cp, v)


def cluster_markers_minibatch(q, p, w, init_idx, batches, L: float):
    """Algorithm 1 with mini-batch k-means: the centres after the batches, a final
    assignment of every marker to them, then the decorated particle of each cluster.
    Returns (decorated state dict, final assignment, absorbed weights v)."""
    cq, cp, v = minibatch(q, p, w, init_idx, batches)
    a = nearest_centre(q, p, cq, cp)
    return cluster_moments(q, p, w, a, np.asarray(init_idx).shape[0], L), a, v
