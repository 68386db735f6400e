"""Seeded synthetic initial states: decorated particles on a jittered phase-space lattice.

This module only produces inputs.  It holds none of the per-step arithmetic (deposit,
solve, push); both the HIP path and the CPU oracle receive the arrays it returns.

Recipe (the paper's initialisation, Section 4, with each lattice cell standing in for a
k-means cluster S_a):
  * the phase-space box [0, L) x [vmin, vmax) is cut into nx x nv cells of size dx x dv;
  * the "central particle" of a cell is a jittered point, deliberately not the cell mean
    (the paper explains that a centre at the mean would zero both dipoles):
        Q = x0 + (1/2 + jx xi) dx,  P = v0 + (1/2 + jv eta) dv,  xi, eta ~ U(-1/2, 1/2);
  * the marker sums of eq. psi-star and eq. moment-def become integrals of f0 over the
    cell, with the periodic moment function c(Q, x) = (L / 2 pi) sin(2 pi (Q - x) / L)
    of the torus initialisation (Section 4.2):
        psi* = int_C f0,
        p*   = int_C f0(x, v) c(Q, x),
        q*   = -int_C f0(x, v) (P - v);
  * integrals use 8-point Gauss-Legendre rules in x and in v; f0 is separable,
    f0(x, v) = X(x) V(v), for every workload here.
Particle order: by default a seeded random permutation of the cells (drawn after xi and
eta), like the arbitrary cluster order of a k-means initialisation, so that particles that
are neighbours in memory are not neighbours in phase space; order="lattice" keeps the
v-major order a = iv * nx + ix.  RNG: NumPy PCG64 seeded from SeedSequence(seed); xi is
drawn first as an (nv, nx) array, then eta, then the permutation.
"""
from __future__ import annotations

import math

import numpy as np

_GL_T, _GL_W = np.polynomial.legendre.leggauss(8)


def _gl_nodes(lo, width):
    """Nodes (cells x 8) and weights (cells x 8) of the 8-point rule on [lo, lo + width)."""
    lo = np.asarray(lo, dtype=np.float64)[:, None]
    x = lo + 0.5 * width * (1.0 + _GL_T[None, :])
    w = np.broadcast_to(0.5 * width * _GL_W[None, :], x.shape)
    return x, w


def landau_profile(alpha: float, k: float):
    """f0 = (1 + alpha cos kx) exp(-v^2/2) / sqrt(2 pi)."""
    X = lambda x: 1.0 + alpha * np.cos(k * x)  # noqa: E731
    V = lambda v: np.exp(-0.5 * v * v) / math.sqrt(2.0 * math.pi)  # noqa: E731
    return X, V


def two_stream_profile(alpha: float, k: float, v0: float, T: float = 1.0):
    """f0 = (1 + alpha cos kx) [exp(-(v-v0)^2/2T) + exp(-(v+v0)^2/2T)] / (2 sqrt(2 pi T))."""
    X = lambda x: 1.0 + alpha * np.cos(k * x)  # noqa: E731
    c = 1.0 / (2.0 * math.sqrt(2.0 * math.pi * T))

    def V(v):
        return c * (np.exp(-0.5 * (v - v0) ** 2 / T) + np.exp(-0.5 * (v + v0) ** 2 / T))
    return X, V


def bump_on_tail_profile(alpha: float = 0.04, k: float = 0.3):
    """f0 = (0.9 exp(-v^2/2) + 0.2 exp(-2 (v - 4.5)^2)) / sqrt(2 pi) (1 + alpha cos kx)."""
    X = lambda x: 1.0 + alpha * np.cos(k * x)  # noqa: E731

    def V(v):
        return (0.9 * np.exp(-0.5 * v * v) + 0.2 * np.exp(-2.0 * (v - 4.5) ** 2)) / math.sqrt(2.0 * math.pi)
    return X, V


def make_lattice(L: float, nx: int, nv: int, vmin: float, vmax: float, profile,
                 seed: int = 0, jx: float = 1.0, jv: float = 1.0, rng=None,
                 order: str = "random", moments: bool = False):
    """Return dict(Q, P, qs, ps, psi) of float64 arrays with nx*nv decorated particles.
    With moments=True also the centred second moments of each cell about its centre (the
    k = 3 particle): Mqq = int_C f0 (L/pi)^2 sin^2(pi (Q - x)/L), Mqp = int_C f0 c (P - v)
    with the first moment's periodic displacement c, Mpp = int_C f0 (P - v)^2."""
    X, V = profile
    dx = float(L) / nx
    dv = (float(vmax) - float(vmin)) / nv
    if rng is None:
        rng = np.random.default_rng(np.random.SeedSequence(seed))
    xi = rng.uniform(-0.5, 0.5, size=(nv, nx))
    eta = rng.uniform(-0.5, 0.5, size=(nv, nx))
    if order not in ("random", "lattice"):
        raise ValueError(f"unknown particle order {order!r}")
    perm = rng.permutation(nx * nv) if order == "random" else None

    x0 = np.arange(nx, dtype=np.float64) * dx
    v0 = float(vmin) + np.arange(nv, dtype=np.float64) * dv
    Q = x0[None, :] + (0.5 + jx * xi) * dx
    P = v0[:, None] + (0.5 + jv * eta) * dv
    Q = np.where(Q < 0.0, Q + L, Q)
    Q = np.where(Q >= L, Q - L, Q)

    xn, xw = _gl_nodes(x0, dx)            # (nx, 8)
    vn, vw = _gl_nodes(v0, dv)            # (nv, 8)
    Xw = X(xn) * xw                       # X(x_k) w_k per x cell
    Vw = V(vn) * vw                       # V(v_k) w_k per v cell
    Ix0 = Xw.sum(axis=1)                  # int_cell X dx
    Iv0 = Vw.sum(axis=1)                  # int_cell V dv

    psi = Iv0[:, None] * Ix0[None, :]
    th = 2.0 * math.pi / L
    ps = np.empty_like(Q)
    qs = np.empty_like(Q)
    if moments:
        Mqq, Mqp, Mpp = np.empty_like(Q), np.empty_like(Q), np.empty_like(Q)
    rows = max(1, (1 << 21) // max(1, nx))      # bound the (rows, nx, 8) temporaries
    for r0 in range(0, nv, rows):
        r1 = min(nv, r0 + rows)
        # p* = Iv0 * int X(x) (L/2pi) sin(th (Q - x)) dx; Q varies per particle
        sx = np.sin(th * (Q[r0:r1, :, None] - xn[None, :, :]))
        ps[r0:r1] = Iv0[r0:r1, None] * (L / (2.0 * math.pi)) * np.sum(Xw[None, :, :] * sx, axis=2)
        # q* = -Ix0 * int V(v) (P - v) dv; P varies per particle
        dvp = P[r0:r1, :, None] - vn[r0:r1, None, :]
        qs[r0:r1] = -Ix0[None, :] * np.sum(Vw[r0:r1, None, :] * dvp, axis=2)
        if moments:
            dq2 = (L / math.pi) ** 2 * np.sin(0.5 * th * (Q[r0:r1, :, None] - xn[None, :, :])) ** 2
            Mqq[r0:r1] = Iv0[r0:r1, None] * np.sum(Xw[None, :, :] * dq2, axis=2)
            cx = (L / (2.0 * math.pi)) * np.sum(Xw[None, :, :] * sx, axis=2)
            Mqp[r0:r1] = cx * np.sum(Vw[r0:r1, None, :] * dvp, axis=2)
            Mpp[r0:r1] = Ix0[None, :] * np.sum(Vw[r0:r1, None, :] * dvp * dvp, axis=2)

    out = {"Q": Q, "P": P, "qs": qs, "ps": ps, "psi": psi}
    if moments:
        out.update(Mqq=Mqq, Mqp=Mqp, Mpp=Mpp)
    if perm is None:
        return {k: v.reshape(-1).copy() for k, v in out.items()}
    return {k: v.reshape(-1)[perm].copy() for k, v in out.items()}


def cast_state(state: dict, dtype):
    """Copy of a state dict with every array converted to dtype."""
    return {k: np.ascontiguousarray(v, dtype=dtype) for k, v in state.items()}
