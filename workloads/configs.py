"""Named synthetic workloads (seeded), with the sizes used by the tests and the benchmark.

Each preset returns a `Workload` with the physical parameters and a `state(dtype)` method
that builds the initial decorated-particle arrays from `workloads.lattice`.

  landau_linear      Linear Landau damping: L = 4 pi (k = 0.5), alpha = 0.01, Ng = 64,
                     64 x 64 lattice (N = 4096) over v in [-6, 6], dt = 0.1, 200 steps, FP64.
  two_stream         Two-stream instability: L = 10 pi (k = 0.2), alpha = 1e-3, beams at
                     +-2.4 with T = 1, Ng = 512, 1024 x 1024 lattice (N = 2^20) over
                     v in [-8, 8], dt = 0.05, 1000 steps, FP32.
  landau_sweep       256 uneven Landau instances: alpha log-uniform [0.01, 0.5], k uniform
                     [0.3, 0.6], L = 2 pi / k, Ng in {64, 128, 256}, N0 log-uniform
                     [2^12, 2^16] -> lattice Ng x max(16, round(N0 / Ng)), v in [-6, 6],
                     dt = 0.1, 500 steps, FP32.
  landau_nonlinear   Strong Landau damping: alpha = 0.5, k = 0.5, Ng = 256,
                     2048 x 2048 lattice (N = 2^22), v in [-6, 6], dt = 0.05, 2000 steps.
  served_stream      Poisson arrivals of mixed Landau / two-stream / bump-on-tail jobs with
                     N log-uniform in [2^12, 2^20], Ng in {64 .. 1024}, horizons 100-2000.
  landau_strong      The paper's strong Landau damping case: L = 12, A = 0.5, k = 2 pi / L,
                     dt = 0.2, Ng = 128; with `random_markers`, the standard particle-in-cell
                     start of the same f0 (the particle-count study).

Particles are stored in a seeded random order (like the arbitrary cluster order of a
k-means initialisation); `order="lattice"` keeps the v-major lattice order.

Every preset jitters the central particle in x only (jx = 1, jv = 0).  Velocity jitter
makes q* = -(P - v_mean) psi* non-zero, and under free streaming the dipole offset p*/psi*
then grows like (P - v_mean) t; once it exceeds the mesh size the first-order (k = 2)
ansatz feeds grid-scale noise into phi_h'' and the shape variables run away.  With the
velocity centre at the cell midpoint, q* only carries the O(dv^2) skew of f0 inside the
cell and the runs stay well behaved over the stated horizons.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .lattice import (bump_on_tail_profile, landau_profile, make_lattice,
                      two_stream_profile, cast_state)


@dataclass
class Workload:
    name: str
    L: float
    ng: int
    nx: int
    nv: int
    vmin: float
    vmax: float
    dt: float
    nsteps: int
    kind: str                      # "landau" | "two_stream" | "bump_on_tail"
    params: dict = field(default_factory=dict)
    seed: int = 0
    jx: float = 1.0
    jv: float = 0.0                # centre velocity at the cell midpoint (see module doc)
    rng_seedseq: object = None     # optional SeedSequence overriding `seed`
    order: str = "random"          # particle order in memory: "random" or "lattice"

    @property
    def n(self) -> int:
        return self.nx * self.nv

    def profile(self):
        p = self.params
        if self.kind == "landau":
            return landau_profile(p["alpha"], p["k"])
        if self.kind == "two_stream":
            return two_stream_profile(p["alpha"], p["k"], p["v0"], p.get("T", 1.0))
        if self.kind == "bump_on_tail":
            return bump_on_tail_profile(p.get("alpha", 0.04), p.get("k", 0.3))
        raise ValueError(self.kind)

    def state(self, dtype=np.float64, moments: bool = False) -> dict:
        """The initial state; moments=True adds each cell's second moments (Mqq, Mqp, Mpp)
        for particles with moments of degree 2 (k = 3)."""
        rng = None
        if self.rng_seedseq is not None:
            rng = np.random.default_rng(self.rng_seedseq)
        st = make_lattice(self.L, self.nx, self.nv, self.vmin, self.vmax, self.profile(),
                          seed=self.seed, jx=self.jx, jv=self.jv, rng=rng, order=self.order,
                          moments=moments)
        return cast_state(st, dtype)


def landau_linear(seed: int = 0, nx: int = 64, nv: int = 64, ng: int = 64) -> Workload:
    k = 0.5
    return Workload("landau_linear", L=2 * math.pi / k, ng=ng, nx=nx, nv=nv, vmin=-6.0,
                    vmax=6.0, dt=0.1, nsteps=200, kind="landau",
                    params={"alpha": 0.01, "k": k}, seed=seed)


def two_stream(seed: int = 0, nx: int = 1024, nv: int = 1024, ng: int = 512) -> Workload:
    k = 0.2
    return Workload("two_stream", L=2 * math.pi / k, ng=ng, nx=nx, nv=nv, vmin=-8.0,
                    vmax=8.0, dt=0.05, nsteps=1000, kind="two_stream",
                    params={"alpha": 1e-3, "k": k, "v0": 2.4, "T": 1.0}, seed=seed)


def landau_nonlinear(seed: int = 0, nx: int = 2048, nv: int = 2048, ng: int = 256) -> Workload:
    k = 0.5
    return Workload("landau_nonlinear", L=2 * math.pi / k, ng=ng, nx=nx, nv=nv, vmin=-6.0,
                    vmax=6.0, dt=0.05, nsteps=2000, kind="landau",
                    params={"alpha": 0.5, "k": k}, seed=seed)


def landau_strong(seed: int = 0, nx: int = 128, nv: int = 128, ng: int = 128) -> Workload:
    """Strong Landau damping with the paper's parameters (L = 12, A = 0.5, k = 2 pi / L,
    dt = 0.2); Ng = 128 (a power of two) in place of the paper's 100 mesh points."""
    L = 12.0
    return Workload("landau_strong", L=L, ng=ng, nx=nx, nv=nv, vmin=-6.0, vmax=6.0, dt=0.2,
                    nsteps=500, kind="landau", params={"alpha": 0.5, "k": 2 * math.pi / L},
                    seed=seed)


def random_markers(w: Workload, n: int, seed: int = 0) -> dict:
    """Standard particle-in-cell start for a Landau workload (f0 = (1 + alpha cos kx) f_M(v),
    f_M the unit Maxwellian): x uniform on [0, L), v drawn from f_M, weight
    (1 + alpha cos kx) L / n, so the weights carry the density perturbation.  Monopoles only
    (Q, P, psi)."""
    if w.kind != "landau":
        raise ValueError("random markers are defined for Landau workloads")
    r = np.random.default_rng(np.random.SeedSequence(seed))
    x = r.uniform(0.0, w.L, n)
    v = r.standard_normal(n)
    a, k = w.params["alpha"], w.params["k"]
    return {"Q": x, "P": v, "psi": (1.0 + a * np.cos(k * x)) * (w.L / n)}


def landau_sweep(seed: int = 0, n_inst: int = 256, nsteps: int = 500) -> list:
    """The uneven batched sweep; instance i draws its parameters from child i of
    SeedSequence(seed) (first three uniforms: alpha, k, N0 exponent; then Ng choice)."""
    children = np.random.SeedSequence(seed).spawn(n_inst)
    out = []
    for i, ss in enumerate(children):
        r = np.random.default_rng(ss)
        alpha = math.exp(r.uniform(math.log(0.01), math.log(0.5)))
        k = r.uniform(0.3, 0.6)
        n0 = 2.0 ** r.uniform(12.0, 16.0)
        ng = int(r.choice([64, 128, 256]))
        nv = max(16, int(round(n0 / ng)))
        lattice_ss = ss.spawn(1)[0]
        out.append(Workload(f"landau_sweep[{i}]", L=2 * math.pi / k, ng=ng, nx=ng, nv=nv,
                            vmin=-6.0, vmax=6.0, dt=0.1, nsteps=nsteps, kind="landau",
                            params={"alpha": alpha, "k": k}, rng_seedseq=lattice_ss))
    return out


def served_jobs(seed: int = 0, n_jobs: int = 64, rate: float = 100.0,
                n_lo: float = 12.0, n_hi: float = 20.0, h_lo: int = 100, h_hi: int = 2000):
    """Seeded job stream: list of (arrival_time_s, Workload).  Job types cycle in thirds
    (Landau, two-stream, bump-on-tail); N = 2^U[n_lo, n_hi] rounded to a multiple of Ng;
    Ng in {64, 128, 256, 512, 1024}; horizon uniform in [h_lo, h_hi]; inter-arrival
    times exponential with the given rate (jobs per second)."""
    ss = np.random.SeedSequence(seed)
    r = np.random.default_rng(ss)
    t = 0.0
    jobs = []
    children = ss.spawn(n_jobs)
    for j in range(n_jobs):
        t += r.exponential(1.0 / rate)
        kind = ("landau", "two_stream", "bump_on_tail")[j % 3]
        ng = int(r.choice([64, 128, 256, 512, 1024]))
        n = 2.0 ** r.uniform(n_lo, n_hi)
        nv = max(16, int(round(n / ng)))
        horizon = int(r.integers(h_lo, h_hi + 1))
        if kind == "landau":
            alpha = math.exp(r.uniform(math.log(0.01), math.log(0.5)))
            k = r.uniform(0.3, 0.6)
            params, vmin, vmax = {"alpha": alpha, "k": k}, -6.0, 6.0
        elif kind == "two_stream":
            k = 0.2
            params = {"alpha": 1e-3, "k": k, "v0": r.uniform(1.5, 3.0), "T": 1.0}
            vmin, vmax = -8.0, 8.0
        else:
            k = 0.3
            params, vmin, vmax = {"alpha": 0.04, "k": k}, -8.0, 10.0
        dt = 0.1 if kind == "landau" else 0.05
        jobs.append((t, Workload(f"job{j}:{kind}", L=2 * math.pi / k, ng=ng, nx=ng, nv=nv,
                                 vmin=vmin, vmax=vmax, dt=dt, nsteps=horizon, kind=kind,
                                 params=params, rng_seedseq=children[j])))
    return jobs
