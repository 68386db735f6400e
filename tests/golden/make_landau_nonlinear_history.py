"""Writes landau_nonlinear_oracle.npz: the FP64 oracle's per-step diagnostics for the
nonlinear Landau damping workload (alpha = 0.5, k = 0.5, Ng = 256, 2048 x 2048 = 2^22
decorated particles, dt = 0.05, 2000 steps), the reference of the precision study.

    python tests/golden/make_landau_nonlinear_history.py [--steps 2000]

Calls only the oracle and the seeded input generator (single thread, about 4 minutes).
Initial state: FP32-rounded lattice state (the bits every GPU mode starts from), promoted
to FP64.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

KEYS = ("step", "t", "K", "W", "H", "charge", "momentum", "e_amp", "e1_re", "e1_im")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "landau_nonlinear_oracle.npz"))
    args = ap.parse_args()
    w = W.landau_nonlinear()
    st = w.state(np.float32)
    s = tuple(np.asarray(st[k], dtype=np.float64) for k in ("Q", "P", "qs", "ps", "psi"))
    fld = O.solve_field(s[0], s[3], s[4], w.L, w.ng)
    rows = [O.diagnostics(s[1], s[2], s[4], fld, w.L)]
    t0 = time.time()
    for n in range(args.steps):
        s, fld = O.step(s, fld, w.L, w.ng, w.dt)
        rows.append(O.diagnostics(s[1], s[2], s[4], fld, w.L))
        if (n + 1) % 100 == 0:
            print(f"step {n + 1} / {args.steps}, {time.time() - t0:.0f} s", flush=True)
    hist = np.array([[r.get(k, np.nan) if k not in ("step", "t") else np.nan for k in KEYS]
                     for r in rows])
    hist[:, 0] = np.arange(len(rows))
    hist[:, 1] = np.arange(len(rows)) * w.dt
    np.savez_compressed(args.out, keys=np.array(KEYS), hist=hist,
                        n=w.n, ng=w.ng, L=w.L, dt=w.dt, steps=args.steps)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
