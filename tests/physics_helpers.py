"""Linear-theory references for the physics tests (independent of the oracle)."""
import math

import numpy as np


def plasma_z(zeta):
    """Plasma dispersion function Z(zeta) = i sqrt(pi) w(zeta) (Faddeeva function)."""
    from scipy.special import wofz
    return 1j * math.sqrt(math.pi) * wofz(zeta)


def newton_complex(D, guess, iters=80):
    om = complex(guess)
    for _ in range(iters):
        d = 1e-7
        om = om - D(om) / ((D(om + d) - D(om - d)) / (2 * d))
    assert abs(D(om)) < 1e-9, abs(D(om))
    return om


def landau_root(k, guess=1.4 - 0.15j):
    """Root of 1 + (1 + zeta Z(zeta)) / k^2 = 0, zeta = omega / (k sqrt 2): unit Maxwellian."""
    def D(om):
        z = om / (k * math.sqrt(2.0))
        return 1.0 + (1.0 + z * plasma_z(z)) / (k * k)
    return newton_complex(D, guess)


def two_stream_root(k, v0, T=1.0, guess=0.3j):
    """Root for two Maxwellian beams at +-v0, temperature T, density 1/2 each."""
    def D(om):
        s = 0.0
        for vb in (v0, -v0):
            z = (om - k * vb) / (k * math.sqrt(2.0 * T))
            s += 0.5 * (1.0 + z * plasma_z(z)) / (k * k * T)
        return 1.0 + s
    return newton_complex(D, guess)


def maxwellian_sum_root(k, beams, guess):
    """Root of the Vlasov dispersion relation for a sum of Maxwellians
    beams = [(density, drift, temperature), ...] (unit total charge):
    1 + sum_s n_s (1 + z_s Z(z_s)) / (k^2 T_s) = 0, z_s = (omega - k v_s) / (k sqrt(2 T_s))."""
    def D(om):
        s = 0.0
        for n, vb, T in beams:
            z = (om - k * vb) / (k * math.sqrt(2.0 * T))
            s += n * (1.0 + z * plasma_z(z)) / (k * k * T)
        return 1.0 + s
    return newton_complex(D, guess)


def bump_on_tail_root(k, guess=1.0 + 0.2j):
    """The bump-on-tail profile (0.9 exp(-v^2/2) + 0.2 exp(-2 (v - 4.5)^2)) / sqrt(2 pi) is
    0.9 N(0, 1) + 0.1 N(4.5, 1/4)."""
    return maxwellian_sum_root(k, [(0.9, 0.0, 1.0), (0.1, 4.5, 0.25)], guess)


def fit_damped_mode(t, z, t0, t1):
    """Least-squares fit of z(t) = exp(gamma t) (a cos wt + b sin wt), complex a, b, over
    t0 <= t <= t1; returns (gamma, omega)."""
    from scipy.optimize import minimize
    m = (t >= t0) & (t <= t1)
    t = np.asarray(t)[m]
    z = np.asarray(z)[m]

    def res(p):
        g, w = p
        B = np.stack([np.exp(g * t) * np.cos(w * t), np.exp(g * t) * np.sin(w * t)], 1)
        coef, *_ = np.linalg.lstsq(B, z, rcond=None)
        return float(np.sum(np.abs(z - B @ coef) ** 2))
    best = min((minimize(res, [g0, w0], method="Nelder-Mead",
                         options={"xatol": 1e-8, "fatol": 1e-16, "maxiter": 4000})
                for g0 in (-0.3, -0.1) for w0 in (1.3, 1.5)), key=lambda r: r.fun)
    return float(best.x[0]), float(best.x[1])


def fit_growth(t, a, t0, t1):
    """Exponential growth rate of a(t) > 0 by a straight-line fit of log a over [t0, t1]."""
    m = (t >= t0) & (t <= t1)
    return float(np.polyfit(np.asarray(t)[m], np.log(np.asarray(a)[m]), 1)[0])
