"""Closed-form two-body propagation for the tests (independent of the oracle).

Propagates a bound relative orbit with Lagrange's f and g functions written
in the eccentric-anomaly difference dE, where Kepler's equation in
difference form, n t = dE + (sigma0/sqrt(a)) (1 - cos dE) - (1 - r0/a) sin dE,
is solved by Newton iteration.
"""
import math

import numpy as np


def propagate(r0, v0, mu, t):
    r0 = np.asarray(r0, dtype=np.float64)
    v0 = np.asarray(v0, dtype=np.float64)
    rn = math.sqrt(float(r0 @ r0))
    v2 = float(v0 @ v0)
    a = 1.0 / (2.0 / rn - v2 / mu)
    if a <= 0:
        raise ValueError("unbound orbit")
    sig = float(r0 @ v0) / math.sqrt(mu)
    n = math.sqrt(mu / a ** 3)
    sa = math.sqrt(a)
    M = n * t
    dE = M
    for _ in range(200):
        f = dE + (sig / sa) * (1.0 - math.cos(dE)) - (1.0 - rn / a) * math.sin(dE) - M
        fp = 1.0 + (sig / sa) * math.sin(dE) - (1.0 - rn / a) * math.cos(dE)
        step = f / fp
        dE -= step
        if abs(step) < 1e-16 * max(1.0, abs(dE)):
            break
    c, s = math.cos(dE), math.sin(dE)
    r = a + (rn - a) * c + sig * sa * s
    F = 1.0 - (a / rn) * (1.0 - c)
    G = a * sig / math.sqrt(mu) * (1.0 - c) + rn * math.sqrt(a / mu) * s
    Fd = -math.sqrt(mu * a) / (r * rn) * s
    Gd = 1.0 - (a / r) * (1.0 - c)
    return F * r0 + G * v0, Fd * r0 + Gd * v0


def two_body_state(m0, m1, a, e, t):
    """Barycentric two-body orbit starting at pericentre in the x-y plane; state at time t."""
    mu = m0 + m1
    rp = a * (1.0 - e)
    vp = math.sqrt(mu * (1.0 + e) / rp)
    r0 = np.array([rp, 0.0, 0.0])
    v0 = np.array([0.0, vp, 0.0])
    if t != 0.0:
        r0, v0 = propagate(r0, v0, mu, t)
    x = np.stack([-m1 / mu * r0, m0 / mu * r0])
    v = np.stack([-m1 / mu * v0, m0 / mu * v0])
    return x, v
