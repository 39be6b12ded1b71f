"""Pins of the MVS oracle (Section 2.2.3's mixed-variable symplectic
integrator) against facts that do not come from it: Kepler orbits through
the classical elements with Kepler's equation solved by bisection, rigid
rotation of circular orbits, the group properties of a Kepler flow,
massless planets (where the method is exact), second order against the
independently pinned Hermite oracle, time reversibility, bounded energy
error, and exact conservation of momentum and angular momentum."""
import math

import numpy as np
import pytest

from paper_1208_1157_amd import gen

TWO_PI = 2 * math.pi


def elements_propagate(r0, v0, mu, t):
    """Independent Kepler propagation: (r, v) -> a, e, perifocal frame and
    mean anomaly; M + n t; Kepler's equation M = E - e sin E by bisection;
    back to Cartesian."""
    r0 = np.asarray(r0, float)
    v0 = np.asarray(v0, float)
    rn = np.linalg.norm(r0)
    h = np.cross(r0, v0)
    evec = np.cross(v0, h) / mu - r0 / rn
    e = np.linalg.norm(evec)
    a = 1.0 / (2.0 / rn - v0 @ v0 / mu)
    W = h / np.linalg.norm(h)
    if e > 1e-12:
        P = evec / e
        cosE = (1.0 - rn / a) / e
        sinE = (r0 @ v0) / (e * math.sqrt(mu * a))
        E0 = math.atan2(sinE, cosE)
    else:
        P, E0 = r0 / rn, 0.0
    Qb = np.cross(W, P)
    n = math.sqrt(mu / a ** 3)
    M = E0 - e * math.sin(E0) + n * t
    lo, hi = M - 1.0, M + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid - e * math.sin(mid) - M > 0:
            hi = mid
        else:
            lo = mid
    E = 0.5 * (lo + hi)
    b = a * math.sqrt(1.0 - e * e)
    den = 1.0 - e * math.cos(E)
    r = a * (math.cos(E) - e) * P + b * math.sin(E) * Qb
    v = (-a * n * math.sin(E) / den) * P + (b * n * math.cos(E) / den) * Qb
    return r, v


def orbit(mu, a, e, inc, node, peri, M):
    """(r, v) of a bound orbit from elements (angles in radians)."""
    E = M
    for _ in range(100):
        E = E - (E - e * math.sin(E) - M) / (1 - e * math.cos(E))
    b = a * math.sqrt(1 - e * e)
    n = math.sqrt(mu / a ** 3)
    den = 1 - e * math.cos(E)
    xp = np.array([a * (math.cos(E) - e), b * math.sin(E), 0.0])
    vp = np.array([-a * n * math.sin(E) / den, b * n * math.cos(E) / den, 0.0])

    def rz(t):
        c, s = math.cos(t), math.sin(t)
        return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])

    def rx(t):
        c, s = math.cos(t), math.sin(t)
        return np.array([[1.0, 0, 0], [0, c, -s], [0, s, c]])

    R = rz(node) @ rx(inc) @ rz(peri)
    return R @ xp, R @ vp


def energy(m, x, v):
    ke = 0.5 * np.sum(m * np.sum(v * v, axis=1))
    pe = 0.0
    for i in range(len(m)):
        for j in range(i + 1, len(m)):
            pe -= m[i] * m[j] / np.linalg.norm(x[i] - x[j])
    return ke + pe


@pytest.mark.parametrize("e", [0.05, 0.3, 0.7])
def test_kepler_drift_matches_elements(ora, e):
    mu = 1.3
    r0, v0 = orbit(mu, 1.7, e, 0.4, 1.1, 2.3, 0.9)
    period = TWO_PI * math.sqrt(1.7 ** 3 / mu)
    for t in (1e-3, 0.37, 0.5 * period, 1.3 * period, -0.2 * period):
        out = ora.kepler_drift(mu, r0, v0, t)
        assert out is not None
        re, ve = elements_propagate(r0, v0, mu, t)
        assert np.abs(out[0] - re).max() < 2e-13 * (1 + np.abs(re).max()), (e, t)
        assert np.abs(out[1] - ve).max() < 2e-13 * (1 + np.abs(ve).max()), (e, t)


def test_kepler_drift_circular_is_a_rotation(ora):
    """A circular orbit rotates rigidly by n t about its angular momentum."""
    mu, a = 0.9, 2.2
    r0, v0 = orbit(mu, a, 0.0, 0.7, 0.3, 0.0, 1.4)
    n = math.sqrt(mu / a ** 3)
    w = np.cross(r0, v0)
    w /= np.linalg.norm(w)
    for t in (0.01, 3.0, 17.5):
        th = n * t
        K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        R = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
        r, v = ora.kepler_drift(mu, r0, v0, t)
        assert np.abs(r - R @ r0).max() < 1e-13 * a
        assert np.abs(v - R @ v0).max() < 1e-13 * math.sqrt(mu / a)


def test_kepler_drift_group_properties(ora):
    mu = 1.0
    r0, v0 = orbit(mu, 1.0, 0.2, 0.1, 0.2, 0.3, 0.4)
    r1, v1 = ora.kepler_drift(mu, r0, v0, 0.3)
    r2, v2 = ora.kepler_drift(mu, r1, v1, 0.5)
    r3, v3 = ora.kepler_drift(mu, r0, v0, 0.8)
    assert np.abs(r2 - r3).max() < 1e-14 and np.abs(v2 - v3).max() < 1e-14
    rb, vb = ora.kepler_drift(mu, r3, v3, -0.8)
    assert np.abs(rb - r0).max() < 1e-14 and np.abs(vb - v0).max() < 1e-14
    # energy and angular momentum of the orbit are invariants
    E0 = 0.5 * v0 @ v0 - mu / np.linalg.norm(r0)
    E3 = 0.5 * v3 @ v3 - mu / np.linalg.norm(r3)
    assert abs(E3 - E0) < 1e-15
    assert np.abs(np.cross(r3, v3) - np.cross(r0, v0)).max() < 1e-15


def test_kepler_drift_refuses_unbound(ora):
    mu = 1.0
    r0 = np.array([1.0, 0.0, 0.0])
    assert ora.kepler_drift(mu, r0, np.array([0.0, 1.5, 0.0]), 0.1) is None   # hyperbolic
    assert ora.kepler_drift(mu, r0, np.array([0.0, math.sqrt(2.0), 0.0]), 0.1) is None  # parabolic


def test_helio_round_trip_and_momenta(ora):
    ens = gen.ragged_hill(3, seed=3, n_lo=4, n_hi=7)
    for s in range(ens.n_sys):
        m, x, v = ens.system(s)
        x = x + np.array([0.3, -0.2, 0.1])
        v = v + np.array([0.01, 0.02, -0.03])
        Q, V, X, Vc = ora.mvs_to_helio(m, x, v)
        assert np.abs(Q[1:] - (x[1:] - x[0])).max() < 1e-15
        assert np.abs(X - (m @ x) / m.sum()).max() < 1e-15
        assert np.abs(Vc - (m @ v) / m.sum()).max() < 1e-15
        x2, v2 = ora.mvs_from_helio(m, Q, V, X, Vc)
        assert np.abs(x2 - x).max() < 1e-14 and np.abs(v2 - v).max() < 1e-14


def test_kick_is_planet_planet_only(ora):
    m = np.array([1.0, 2e-3, 3e-3, 0.0])
    Q = np.array([[0, 0, 0], [1.0, 0, 0], [1.0, 2.0, 0], [0, 0, 5.0]])
    acc = ora.mvs_kick_acc(m, Q)
    # planet 3 is massless: only planet 2, at (0, 2, 0) from planet 1, pulls on it
    assert np.abs(acc[1] - np.array([0.0, 3e-3 / 4.0, 0.0])).max() < 1e-18
    assert np.abs(acc[2] - np.array([0.0, -2e-3 / 4.0, 0.0])).max() < 1e-18
    d31, d32 = Q[1] - Q[3], Q[2] - Q[3]
    exp3 = 2e-3 * d31 / np.linalg.norm(d31) ** 3 + 3e-3 * d32 / np.linalg.norm(d32) ** 3
    assert np.abs(acc[3] - exp3).max() < 1e-18
    assert np.all(acc[0] == 0)


@pytest.mark.parametrize("dt_frac", [0.003, 0.11, 0.5])
def test_massless_planets_follow_exact_kepler_orbits(ora, dt_frac):
    """With massless planets the interaction and drift terms vanish and the
    star stays at the barycentre: MVS is exact at any step size."""
    mu = 1.0
    els = [(1.0, 0.1, 0.02, 0.3, 0.5, 0.1), (1.6, 0.4, 0.2, 1.0, 2.0, 3.0), (2.9, 0.05, 0.1, 4.0, 0.2, 5.5)]
    m = np.array([mu] + [0.0] * len(els))
    x = np.zeros((len(m), 3))
    v = np.zeros((len(m), 3))
    for k, el in enumerate(els):
        x[k + 1], v[k + 1] = orbit(mu, *el)
    dt = dt_frac * TWO_PI
    nsteps = 40
    out = ora.integrate_mvs(m, x, v, dt, nsteps)
    assert out["status"] == ora.DONE and out["steps"] == nsteps
    assert np.abs(out["pos"][0]).max() == 0.0
    for k in range(len(els)):
        re, ve = elements_propagate(x[k + 1], v[k + 1], mu, dt * nsteps)
        assert np.abs(out["pos"][k + 1] - re).max() < 1e-11
        assert np.abs(out["vel"][k + 1] - ve).max() < 1e-11


def test_second_order_against_hermite(ora):
    """Position error against the (independently pinned) Hermite oracle at a
    tiny step falls by 4 on halving the MVS step."""
    ens = gen.paper_ics(1, 3)
    m, x, v = ens.system(0)
    T = TWO_PI * 3
    ref = ora.integrate_fixed(m, x, v, T / 24000, 24000)
    errs = []
    for k in (150, 300, 600):
        out = ora.integrate_mvs(m, x, v, T / k, k)
        errs.append(np.abs(out["pos"] - ref[0]).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


def test_time_reversible(ora):
    ens = gen.ragged_hill(1, seed=12, n_lo=5, n_hi=5)
    m, x, v = ens.system(0)
    dt = TWO_PI / 60
    fwd = ora.integrate_mvs(m, x, v, dt, 300)
    back = ora.integrate_mvs(m, fwd["pos"], fwd["vel"], -dt, 300)
    assert np.abs(back["pos"] - x).max() < 1e-12
    assert np.abs(back["vel"] - v).max() < 1e-12


def test_energy_error_bounded_and_momenta_exact(ora):
    """Symplectic: on a stable two-planet system the energy error oscillates
    without secular growth over 1000 orbits (its envelope in the first 100
    orbits bounds the rest), while linear and angular momentum are conserved
    to rounding."""
    ens = gen.paper_ics(1, 3)
    m, x, v = ens.system(0)
    dt = TWO_PI / 40
    E0 = energy(m, x, v)
    P0 = m @ v
    L0 = np.sum(m[:, None] * np.cross(x, v), axis=0)
    early, late = 0.0, 0.0
    for k in range(200):
        out = ora.integrate_mvs(m, x, v, dt, 200)
        x, v = out["pos"], out["vel"]
        err = abs(energy(m, x, v) / E0 - 1)
        if k < 20:
            early = max(early, err)
        else:
            late = max(late, err)
    assert late < 1.5 * early, (early, late)
    assert np.abs(m @ v - P0).max() < 1e-16
    L = np.sum(m[:, None] * np.cross(x, v), axis=0)
    assert np.abs(L - L0).max() < 1e-12 * np.abs(L0).max()
