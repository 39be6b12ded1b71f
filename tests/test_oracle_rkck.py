"""Pins of the Runge-Kutta Cash-Karp oracle (Sections 2.2.2 and 4.3.2)
against facts that do not come from it: straight-line motion of massless
bodies, the closed-form Kepler orbit (fifth order, an error estimate of
order h^5 that measures the fourth-order solution's error), convergence to
the independently pinned Hermite oracle, and adaptive control that meets
its tolerance, rejects oversized trials and lands on t_end."""
import math

import numpy as np
import pytest

from paper_1208_1157_amd import gen
from tests import kepler

TWO_PI = 2 * math.pi


def test_massless_bodies_move_on_straight_lines(ora):
    rng = np.random.default_rng(1)
    m = np.zeros(4)
    x, v = rng.normal(size=(4, 3)), rng.normal(size=(4, 3))
    for h in (1e-3, 0.7, 13.0):
        x5, v5, ex, ev = ora.rkck_step(m, x, v, h)
        assert np.abs(x5 - (x + h * v)).max() <= 1e-14 * (1 + np.abs(x + h * v).max())
        assert np.array_equal(v5, v)
        assert np.abs(ex).max() <= 1e-15 * h * np.abs(v).max() and np.all(ev == 0)


def kepler_error(ora, h, T, e=0.3):
    m0, m1 = 1.0, 1e-3
    x, v = kepler.two_body_state(m0, m1, 1.0, e, 0.0)
    nsteps = int(round(T / h))
    out = ora.integrate_rkck_fixed(np.array([m0, m1]), x, v, T / nsteps, nsteps)
    xe, _ = kepler.two_body_state(m0, m1, 1.0, e, T)
    return np.abs(out["pos"] - xe).max()


def test_fifth_order_on_kepler(ora):
    T = TWO_PI * 2
    e1, e2, e3 = (kepler_error(ora, T / k, T) for k in (200, 400, 800))
    assert 26 < e1 / e2 < 38 and 26 < e2 / e3 < 38, (e1, e2, e3)


def test_error_estimate_is_the_fourth_order_error(ora):
    """One step from a point of an eccentric orbit: the estimate shrinks as
    h^5, and y5 - estimate (the fourth-order result) misses the exact state
    by about the estimate."""
    m0, m1 = 1.0, 1e-3
    x, v = kepler.two_body_state(m0, m1, 1.0, 0.5, 0.4)
    m = np.array([m0, m1])
    est = []
    for h in (0.02, 0.01):
        x5, v5, ex, ev = ora.rkck_step(m, x, v, h)
        xe, _ = kepler.two_body_state(m0, m1, 1.0, 0.5, 0.4 + h)
        err4 = np.abs(x5 - ex - xe).max()
        assert 0.85 < err4 / np.abs(ex).max() < 1.15, (h, err4, np.abs(ex).max())
        assert np.abs(x5 - xe).max() < 0.2 * np.abs(ex).max()
        est.append(np.abs(ex).max())
    assert 26 < est[0] / est[1] < 38


def test_converges_to_hermite(ora):
    ens = gen.paper_ics(1, 4)
    m, x, v = ens.system(0)
    T = TWO_PI
    ref = ora.integrate_fixed(m, x, v, T / 20000, 20000)[0]
    errs = [np.abs(ora.integrate_rkck_fixed(m, x, v, T / k, k)["pos"] - ref).max() for k in (100, 200)]
    assert 26 < errs[0] / errs[1] < 38, errs


def test_acceleration_matches_hermite_oracle(ora):
    ens = gen.ragged_hill(3, seed=5, n_lo=3, n_hi=9)
    for s in range(ens.n_sys):
        m, x, v = ens.system(s)
        a_h, _ = ora.accjerk(m, x, v)
        assert np.abs(ora.rk_acc(m, x) - a_h).max() <= 1e-15 * np.abs(a_h).max()


def test_error_norm_by_hand(ora):
    x = np.array([[0.0, 0, 0], [3.0, 4.0, 0]])           # X = 5
    v = np.array([[0.0, 0, 1.0], [0, 2.0, 0]])           # V = 2
    ex = np.array([[1e-9, 0, 0], [0, 0, 0]])
    ev = np.array([[0, 0, 0], [0, 3e-9, 4e-9]])          # |ev| = 5e-9
    assert ora.rkck_error_norm(x, v, ex, ev, 1e-9) == pytest.approx(max(1e-9 / 5e-9, 5e-9 / 2e-9))


@pytest.mark.parametrize("e", [0.1, 0.6])
def test_adaptive_error_tracks_tolerance(ora, e):
    m0, m1 = 1.0, 1e-3
    x, v = kepler.two_body_state(m0, m1, 1.0, e, 0.0)
    T = TWO_PI * 3
    xe, _ = kepler.two_body_state(m0, m1, 1.0, e, T)
    errs, steps = [], []
    for eps in (1e-9, 1e-11):
        out = ora.integrate_rkck_adaptive(np.array([m0, m1]), x, v, T, eps, 0.05)
        assert out["status"] == ora.DONE and out["t"] == T
        errs.append(np.abs(out["pos"] - xe).max())
        steps.append(out["steps"])
    assert errs[1] < errs[0] / 10 and errs[0] < 1e4 * 1e-9
    assert steps[1] > steps[0]


def test_adaptive_rejects_an_oversized_first_trial(ora):
    m0, m1 = 1.0, 1e-3
    x, v = kepler.two_body_state(m0, m1, 1.0, 0.3, 0.0)
    T = TWO_PI
    out = ora.integrate_rkck_adaptive(np.array([m0, m1]), x, v, T, 1e-10, 5.0)
    xe, _ = kepler.two_body_state(m0, m1, 1.0, 0.3, T)
    assert out["rejects"] >= 1 and out["status"] == ora.DONE
    assert np.abs(out["pos"] - xe).max() < 1e-6


def test_adaptive_eccentric_orbits_take_more_steps(ora):
    m0, m1 = 1.0, 1e-3
    n = []
    for e in (0.05, 0.8):
        x, v = kepler.two_body_state(m0, m1, 1.0, e, 0.0)
        n.append(ora.integrate_rkck_adaptive(np.array([m0, m1]), x, v, TWO_PI, 1e-10, 0.01)["steps"])
    assert n[1] > 1.3 * n[0]


def test_adaptive_limits(ora):
    m0, m1 = 1.0, 1e-3
    x, v = kepler.two_body_state(m0, m1, 1.0, 0.2, 0.0)
    out = ora.integrate_rkck_adaptive(np.array([m0, m1]), x, v, TWO_PI, 1e-10, 0.01, max_steps=7)
    assert out["status"] == ora.MAXSTEPS and out["steps"] == 7
    out = ora.integrate_rkck_adaptive(np.array([m0, m1]), x, v, TWO_PI, 1e-10, 1e-13)
    assert out["status"] == ora.STALLED_DT and out["steps"] == 0


def test_acceptance_threshold(ora):
    """A first trial whose error norm is about 10 is rejected; one of about
    0.5 is accepted (E = 1 is the boundary)."""
    m0, m1 = 1.0, 1e-3
    m = np.array([m0, m1])
    x, v = kepler.two_body_state(m0, m1, 1.0, 0.4, 0.0)
    eps = 1e-10

    def norm(h):
        x5, v5, ex, ev = ora.rkck_step(m, x, v, h)
        return ora.rkck_error_norm(x, v, ex, ev, eps)

    def h_for(target):
        lo, hi = 1e-6, 1.0
        for _ in range(100):
            mid = math.sqrt(lo * hi)
            lo, hi = (mid, hi) if norm(mid) < target else (lo, mid)
        return math.sqrt(lo * hi)

    h_bad, h_good = h_for(10.0), h_for(0.5)
    assert 5 < norm(h_bad) < 20 and 0.3 < norm(h_good) < 0.8
    out = ora.integrate_rkck_adaptive(m, x, v, 100.0, eps, h_bad, max_steps=1)
    assert out["rejects"] >= 1 and out["steps"] == 1
    out = ora.integrate_rkck_adaptive(m, x, v, 100.0, eps, h_good, max_steps=1)
    assert out["rejects"] == 0 and out["steps"] == 1
    assert out["dt_next"] == pytest.approx(h_good * 0.9 * norm(h_good) ** -0.2)
