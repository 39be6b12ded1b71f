"""GPU stop statuses against the oracle: STALLED_DT and MAXSTEPS.

The adaptive step stalls a system when its proposal falls below 1e-12 of the
destination time; a per-system cap on steps stops it with MAXSTEPS (the
maximum-iterations stop of Algorithm 1's loop, Section 4.3).  Both are
reached here on the GPU, in both lane mappings and both schedules, and
compared system by system with the oracle: status, step count and state.
"""
import math
import sys

import numpy as np
import pytest

from paper_1208_1157_amd import gen
from tests import kepler
from tests.helpers import REL_TOL, assert_parity, check_adaptive_systems, oracle_fixed

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def plunging_ensemble():
    """Star (m0 = 1, at rest at the origin) + one planet on a nearly radial
    orbit (a = 1, pericentre q) that is falling in, + 0..5 planets on wide
    circular orbits.  The pairwise step shrinks with the separation near
    pericentre: small q stall (step below 1e-8 = 1e-12 t_end for t_end =
    1e4), larger q pass pericentre and run on until the step cap."""
    rng = np.random.default_rng(17)
    nb, ms, xs, vs = [], [], [], []
    for q in (1e-6, 3e-6, 1e-5, 3e-5, 1e-4, 3e-4, 1e-3):
        for n in (2, 3, 5, 7):
            m1 = 10 ** rng.uniform(-7, -5)
            mu = 1.0 + m1
            e = 1.0 - q
            r0 = np.array([q, 0.0, 0.0])
            v0 = np.array([0.0, math.sqrt(mu * (1 + e) / q), 0.0])
            r, v = kepler.propagate(r0, v0, mu, 2 * math.pi * rng.uniform(0.75, 0.9))
            m = [1.0, m1]
            x = [np.zeros(3), r]
            u = [np.zeros(3), v]
            for k in range(n - 2):
                a = 6.0 + 4.0 * k
                th = rng.uniform(0, 2 * math.pi)
                mk = 10 ** rng.uniform(-7, -5)
                vc = math.sqrt((1.0 + mk) / a)
                m.append(mk)
                x.append(np.array([a * math.cos(th), a * math.sin(th), 0.0]))
                u.append(np.array([-vc * math.sin(th), vc * math.cos(th), 0.0]))
            nb.append(n)
            ms.extend(m)
            xs.extend(x)
            vs.extend(u)
    return gen.Ensemble(np.array(nb, dtype=np.int32), np.array(ms), np.array(xs), np.array(vs))


@pytest.mark.parametrize("sched", ["plain", "persistent_compact"])
@pytest.mark.parametrize("mapping", ["spl", "bpl"])
def test_stalled_dt_and_max_steps_match_the_oracle(plans, ora, sched, mapping):
    fb = plans
    for n in range(2, 17):
        fb.set_plan(n, fb.MAP_SPL if mapping == "spl" and n <= 8 else fb.MAP_BPL, 2)
    fb.set_plan(0, fb.MAP_SPL if mapping == "spl" else fb.MAP_BPL, 2, 8)
    ens = plunging_ensemble()
    t_end, eta, cap = 1e4, 0.01, 3000
    opts = fb.Opts(adaptive=1, eta=eta, stop_rules=3, r_eject=100.0, max_steps=cap)
    if sched != "plain":
        opts.schedule, opts.steps_per_quantum, opts.compact = fb.SCHED_PERSISTENT, 400, True
    say("stall / max steps", sched, mapping, ens.n_sys)
    E = fb.from_gen(ens)
    E.integrate(t_end, 0.0, opts)
    st = E.state()
    E.close()
    agree, nflip, worst, flips = check_adaptive_systems(fb, ora, ens, range(ens.n_sys), st, t_end, eta, 3,
                                                        100.0, False, max_steps=cap)
    stalled = int(np.sum(st["status"] == fb.STALLED_DT))
    capped = int(np.sum(st["status"] == fb.MAXSTEPS))
    say("agree", agree, "flips", nflip, flips, "stalled", stalled, "capped", capped, "worst", worst)
    assert agree + nflip == ens.n_sys
    assert stalled >= 8 and capped >= 8, (stalled, capped)
    assert np.all(st["steps"][st["status"] == fb.MAXSTEPS] == cap)


def test_stall_threshold_both_sides(fb, ora):
    """Circular two-body orbits whose first proposal sits 1e-6 below or above
    the stall threshold: below stalls before the first step (state, time and
    step count untouched), above steps until the cap."""
    m0, m1 = 1.0, 1e-3
    x, v = kepler.two_body_state(m0, m1, 1.0, 0.0, 0.4)
    m = np.array([m0, m1])
    r, u = x[1] - x[0], v[1] - v[0]
    ur = (r @ u) / np.linalg.norm(r)
    dt0 = 0.01 * np.linalg.norm(r) / math.sqrt(u @ u - ur * ur + 4 * ur * ur)
    ens = gen.Ensemble(np.array([2] * 8, dtype=np.int32), np.tile(m, 8), np.tile(x, (8, 1)), np.tile(v, (8, 1)))
    for side, t_end, want in (("stall", dt0 / 1e-12 * (1 + 1e-6), fb.STALLED_DT),
                              ("go", dt0 / 1e-12 * (1 - 1e-6), fb.MAXSTEPS)):
        say("stall threshold", side)
        E = fb.from_gen(ens)
        E.integrate(t_end, 0.0, fb.Opts(adaptive=1, eta=0.01, max_steps=3))
        st = E.state()
        E.close()
        o = ora.integrate_adaptive(m, x, v, t_end=t_end, eta=0.01, stop_rules=0, max_steps=3)
        assert o["status"] == want and np.all(st["status"] == want), (side, st["status"])
        assert np.all(st["steps"] == o["steps"])
        assert_parity(ens.n_body, st["pos"], st["vel"], np.tile(o["pos"], (8, 1)), np.tile(o["vel"], (8, 1)),
                      label=side)
        if want == fb.STALLED_DT:
            assert np.array_equal(st["pos"], ens.pos) and np.all(st["t"] == 0.0)


@pytest.mark.parametrize("sched", ["plain", "persistent"])
def test_fixed_step_cap_and_continuation(fb, ora, sched):
    """Fixed steps with max_steps below the requested count stop every system
    at the cap (MAXSTEPS, the oracle's state after that many steps); a later
    call without a cap continues from there and matches the oracle's
    uninterrupted run of the total."""
    ens = gen.ragged_hill(300, seed=23, n_lo=2, n_hi=16)
    h = 2 * math.pi / 2000
    o1 = fb.Opts(max_steps=60)
    o2 = fb.Opts()
    if sched == "persistent":
        for o in (o1, o2):
            o.schedule, o.steps_per_quantum = fb.SCHED_PERSISTENT, 25
    say("fixed-step cap", sched)
    E = fb.from_gen(ens)
    E.integrate_steps(100, h, o1)
    a = E.state()
    E.integrate_steps(100, h, o2)
    b = E.state()
    E.close()
    assert np.all(a["status"] == fb.MAXSTEPS) and np.all(a["steps"] == 60)
    X, V, _, _ = oracle_fixed(ora, ens, h, 60)
    assert_parity(ens.n_body, a["pos"], a["vel"], X, V, label="cap")
    assert np.all(b["status"] == fb.DONE) and np.all(b["steps"] == 160)
    X, V, _, _ = oracle_fixed(ora, ens, h, 160)
    assert_parity(ens.n_body, b["pos"], b["vel"], X, V, label="continued")
