"""The Runge-Kutta Cash-Karp kernels against the RKCK oracle: fixed-step
parity on 2..16-body ensembles, on 17..130-body systems (one body per lane
across a workgroup) and on a sampled full-size ensemble,
adaptive parity (step counts and states), bitwise independence of quanta,
straight-line motion of massless bodies, hand-over to Hermite, and
argument checks."""
import math
import sys

import numpy as np
import pytest

from paper_1208_1157_amd import gen
from tests.helpers import REL_TOL, explain_rkck_mismatch, per_system_rel_err

pytestmark = pytest.mark.gpu
TWO_PI = 2 * math.pi


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def ragged():
    parts = [gen.ragged_hill(160, seed=51, n_lo=2, n_hi=16), gen.paper_ics(4, 3), gen.paper_ics(4, 6)]
    nb = np.concatenate([p.n_body for p in parts])
    return gen.Ensemble(nb, np.concatenate([p.mass for p in parts]), np.concatenate([p.pos for p in parts]),
                        np.concatenate([p.vel for p in parts]))


def parity(ens, st, refs):
    off = ens.offsets
    worst = 0.0
    for s, o in refs.items():
        sl = slice(off[s], off[s + 1])
        ex = per_system_rel_err([ens.n_body[s]], st["pos"][sl], o["pos"])[0]
        ev = per_system_rel_err([ens.n_body[s]], st["vel"][sl], o["vel"])[0]
        worst = max(worst, ex, ev)
        assert ex <= REL_TOL and ev <= REL_TOL, (s, int(ens.n_body[s]), ex, ev)
    return worst


def test_fixed_parity_2_to_16(fb, ora):
    ens = ragged()
    dt, nsteps = TWO_PI / 200, 300
    say("RKCK fixed", ens.n_sys)
    E = fb.from_gen(ens)
    E.integrate_rkck_steps(nsteps, dt)
    st = E.state()
    E.close()
    assert np.all(st["status"] == fb.DONE) and np.all(st["steps"] == nsteps)
    refs = {s: ora.integrate_rkck_fixed(*ens.system(s), dt, nsteps) for s in range(ens.n_sys)}
    say("worst", parity(ens, st, refs))


def test_full_size_sampled_parity(fb, ora):
    ens, _ = gen.workload("homog_131072x3")
    dt, nsteps = TWO_PI / 200, 400
    say("RKCK full size")
    E = fb.from_gen(ens)
    E.integrate_rkck_steps(nsteps, dt)
    st = E.state()
    E.close()
    sample = np.random.default_rng(1).choice(ens.n_sys, 160, replace=False)
    parity(ens, st, {int(s): ora.integrate_rkck_fixed(*ens.system(int(s)), dt, nsteps) for s in sample})


def rkck_rerun(fb, system, t_end, eps, dt0):
    """rerun(k) for explain_rkck_mismatch: the system alone on the GPU, at
    most k accepted steps."""
    m, x, v = system

    def rerun(k):
        if k == 0:
            return {"pos": x, "vel": v, "t": 0.0, "steps": 0}
        E = fb.Ensemble(np.array([len(m)], dtype=np.int32), m, x, v)
        E.integrate_rkck(t_end, dt0, eps, fb.Opts(max_steps=int(k)))
        st = E.state()
        E.close()
        return {"pos": st["pos"], "vel": st["vel"], "t": float(st["t"][0]), "steps": int(st["steps"][0])}
    return rerun


def test_adaptive_parity(fb, ora):
    """Every system on a two-orbit horizon: where the accepted-step counts
    equal the oracle's, parity to 1e-10; where they differ, both sides match
    up to the first step whose decisions differ, and one of that step's
    decisions (a trial's acceptance, E against 1, or the clamp onto t_end)
    sits within 1e-8 of its threshold in the oracle's state."""
    ens = gen.ragged_hill(120, seed=52, n_lo=2, n_hi=12)
    t_end, dt0, eps = TWO_PI * 2, 0.02, 1e-10
    say("RKCK adaptive", ens.n_sys)
    E = fb.from_gen(ens)
    E.integrate_rkck(t_end, dt0, eps)
    st = E.state()
    E.close()
    assert np.all(st["status"] == fb.DONE) and np.all(st["t"] == t_end)
    refs, flips = {}, []
    for s in range(ens.n_sys):
        o = ora.integrate_rkck_adaptive(*ens.system(s), t_end, eps, dt0)
        assert o["status"] == ora.DONE
        if o["steps"] == st["steps"][s]:
            refs[s] = o
            continue
        flips.append((s, explain_rkck_mismatch(ora, ens.system(s), t_end, eps, dt0,
                                               rkck_rerun(fb, ens.system(s), t_end, eps, dt0),
                                               st["steps"][s], o)))
    say("worst", parity(ens, st, refs), "agree", len(refs), "flipped at a threshold", flips)
    assert len(refs) + len(flips) == ens.n_sys


@pytest.mark.parametrize("adaptive", [False, True])
def test_quanta_are_bitwise_invisible(fb, adaptive):
    ens = gen.ragged_hill(150, seed=53, n_lo=3, n_hi=11)
    dt = TWO_PI / 150
    say("RKCK quanta", adaptive)
    out = []
    for q in (0, 37):
        E = fb.from_gen(ens)
        o = fb.Opts(steps_per_quantum=q)
        if adaptive:
            E.integrate_rkck(TWO_PI, 0.05, 1e-9, o)
        else:
            E.integrate_rkck_steps(200, dt, o)
        out.append(E.state())
        E.close()
    assert np.array_equal(out[0]["pos"], out[1]["pos"]) and np.array_equal(out[0]["vel"], out[1]["vel"])
    assert np.array_equal(out[0]["steps"], out[1]["steps"])


def test_massless_bodies_move_on_straight_lines(fb):
    rng = np.random.default_rng(2)
    n, reps = 5, 40
    m = np.zeros(n * reps)
    x, v = rng.normal(size=(n * reps, 3)), rng.normal(size=(n * reps, 3))
    ens = gen.Ensemble(np.full(reps, n, dtype=np.int32), m, x, v)
    E = fb.from_gen(ens)
    E.integrate_rkck_steps(50, 0.3)
    st = E.state()
    E.close()
    assert np.abs(st["pos"] - (x + 15.0 * v)).max() < 1e-12 * (1 + np.abs(x + 15.0 * v).max())
    assert np.array_equal(st["vel"], v)


def test_hand_over_to_hermite(fb, ora):
    ens = gen.ragged_hill(40, seed=54, n_lo=3, n_hi=7)
    dt_r, dt_h = TWO_PI / 200, TWO_PI / 1000
    say("RKCK then Hermite")
    E = fb.from_gen(ens)
    E.integrate_rkck_steps(100, dt_r)
    acc, jerk, _ = E.hermite_state()          # re-evaluated at the current state
    E.integrate_steps(150, dt_h)
    st = E.state()
    E.close()
    off = ens.offsets
    for s in range(ens.n_sys):
        m = ens.system(s)[0]
        o = ora.integrate_rkck_fixed(*ens.system(s), dt_r, 100)
        a_ref, j_ref = ora.accjerk(m, o["pos"], o["vel"])
        sl = slice(off[s], off[s + 1])
        assert per_system_rel_err([ens.n_body[s]], acc[sl], a_ref)[0] <= REL_TOL
        x, v, _, _ = ora.integrate_fixed(m, o["pos"], o["vel"], dt_h, 150)
        assert per_system_rel_err([ens.n_body[s]], st["pos"][sl], x)[0] <= REL_TOL
        assert per_system_rel_err([ens.n_body[s]], st["vel"][sl], v)[0] <= REL_TOL


def test_argument_checks(fb):
    E = fb.from_gen(gen.three_body(4, seed=55))
    bad = [lambda: E.integrate_rkck_steps(10, 0.0),
           lambda: E.integrate_rkck_steps(-1, 0.01),
           lambda: E.integrate_rkck(1.0, 0.0, 1e-9),
           lambda: E.integrate_rkck(1.0, 0.01, 0.0),
           lambda: E.integrate_rkck(1.0, 0.01, 1e-9, fb.Opts(schedule=fb.SCHED_PERSISTENT)),
           lambda: E.integrate_rkck_steps(10, 0.01, fb.Opts(stop_rules=1)),
           lambda: E.integrate_rkck_steps(10, 0.01, fb.Opts(adaptive=True))]
    for f in bad:
        with pytest.raises(fb.FewbodyError) as ei:
            f()
        assert ei.value.code == fb.E_INVAL
    E.close()


def larger():
    parts = [gen.planetesimal_disk(6, 17, seed=56), gen.planetesimal_disk(3, 40, seed=57),
             gen.planetesimal_disk(2, 130, seed=58), gen.ragged_hill(20, seed=59, n_lo=3, n_hi=16)]
    nb = np.concatenate([p.n_body for p in parts])
    return gen.Ensemble(nb, np.concatenate([p.mass for p in parts]), np.concatenate([p.pos for p in parts]),
                        np.concatenate([p.vel for p in parts]))


def test_larger_systems_fixed_and_adaptive(fb, ora):
    ens = larger()
    dt, nsteps = TWO_PI / 200, 120
    say("RKCK larger systems", ens.n_sys)
    E = fb.from_gen(ens)
    E.integrate_rkck_steps(nsteps, dt, fb.Opts(steps_per_quantum=50))
    st = E.state()
    E.close()
    assert np.all(st["status"] == fb.DONE) and np.all(st["steps"] == nsteps)
    parity(ens, st, {s: ora.integrate_rkck_fixed(*ens.system(s), dt, nsteps) for s in range(ens.n_sys)})
    t_end, eps = 1.0, 1e-10
    E = fb.from_gen(ens)
    E.integrate_rkck(t_end, 0.02, eps)
    st = E.state()
    E.close()
    assert np.all(st["status"] == fb.DONE) and np.all(st["t"] == t_end)
    refs, flips = {}, []
    for s in range(ens.n_sys):
        o = ora.integrate_rkck_adaptive(*ens.system(s), t_end, eps, 0.02)
        assert o["status"] == ora.DONE
        if o["steps"] == st["steps"][s]:
            refs[s] = o
            continue
        flips.append((s, explain_rkck_mismatch(ora, ens.system(s), t_end, eps, 0.02,
                                               rkck_rerun(fb, ens.system(s), t_end, eps, 0.02),
                                               st["steps"][s], o)))
    say("adaptive worst", parity(ens, st, refs), "agree", len(refs), "flipped at a threshold", flips)
    assert len(refs) + len(flips) == ens.n_sys
