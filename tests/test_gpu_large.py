"""The large-n gravitation (Section 4.2's variant for larger systems: one
body per lane across a workgroup, each pair evaluated from both sides)
against the Hermite oracle: fixed-step parity for 17..512 bodies beside
small systems in one ensemble, a sampled full-size disk ensemble, the
set-up evaluation, the last shortened step of a run to t_end, adaptive
steps under both rules, the stop rules, the persistent schedule beside the
fused launch of small systems, diagnostics, logging, invisible quanta, and
the calls that refuse such systems."""
import math
import sys

import numpy as np
import pytest

from paper_1208_1157_amd import gen
from tests.helpers import REL_TOL, per_system_rel_err, threads

pytestmark = pytest.mark.gpu
TWO_PI = 2 * math.pi


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def concat(parts):
    return gen.Ensemble(np.concatenate([p.n_body for p in parts]), np.concatenate([p.mass for p in parts]),
                        np.concatenate([p.pos for p in parts]), np.concatenate([p.vel for p in parts]))


def mixed():
    """Small and large systems together; the large counts leave partial
    workgroups (17 and 33 bodies run 15 systems per workgroup)."""
    parts = [gen.three_body(40, seed=71), gen.ragged_hill(30, seed=72, n_lo=14, n_hi=16)]
    for n, k, seed in ((17, 20, 73), (24, 7, 74), (33, 20, 75), (64, 5, 76), (100, 3, 77),
                       (129, 2, 78), (256, 2, 79), (512, 1, 80)):
        parts.append(gen.planetesimal_disk(k, n, seed=seed))
    return concat(parts)


def check(ens, pos, vel, x, v, label):
    ex = per_system_rel_err(ens.n_body, pos, x)
    ev = per_system_rel_err(ens.n_body, vel, v)
    w = int(np.argmax(np.maximum(ex, ev)))
    assert ex.max() <= REL_TOL and ev.max() <= REL_TOL, (label, w, int(ens.n_body[w]), ex.max(), ev.max())
    return max(ex.max(), ev.max())


def test_fixed_step_parity_17_to_512(fb, ora):
    ens = mixed()
    dt, nsteps = TWO_PI / 1000, 150
    say("large-n parity", ens.n_sys, sorted(set(ens.n_body.tolist())))
    E = fb.from_gen(ens)
    E.integrate_steps(nsteps, dt)
    st = E.state()
    E.close()
    assert np.all(st["status"] == fb.DONE) and np.all(st["steps"] == nsteps)
    assert np.allclose(st["t"], nsteps * dt, rtol=1e-14, atol=0)
    x, v, _, _ = ora.ensemble_fixed(ens.n_body, ens.mass, ens.pos, ens.vel, dt, nsteps, nthreads=threads())
    say("worst", check(ens, st["pos"], st["vel"], x, v, "mixed"))


def test_setup_evaluation(fb, ora):
    ens = concat([gen.planetesimal_disk(4, 40, seed=81), gen.planetesimal_disk(2, 300, seed=82)])
    E = fb.from_gen(ens)
    acc, jerk, _ = E.hermite_state()
    E.close()
    off = ens.offsets
    for s in range(ens.n_sys):
        a_ref, j_ref = ora.accjerk(*ens.system(s))
        sl = slice(off[s], off[s + 1])
        assert per_system_rel_err([ens.n_body[s]], acc[sl], a_ref)[0] <= 1e-13
        assert per_system_rel_err([ens.n_body[s]], jerk[sl], j_ref)[0] <= 1e-13


def test_full_size_sampled_parity(fb, ora):
    ens, p = gen.workload("disk_4096x64")
    nsteps = 200
    say("large-n full size", ens.n_sys)
    E = fb.from_gen(ens)
    E.integrate_steps(nsteps, p["dt"])
    st = E.state()
    E.close()
    assert np.all(st["status"] == fb.DONE)
    sample = np.random.default_rng(3).choice(ens.n_sys, 24, replace=False)
    off = ens.offsets
    for s in sample:
        s = int(s)
        x, v, _, _ = ora.integrate_fixed(*ens.system(s), p["dt"], nsteps)
        sl = slice(off[s], off[s + 1])
        check(ens.subset([s]), st["pos"][sl], st["vel"][sl], x, v, f"system {s}")


def test_run_to_t_end_shortens_the_last_step(fb, ora):
    ens = gen.planetesimal_disk(6, 48, seed=83)
    dt = TWO_PI / 500
    t_end = 37.4 * dt
    E = fb.from_gen(ens)
    E.integrate(t_end, dt)
    st = E.state()
    E.close()
    assert np.all(st["t"] == t_end) and np.all(st["steps"] == 38)
    off = ens.offsets
    for s in range(ens.n_sys):
        m, x0, v0 = ens.system(s)
        x, v, a, j = ora.integrate_fixed(m, x0, v0, dt, 37)
        x, v, _, _ = ora.integrate_fixed(m, x, v, t_end - 37 * dt, 1, acc=a, jerk=j)
        sl = slice(off[s], off[s + 1])
        check(ens.subset([s]), st["pos"][sl], st["vel"][sl], x, v, f"system {s}")


def test_diagnostics(fb, ora):
    ens = concat([gen.planetesimal_disk(5, 20, seed=84), gen.planetesimal_disk(3, 200, seed=85),
                  gen.three_body(5, seed=86)])
    E = fb.from_gen(ens)
    e0, l0 = E.diagnostics()
    E.integrate_steps(100, TWO_PI / 1000)
    e1, l1 = E.diagnostics()
    st = E.state()
    E.close()
    r0 = ora.ensemble_energy(ens.n_body, ens.mass, ens.pos, ens.vel)
    r1 = ora.ensemble_energy(ens.n_body, ens.mass, st["pos"], st["vel"])
    for (e, l), (er, lr) in (((e0, l0), r0), ((e1, l1), r1)):
        assert np.all(np.abs(e - er) <= 1e-12 * np.abs(er))
        assert np.all(np.linalg.norm(l - lr, axis=1) <= 1e-12 * np.linalg.norm(lr, axis=1))


@pytest.mark.parametrize("kind", ["state", "rv", "energy"])
def test_logging(fb, ora, kind):
    ens = concat([gen.planetesimal_disk(4, 30, seed=87), gen.planetesimal_disk(2, 130, seed=88)])
    dt, nsteps, every = TWO_PI / 1000, 90, 40          # records at 0, 40, 80, 90
    k = {"state": fb.LOG_STATE, "rv": fb.LOG_RV, "energy": fb.LOG_ENERGY}[kind]
    E = fb.from_gen(ens)
    rec = E.integrate_steps_logged(nsteps, dt, every, kind=k, los=(0.3, -1.0, 2.0))
    E.close()
    off = ens.offsets
    lhat = np.array([0.3, -1.0, 2.0]) / np.linalg.norm([0.3, -1.0, 2.0])
    for r, steps in enumerate((0, 40, 80, 90)):
        if steps:
            x, v, _, _ = ora.ensemble_fixed(ens.n_body, ens.mass, ens.pos, ens.vel, dt, steps,
                                            nthreads=threads())
        else:
            x, v = ens.pos, ens.vel
        assert np.allclose(rec[0][:, r], steps * dt, rtol=1e-14, atol=0)
        if kind == "state":
            check(ens, rec[1][r], rec[2][r], x, v, f"record {r}")
        elif kind == "rv":
            for s in range(ens.n_sys):
                m, vs = ens.mass[off[s]:off[s + 1]], v[off[s]:off[s + 1]]
                want = (vs[0] - m @ vs / m.sum()) @ lhat
                scale = np.linalg.norm(vs, axis=1).max()
                assert abs(rec[1][s, r] - want) <= 2 * REL_TOL * scale + 1e-14 * scale, (s, r)
        else:
            er, lr = ora.ensemble_energy(ens.n_body, ens.mass, x, v)
            tol = 1e-12 if r == 0 else 2e-9
            assert np.all(np.abs(rec[1][:, r] - er) <= tol * np.abs(er)), r
            assert np.all(np.linalg.norm(rec[2][:, r] - lr, axis=1) <= tol * np.linalg.norm(lr, axis=1)), r


def test_quanta_are_bitwise_invisible(fb):
    ens = concat([gen.planetesimal_disk(9, 21, seed=89), gen.planetesimal_disk(2, 70, seed=90)])
    out = []
    for q in (0, 23):
        E = fb.from_gen(ens)
        E.integrate_steps(100, TWO_PI / 1000, fb.Opts(steps_per_quantum=q))
        out.append(E.state())
        E.close()
    assert np.array_equal(out[0]["pos"], out[1]["pos"]) and np.array_equal(out[0]["vel"], out[1]["vel"])


def test_autotune_and_server(plans):
    fb = plans
    ens = concat([gen.planetesimal_disk(2, 20, seed=91), gen.three_body(3, seed=92)])
    E = fb.from_gen(ens)
    entries = E.autotune(5, 0.01)                 # tunes the small bucket and the fused launch only
    assert entries and all(e["n"] <= 16 for e in entries)
    assert np.all(E.state()["steps"] == 0)          # state restored after tuning
    E.close()
    with fb.Server() as S:
        with pytest.raises(fb.FewbodyError) as ei:
            S.submit_gen(gen.planetesimal_disk(1, 17, seed=93), 1.0, 0.01)
        assert ei.value.code == fb.E_INVAL


@pytest.mark.parametrize("rule", [1, 2])
def test_adaptive_parity(fb, ora, rule):
    """Adaptive steps (the pairwise rule, or Eq. 5) for 20..130 bodies: the
    same accepted-step counts as the oracle and parity to 1e-10."""
    ens = concat([gen.planetesimal_disk(4, 20, seed=94), gen.planetesimal_disk(3, 41, seed=95),
                  gen.planetesimal_disk(2, 130, seed=96), gen.three_body(6, seed=97)])
    eta = 0.01 if rule == 1 else 1.7e-2
    t_end = 0.5
    say("large-n adaptive", rule)
    E = fb.from_gen(ens)
    E.integrate(t_end, 0.0, fb.Opts(adaptive=rule, eta=eta, steps_per_quantum=7))
    st = E.state()
    E.close()
    assert np.all(st["status"] == fb.DONE) and np.all(st["t"] == t_end)
    off = ens.offsets
    for s in range(ens.n_sys):
        o = ora.integrate_adaptive(*ens.system(s), t_end, eta=eta, stop_rules=0, paper_rule=rule == 2)
        assert o["status"] == ora.DONE and o["steps"] == st["steps"][s], (s, o["steps"], st["steps"][s])
        sl = slice(off[s], off[s + 1])
        check(ens.subset([s]), st["pos"][sl], st["vel"][sl], o["pos"], o["vel"], f"system {s}")


def test_stop_rules(fb, ora):
    """A disk with a body beyond r_eject, one with two bodies inside a
    mutual Hill radius, one with a non-finite-free ordinary run: the same
    status, step count and state as the oracle."""
    base = gen.planetesimal_disk(3, 24, seed=98)
    pos, vel = base.pos.copy(), base.vel.copy()
    off = base.offsets
    pos[off[0] + 5] = [150.0, 0.0, 0.0]            # ejected once it has taken a step
    vel[off[0] + 5] = [0.0, 0.0, 0.0]
    pos[off[1] + 7] = pos[off[1] + 6] + [1e-3, 0.0, 0.0]   # well inside a mutual Hill radius
    vel[off[1] + 7] = vel[off[1] + 6]
    ens = gen.Ensemble(base.n_body, base.mass, pos, vel)
    t_end = 0.3
    E = fb.from_gen(ens)
    E.integrate(t_end, 0.0, fb.Opts(adaptive=1, eta=0.01, stop_rules=3, r_eject=100.0))
    st = E.state()
    E.close()
    assert list(st["status"]) == [fb.EJECTED, fb.ENCOUNTER, fb.DONE]
    for s in range(ens.n_sys):
        o = ora.integrate_adaptive(*ens.system(s), t_end, eta=0.01, stop_rules=3, r_eject=100.0)
        assert o["status"] == st["status"][s] and o["steps"] == st["steps"][s], (s, o["status"], o["steps"])
        sl = slice(off[s], off[s + 1])
        check(ens.subset([s]), st["pos"][sl], st["vel"][sl], o["pos"], o["vel"], f"system {s}")


@pytest.mark.parametrize("compact", [False, True])
def test_persistent_schedule_with_small_and_large_systems(fb, ora, compact):
    """Large systems run as plain launches inside every quantum of the
    persistent schedule: the whole mix matches the oracle, and the large
    systems are bitwise the plain schedule's."""
    ens = concat([gen.ragged_hill(60, seed=99, n_lo=2, n_hi=16), gen.planetesimal_disk(5, 17, seed=100),
                  gen.planetesimal_disk(3, 40, seed=101), gen.planetesimal_disk(2, 130, seed=102)])
    dt, nsteps = TWO_PI / 1000, 120
    say("large-n persistent", compact)
    out = {}
    for sched in (fb.SCHED_PLAIN, fb.SCHED_PERSISTENT):
        E = fb.from_gen(ens)
        E.integrate_steps(nsteps, dt, fb.Opts(schedule=sched, steps_per_quantum=37, compact=compact))
        out[sched] = E.state()
        E.close()
    st = out[fb.SCHED_PERSISTENT]
    assert np.all(st["status"] == fb.DONE) and np.all(st["steps"] == nsteps)
    x, v, _, _ = ora.ensemble_fixed(ens.n_body, ens.mass, ens.pos, ens.vel, dt, nsteps, nthreads=threads())
    check(ens, st["pos"], st["vel"], x, v, "persistent mix")
    big = np.repeat(ens.n_body > 16, ens.n_body)
    assert np.array_equal(st["pos"][big], out[fb.SCHED_PLAIN]["pos"][big])
    assert np.array_equal(st["vel"][big], out[fb.SCHED_PLAIN]["vel"][big])


def test_persistent_adaptive_stop_rules_large_only_and_mixed(fb, ora):
    """Adaptive steps with both stop rules under compaction: an ensemble of
    large systems only (no fused launch at all) and one mixed with small
    systems; statuses, step counts and states against the oracle."""
    base = gen.planetesimal_disk(3, 24, seed=98)
    pos, vel = base.pos.copy(), base.vel.copy()
    off = base.offsets
    pos[off[0] + 5] = [150.0, 0.0, 0.0]
    vel[off[0] + 5] = [0.0, 0.0, 0.0]
    pos[off[1] + 7] = pos[off[1] + 6] + [1e-3, 0.0, 0.0]
    vel[off[1] + 7] = vel[off[1] + 6]
    large = gen.Ensemble(base.n_body, base.mass, pos, vel)
    mixed_ens = concat([large, gen.three_body(20, seed=103), gen.ragged_hill(10, seed=104, n_lo=4, n_hi=8)])
    t_end = 0.3
    opts = fb.Opts(adaptive=1, eta=0.01, stop_rules=3, r_eject=100.0, schedule=fb.SCHED_PERSISTENT,
                   steps_per_quantum=5, compact=True)
    for ens in (large, mixed_ens):
        say("large-n persistent adaptive", ens.n_sys)
        E = fb.from_gen(ens)
        E.integrate(t_end, 0.0, opts)
        st = E.state()
        E.close()
        assert list(st["status"][:3]) == [fb.EJECTED, fb.ENCOUNTER, fb.DONE]
        o_off = ens.offsets
        for s in range(ens.n_sys):
            o = ora.integrate_adaptive(*ens.system(s), t_end, eta=0.01, stop_rules=3, r_eject=100.0)
            assert o["status"] == st["status"][s] and o["steps"] == st["steps"][s], (s, o["status"], o["steps"])
            sl = slice(o_off[s], o_off[s + 1])
            check(ens.subset([s]), st["pos"][sl], st["vel"][sl], o["pos"], o["vel"], f"system {s}")
