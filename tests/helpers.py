"""Shared test helpers: per-system error metrics and oracle drivers."""
import os

import numpy as np

# Parity bar: per system, max_i |x_i^gpu - x_i^ora| / max_i |x_i^ora| (and the
# same for v) must not exceed this over the parity horizon (Section 5.2.1's
# 1e-10 test-mode threshold, read as relative to the system's scale).
REL_TOL = 1e-10


def threads():
    return max(1, min(16, os.cpu_count() or 1))


def per_system_rel_err(n_body, a, b):
    """max_i |a_i - b_i| / max_i |b_i| for each system (rows body-major)."""
    off = np.zeros(len(n_body) + 1, dtype=np.int64)
    np.cumsum(n_body, out=off[1:])
    d = np.linalg.norm(np.asarray(a) - np.asarray(b), axis=1)
    mag = np.linalg.norm(np.asarray(b), axis=1)
    out = np.empty(len(n_body))
    for s in range(len(n_body)):
        sl = slice(off[s], off[s + 1])
        out[s] = d[sl].max() / max(mag[sl].max(), 1e-300)
    return out


def oracle_fixed(ora, ens, h, steps, nthreads=None):
    return ora.ensemble_fixed(ens.n_body, ens.mass, ens.pos, ens.vel, h, steps,
                              nthreads=nthreads or threads())


def assert_parity(n_body, gpu_pos, gpu_vel, ora_pos, ora_vel, tol=REL_TOL, label=""):
    ex = per_system_rel_err(n_body, gpu_pos, ora_pos)
    ev = per_system_rel_err(n_body, gpu_vel, ora_vel)
    worst = int(np.argmax(np.maximum(ex, ev)))
    assert ex.max() <= tol and ev.max() <= tol, (
        f"{label}: parity failed: max rel err x={ex.max():.3e} v={ev.max():.3e} "
        f"(system {worst}, n={n_body[worst]})")
    return ex.max(), ev.max()


# ---------------------------------------------------------------------------
# Adaptive runs: a system whose discrete decisions differ between the GPU and
# the oracle is compared up to its first differing decision, and that decision
# must sit within roundoff-scale reach of its threshold.
# ---------------------------------------------------------------------------
DECISION_MARGIN = 1e-8


def stop_margins(mass, pos, r_eject):
    """Relative distance of the oracle's state to each stop threshold: the
    smallest |sep / R_hill - 1| over planet pairs, R_hill the mutual Hill
    radius ((m_i + m_j) / (3 m0))^(1/3) (r_i + r_j) / 2 with r the distance
    from the star, and the smallest |r / r_eject - 1| over planets."""
    m = np.asarray(mass, dtype=np.float64)
    x = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    r = np.linalg.norm(x[1:] - x[0], axis=1)
    hill = np.inf
    for i in range(1, len(m)):
        for j in range(i + 1, len(m)):
            sep = np.linalg.norm(x[i] - x[j])
            rh = np.cbrt((m[i] + m[j]) / (3.0 * m[0])) * 0.5 * (r[i - 1] + r[j - 1])
            hill = min(hill, abs(sep / rh - 1.0))
    eject = float(np.min(np.abs(r / r_eject - 1.0))) if len(r) else np.inf
    return hill, eject


def explain_adaptive_mismatch(ora, system, t_end, eta, stop_rules, r_eject, paper_rule,
                              rerun, got_status, got_steps, ref, margin=DECISION_MARGIN,
                              tol=REL_TOL, max_steps=10**9, start=None):
    """For one system whose final status or step count differs from the
    oracle's `ref`: rerun both sides up to the step before the first differing
    decision (rerun(k) returns the candidate's dict(pos, vel, t, status, steps)
    after at most k steps), require parity there, then require the criterion
    that flipped to lie within `margin` (relative) of its threshold in the
    oracle's state.  With `start` (t0, acc, jerk, dt_next, steps of a run in
    progress) both sides continue from that state and step counts are
    absolute.  Returns (k1, criterion, its margin); raises AssertionError with
    the numbers otherwise."""
    m, x0, v0 = system
    kw = dict(t_end=t_end, eta=eta, stop_rules=stop_rules, r_eject=r_eject, paper_rule=paper_rule,
              **(start or {}))
    s0 = int((start or {}).get("steps", 0))
    k1 = min(int(got_steps), int(ref["steps"]))
    assert k1 <= max_steps
    events = []
    for st, steps in ((int(got_status), int(got_steps)), (int(ref["status"]), int(ref["steps"]))):
        events.append(st if steps == k1 else ora.ACTIVE)
    assert events[0] != events[1], (k1, events)
    crit = set()
    for ev in events:
        if ev == ora.ENCOUNTER:
            crit.add("hill")
        elif ev == ora.EJECTED:
            crit.add("eject")
        elif ev == ora.STALLED_DT:
            crit.add("stall")
        elif ev in (ora.NONFINITE, ora.MAXSTEPS):
            raise AssertionError(f"decision {ev} at step {k1} cannot differ by roundoff")
    if not crit:
        crit.add("clamp")            # one side took its shortened last step at k1
    pre = k1 - 1
    if pre >= max(1, s0 + 1):
        o_pre = ora.integrate_adaptive(m, x0, v0, max_steps=pre, **kw)
        g_pre = rerun(pre)
        assert o_pre["status"] == ora.MAXSTEPS and o_pre["steps"] == pre, o_pre["status"]
        assert int(g_pre["status"]) == ora.MAXSTEPS and int(g_pre["steps"]) == pre, g_pre["status"]
        n = [len(m)]
        ex = per_system_rel_err(n, g_pre["pos"], o_pre["pos"])[0]
        ev = per_system_rel_err(n, g_pre["vel"], o_pre["vel"])[0]
        et = abs(float(g_pre["t"]) - o_pre["t"]) / max(abs(o_pre["t"]), 1e-300)
        assert ex <= tol and ev <= tol and et <= tol, (
            f"before the first differing decision (step {k1}): rel err x={ex:.3e} v={ev:.3e} t={et:.3e}")
    else:
        o_pre = ora.integrate_adaptive(m, x0, v0, max_steps=s0, **kw)
    o_k1 = ora.integrate_adaptive(m, x0, v0, max_steps=k1, **kw)
    hill, eject = stop_margins(m, o_k1["pos"], r_eject)
    margins = {
        "hill": hill,
        "eject": eject,
        "clamp": abs(o_pre["t"] + o_pre["dt_next"] - t_end) / abs(t_end),
        "stall": abs(o_k1["dt_next"] / (1e-12 * abs(t_end)) - 1.0),
    }
    worst = max(crit, key=lambda c: margins[c])
    assert margins[worst] <= margin, (
        f"decision '{worst}' at step {k1} differs but sits {margins[worst]:.3e} from its threshold "
        f"(events gpu/oracle {events}; margins {margins})")
    return k1, worst, margins[worst]


def gpu_adaptive_rerun(fb, system, t_end, **opts):
    """rerun(k) for explain_adaptive_mismatch: the system alone on the GPU,
    integrated to t_end with the given fb.Opts fields and max_steps = k."""
    m, x, v = system

    def rerun(k):
        E = fb.Ensemble(np.array([len(m)], dtype=np.int32), m, x, v)
        E.integrate(t_end, 0.0, fb.Opts(max_steps=int(k), **opts))
        st = E.state()
        E.close()
        return {"pos": st["pos"], "vel": st["vel"], "t": float(st["t"][0]),
                "status": int(st["status"][0]), "steps": int(st["steps"][0])}
    return rerun


def check_adaptive_systems(fb, ora, ens, idx, st, t_end, eta, stop_rules, r_eject, paper_rule,
                           refs=None, tol=REL_TOL, max_steps=10**9):
    """Every system s in idx: if its status and step count equal the oracle's,
    parity to tol (and t == t_end when done); otherwise its first differing
    decision is explained (explain_adaptive_mismatch).  Returns (agree,
    flipped, worst error, list of flips) and raises with the counts."""
    off = ens.offsets
    agree, flips, worst = 0, [], 0.0
    for s in idx:
        s = int(s)
        system = ens.system(s)
        o = refs[s] if refs is not None else ora.integrate_adaptive(
            *system, t_end=t_end, eta=eta, stop_rules=stop_rules, r_eject=r_eject, paper_rule=paper_rule,
            max_steps=max_steps)
        sl = slice(off[s], off[s + 1])
        if o["status"] == st["status"][s] and o["steps"] == st["steps"][s]:
            agree += 1
            n = [len(system[0])]
            ex = per_system_rel_err(n, st["pos"][sl], o["pos"])[0]
            ev = per_system_rel_err(n, st["vel"][sl], o["vel"])[0]
            worst = max(worst, ex, ev)
            assert ex <= tol and ev <= tol, (
                f"system {s}: rel err x={ex:.3e} v={ev:.3e} (agree so far {agree}, flips {len(flips)})")
            if o["status"] == ora.DONE:
                assert st["t"][s] == t_end, (s, st["t"][s])
            continue
        rerun = gpu_adaptive_rerun(fb, system, t_end, adaptive=2 if paper_rule else 1, eta=eta,
                                   stop_rules=stop_rules, r_eject=r_eject)
        try:
            k1, crit, margin = explain_adaptive_mismatch(
                ora, system, t_end, eta, stop_rules, r_eject, paper_rule, rerun,
                st["status"][s], st["steps"][s], o, tol=tol, max_steps=max_steps)
        except AssertionError as exc:
            raise AssertionError(f"system {s} (gpu {st['status'][s]}/{st['steps'][s]}, oracle "
                                 f"{o['status']}/{o['steps']}; agree {agree}, flips {len(flips)}): {exc}")
        flips.append((s, k1, crit, margin))
    return agree, len(flips), worst, flips


def explain_rkck_mismatch(ora, system, t_end, eps, dt0, rerun, got_steps, ref, margin=DECISION_MARGIN,
                          tol=REL_TOL):
    """Adaptive Runge-Kutta Cash-Karp: for one system whose accepted-step
    count differs from the oracle's, find the first accepted step k* after
    which the two sides' times differ (bisection over max_steps; a trial
    accepted on one side and rejected on the other, or a last step clamped on
    one side only, shows in t at once), require parity of the state and time
    after k* - 1 steps, then require that one of step k*'s decisions in the
    oracle's state -- the acceptance of each trial (error norm E against 1) or
    the clamp onto t_end -- lies within `margin` of its threshold.  rerun(k)
    returns the candidate's dict(pos, vel, t, steps) after at most k accepted
    steps.  Returns (k*, criterion, margin)."""
    m, x0, v0 = system
    k1 = min(int(got_steps), int(ref["steps"]))

    def ora_at(k):
        return ora.integrate_rkck_adaptive(m, x0, v0, t_end, eps, dt0, max_steps=k)

    def same_t(k):
        a, b = rerun(k), ora_at(k)
        return abs(float(a["t"]) - b["t"]) <= 1e-12 * max(abs(b["t"]), 1e-300)

    if same_t(k1):
        # identical through step k1: the side that stopped there clamped its
        # step k1 onto t_end and the other did not
        kstar = k1
    else:
        lo, hi = 0, k1              # same t after lo steps, different after hi
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if same_t(mid):
                lo = mid
            else:
                hi = mid
        kstar = hi
    a, b = rerun(kstar - 1), ora_at(kstar - 1)
    n = [len(m)]
    ex = per_system_rel_err(n, a["pos"], b["pos"])[0]
    ev = per_system_rel_err(n, a["vel"], b["vel"])[0]
    assert ex <= tol and ev <= tol, (
        f"before the first differing decision (step {kstar}): rel err x={ex:.3e} v={ev:.3e}")
    # step k*'s decisions in the oracle's state: its trials, then the clamp
    t, h = b["t"], b["dt_next"]
    margins = {}
    x, v = b["pos"], b["vel"]
    margins["clamp"] = float("inf")
    for trial in range(64):
        last = t + h >= t_end
        margins["clamp"] = min(margins["clamp"], abs(t + h - t_end) / abs(t_end))
        hh = t_end - t if last else h
        _, _, exr, evr = ora.rkck_step(m, x, v, hh)
        E = ora.rkck_error_norm(x, v, exr, evr, eps)
        margins[f"accept trial {trial}"] = abs(E - 1.0)
        if E <= 1.0:
            break
        h = hh * max(0.1, 0.9 * E ** -0.25)
    crit = min(margins, key=margins.get)
    assert margins[crit] <= margin, (
        f"step {kstar} differs but no decision sits within {margin:g} of its threshold: {margins}")
    return kstar, crit, margins[crit]
