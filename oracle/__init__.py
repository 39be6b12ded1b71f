"""CPU oracle for the fewbody integrators -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``hermite_oracle.c``, ``mvs_oracle.c`` and
``rkck_oracle.c`` (plain FP64 C, built with ``-O2 -ffp-contract=off``).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does.  It shares no code with the HIP path: the only inputs both sides
see come from the seeded generators.

Every routine works on one system with bodies in rows (body 0 = star):
``mass[n]``, ``pos[n, 3]``, ``vel[n, 3]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "hermite_oracle.c"), os.path.join(HERE, "mvs_oracle.c"),
        os.path.join(HERE, "rkck_oracle.c")]
LIB = os.environ.get("FEWBODY_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

ACTIVE, DONE, ENCOUNTER, EJECTED, NONFINITE, STALLED_DT, MAXSTEPS, UNBOUND = range(8)
STOP_ENCOUNTER, STOP_EJECT = 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64, no contraction)."""
    stale = not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(s) for s in SRCS)
    if force or stale:
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-fPIC", "-shared", "-o", tmp, *SRCS, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        d, i, l, p = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        L.ora_accjerk.argtypes = [i, p, p, p, p, p]
        L.ora_predict.argtypes = [i, d, p, p, p, p, p, p]
        L.ora_correct.argtypes = [i, d, p, p, p, p, p, p, p, p]
        L.ora_integrate_fixed.argtypes = [i, p, p, p, p, p, d, l, i, i]
        L.ora_integrate_fixed.restype = i
        L.ora_energy.argtypes = [i, p, p, p, p, p]
        L.ora_pair_timestep.argtypes = [i, p, p, p, d]
        L.ora_pair_timestep.restype = d
        L.ora_paper_timestep.argtypes = [i, p, p, d]
        L.ora_paper_timestep.restype = d
        L.ora_check_stop.argtypes = [i, p, p, p, i, d]
        L.ora_check_stop.restype = i
        L.ora_integrate_adaptive.argtypes = [i, p, p, p, p, p, p, d, d, i, d, l, p, p, i]
        L.ora_integrate_adaptive.restype = i
        L.ora_ensemble_fixed.argtypes = [i, p, p, p, p, p, p, d, l, i, i, i]
        L.ora_ensemble_fixed.restype = i
        L.ora_ensemble_energy.argtypes = [i, p, p, p, p, p, p]
        L.ora_ensemble_energy.restype = i
        L.ora_mvs_to_helio.argtypes = [i, p, p, p, p, p, p, p]
        L.ora_mvs_from_helio.argtypes = [i, p, p, p, p, p, p, p]
        L.ora_kepler_drift.argtypes = [d, p, p, d]
        L.ora_kepler_drift.restype = i
        L.ora_mvs_kick_acc.argtypes = [i, p, p, p]
        L.ora_mvs_step.argtypes = [i, p, p, p, p, p, d]
        L.ora_mvs_step.restype = i
        L.ora_integrate_mvs.argtypes = [i, p, p, p, d, l, p]
        L.ora_integrate_mvs.restype = i
        L.ora_rk_acc.argtypes = [i, p, p, p]
        L.ora_rkck_step.argtypes = [i, p, p, p, d, p, p, p, p]
        L.ora_integrate_rkck_fixed.argtypes = [i, p, p, p, d, l]
        L.ora_integrate_rkck_fixed.restype = i
        L.ora_rkck_error_norm.argtypes = [i, p, p, p, p, d]
        L.ora_rkck_error_norm.restype = d
        L.ora_integrate_rkck_adaptive.argtypes = [i, p, p, p, p, d, d, p, l, p, p]
        L.ora_integrate_rkck_adaptive.restype = i
        _lib = L
    return _lib


def _f64(a, shape=None):
    out = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        out = out.reshape(shape)
    return out


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def accjerk(mass, pos, vel):
    """Acceleration and jerk of every body (Eq. 1 and its time derivative)."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)), _f64(vel, (n, 3))
    a, j = np.zeros((n, 3)), np.zeros((n, 3))
    lib().ora_accjerk(n, _p(m), _p(x), _p(v), _p(a), _p(j))
    return a, j


def predict(h, x0, v0, a0, j0):
    n = np.asarray(x0).reshape(-1, 3).shape[0]
    arrs = [_f64(z, (n, 3)) for z in (x0, v0, a0, j0)]
    xp, vp = np.zeros((n, 3)), np.zeros((n, 3))
    lib().ora_predict(n, float(h), *[_p(z) for z in arrs], _p(xp), _p(vp))
    return xp, vp


def correct(h, xp, vp, a0, j0, ak, jk):
    n = np.asarray(xp).reshape(-1, 3).shape[0]
    arrs = [_f64(z, (n, 3)) for z in (xp, vp, a0, j0, ak, jk)]
    xc, vc = np.zeros((n, 3)), np.zeros((n, 3))
    lib().ora_correct(n, float(h), *[_p(z) for z in arrs], _p(xc), _p(vc))
    return xc, vc


def integrate_fixed(mass, pos, vel, h, nsteps, n_corr=2, acc=None, jerk=None,
                    converged=False):
    """Fixed-step P(EC)^n_corr integration of one system.

    If ``acc``/``jerk`` are None the set-up evaluation computes them.
    Returns (pos, vel, acc0, jerk0) after ``nsteps`` steps."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)).copy(), _f64(vel, (n, 3)).copy()
    flags = 0
    if acc is None or jerk is None:
        a, j = np.zeros((n, 3)), np.zeros((n, 3))
        flags |= 1
    else:
        a, j = _f64(acc, (n, 3)).copy(), _f64(jerk, (n, 3)).copy()
    if converged:
        flags |= 2
    rc = lib().ora_integrate_fixed(n, _p(m), _p(x), _p(v), _p(a), _p(j), float(h),
                                   int(nsteps), int(n_corr), flags)
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return x, v, a, j


def energy(mass, pos, vel):
    """(E, L[3]) of one system: Eq. 6 with pairs counted once, L = sum m x cross v."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)), _f64(vel, (n, 3))
    e = np.zeros(1)
    L = np.zeros(3)
    lib().ora_energy(n, _p(m), _p(x), _p(v), _p(e), _p(L))
    return float(e[0]), L


def pair_timestep(mass, pos, vel, eta):
    m = _f64(mass)
    n = m.shape[0]
    return lib().ora_pair_timestep(n, _p(m), _p(_f64(pos, (n, 3))), _p(_f64(vel, (n, 3))), float(eta))


def check_stop(mass, pos, vel, stop_rules=3, r_eject=100.0):
    m = _f64(mass)
    n = m.shape[0]
    return lib().ora_check_stop(n, _p(m), _p(_f64(pos, (n, 3))), _p(_f64(vel, (n, 3))),
                                int(stop_rules), float(r_eject))


def paper_timestep(acc, jerk, tau):
    """Eq. 5: tau [sum_i |j_i|^2/|a_i|^2]^(-1/2)."""
    a = _f64(acc).reshape(-1, 3)
    j = _f64(jerk).reshape(-1, 3)
    return lib().ora_paper_timestep(a.shape[0], _p(a), _p(j), float(tau))


def integrate_adaptive(mass, pos, vel, t_end, eta=0.01, stop_rules=3, r_eject=100.0,
                       max_steps=10**9, t0=0.0, paper_rule=False, acc=None, jerk=None,
                       dt_next=None, steps=0):
    """Adaptive integration of one system to t_end or a stop rule.

    paper_rule selects Eq. 5 (eta is tau) instead of the pairwise rule.  With
    acc, jerk and dt_next given (a previous call's results) the run continues
    from them instead of the set-up evaluation; steps counts on from `steps`.
    Returns dict(pos, vel, acc, jerk, t, dt_next, steps, status)."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)).copy(), _f64(vel, (n, 3)).copy()
    flags = 2 if paper_rule else 0
    if acc is None or jerk is None or dt_next is None:
        a, j = np.zeros((n, 3)), np.zeros((n, 3))
        dtn = np.zeros(1)
        flags |= 1
    else:
        a, j = _f64(acc, (n, 3)).copy(), _f64(jerk, (n, 3)).copy()
        dtn = np.array([dt_next], dtype=np.float64)
    t = np.array([t0], dtype=np.float64)
    steps = np.array([steps], dtype=np.int64)
    st = lib().ora_integrate_adaptive(n, _p(m), _p(x), _p(v), _p(a), _p(j), _p(t), float(t_end),
                                      float(eta), int(stop_rules), float(r_eject), int(max_steps),
                                      _p(dtn), _p(steps), flags)
    return {"pos": x, "vel": v, "acc": a, "jerk": j, "t": float(t[0]), "dt_next": float(dtn[0]),
            "steps": int(steps[0]), "status": int(st)}


def ensemble_fixed(n_body, mass, pos, vel, h, nsteps, n_corr=2, nthreads=1):
    """Integrate a ragged ensemble (flat arrays) for nsteps fixed steps.

    Returns (pos, vel, acc0, jerk0) as new flat arrays."""
    nb = np.ascontiguousarray(n_body, dtype=np.int32)
    m = _f64(mass)
    N = m.shape[0]
    x, v = _f64(pos, (N, 3)).copy(), _f64(vel, (N, 3)).copy()
    a, j = np.zeros((N, 3)), np.zeros((N, 3))
    rc = lib().ora_ensemble_fixed(int(nb.shape[0]), _p(nb), _p(m), _p(x), _p(v), _p(a), _p(j),
                                  float(h), int(nsteps), int(n_corr), 1, int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return x, v, a, j


def ensemble_energy(n_body, mass, pos, vel):
    nb = np.ascontiguousarray(n_body, dtype=np.int32)
    m = _f64(mass)
    N = m.shape[0]
    E = np.zeros(nb.shape[0])
    L = np.zeros((nb.shape[0], 3))
    rc = lib().ora_ensemble_energy(int(nb.shape[0]), _p(nb), _p(m), _p(_f64(pos, (N, 3))),
                                   _p(_f64(vel, (N, 3))), _p(E), _p(L))
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return E, L


# ---------------------------------------------------------------- MVS
def mvs_to_helio(mass, pos, vel):
    """(Q, V, X, Vc): heliocentric planet positions and barycentric velocities
    (row 0 zero), centre of mass and its velocity (mvs_oracle.c)."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)), _f64(vel, (n, 3))
    Q, V, X, Vc = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(3), np.zeros(3)
    lib().ora_mvs_to_helio(n, _p(m), _p(x), _p(v), _p(Q), _p(V), _p(X), _p(Vc))
    return Q, V, X, Vc


def mvs_from_helio(mass, Q, V, X, Vc):
    m = _f64(mass)
    n = m.shape[0]
    Q, V, X, Vc = _f64(Q, (n, 3)), _f64(V, (n, 3)), _f64(X), _f64(Vc)
    x, v = np.zeros((n, 3)), np.zeros((n, 3))
    lib().ora_mvs_from_helio(n, _p(m), _p(Q), _p(V), _p(X), _p(Vc), _p(x), _p(v))
    return x, v


def kepler_drift(mu, r, v, dt):
    """(r, v) after dt on the Kepler orbit about mu, or None if unbound."""
    r, v = _f64(r).copy(), _f64(v).copy()
    rc = lib().ora_kepler_drift(float(mu), _p(r), _p(v), float(dt))
    return None if rc != 0 else (r, v)


def mvs_kick_acc(mass, Q):
    m = _f64(mass)
    n = m.shape[0]
    Q = _f64(Q, (n, 3))
    acc = np.zeros((n, 3))
    lib().ora_mvs_kick_acc(n, _p(m), _p(Q), _p(acc))
    return acc


def mvs_step(mass, Q, V, X, Vc, dt):
    """One MVS step in place on copies; returns (status, Q, V, X)."""
    m = _f64(mass)
    n = m.shape[0]
    Q, V, X = _f64(Q, (n, 3)).copy(), _f64(V, (n, 3)).copy(), _f64(X).copy()
    Vc = _f64(Vc)
    st = lib().ora_mvs_step(n, _p(m), _p(Q), _p(V), _p(X), _p(Vc), float(dt))
    return st, Q, V, X


def integrate_mvs(mass, pos, vel, dt, nsteps):
    """nsteps MVS steps of dt on inertial pos/vel; returns dict(pos, vel, status, steps)."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)).copy(), _f64(vel, (n, 3)).copy()
    done = ctypes.c_long()
    st = lib().ora_integrate_mvs(n, _p(m), _p(x), _p(v), float(dt), int(nsteps), ctypes.byref(done))
    return {"pos": x, "vel": v, "status": st, "steps": done.value}


# ---------------------------------------------------------------- RKCK
def rk_acc(mass, pos):
    m = _f64(mass)
    n = m.shape[0]
    x = _f64(pos, (n, 3))
    a = np.zeros((n, 3))
    lib().ora_rk_acc(n, _p(m), _p(x), _p(a))
    return a


def rkck_step(mass, pos, vel, h):
    """One Cash-Karp step: (x5, v5, err_x, err_v)."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)), _f64(vel, (n, 3))
    x5, v5, ex, ev = (np.zeros((n, 3)) for _ in range(4))
    lib().ora_rkck_step(n, _p(m), _p(x), _p(v), float(h), _p(x5), _p(v5), _p(ex), _p(ev))
    return x5, v5, ex, ev


def rkck_error_norm(pos, vel, err_x, err_v, eps):
    x = _f64(pos).reshape(-1, 3)
    n = x.shape[0]
    v, ex, ev = _f64(vel, (n, 3)), _f64(err_x, (n, 3)), _f64(err_v, (n, 3))
    return float(lib().ora_rkck_error_norm(n, _p(x), _p(v), _p(ex), _p(ev), float(eps)))


def integrate_rkck_fixed(mass, pos, vel, h, nsteps):
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)).copy(), _f64(vel, (n, 3)).copy()
    st = lib().ora_integrate_rkck_fixed(n, _p(m), _p(x), _p(v), float(h), int(nsteps))
    if st < 0:
        raise ValueError("oracle rejected arguments")
    return {"pos": x, "vel": v, "status": st}


def integrate_rkck_adaptive(mass, pos, vel, t_end, eps, dt, t0=0.0, max_steps=10**9):
    """Adaptive Cash-Karp to t_end from t0 with first trial step dt; returns
    dict(pos, vel, t, status, steps, rejects, dt_next)."""
    m = _f64(mass)
    n = m.shape[0]
    x, v = _f64(pos, (n, 3)).copy(), _f64(vel, (n, 3)).copy()
    t = ctypes.c_double(t0)
    h = ctypes.c_double(dt)
    steps, rej = ctypes.c_long(), ctypes.c_long()
    st = lib().ora_integrate_rkck_adaptive(n, _p(m), _p(x), _p(v), ctypes.byref(t), float(t_end),
                                           float(eps), ctypes.byref(h), int(max_steps),
                                           ctypes.byref(steps), ctypes.byref(rej))
    if st < 0:
        raise ValueError("oracle rejected arguments")
    return {"pos": x, "vel": v, "t": t.value, "status": st, "steps": steps.value,
            "rejects": rej.value, "dt_next": h.value}
