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
