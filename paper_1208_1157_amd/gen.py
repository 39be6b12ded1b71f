"""Seeded synthetic planetary ensembles.

This module only builds inputs: masses, positions and velocities of many
independent star + planets systems, plus the request trace of the serving
workload.  It holds none of the integrator's arithmetic, so both the CPU
oracle and the HIP path can consume what it returns.

Conventions (Section 2.1 of the paper: G = 1, the inner orbit has period
2*pi when m0 = 1 and a = 1):

* body 0 of every system is the central star, m0 = 1;
* planets start on Keplerian orbits about the star, built from astrocentric
  elements with mu = m0 + m_i, then the whole system is shifted to its
  barycentric frame (zero total momentum, centre of mass at the origin);
* "log-uniform on [a, b]" means 10**U(log10 a, log10 b);
* angles given in degrees are converted to radians;
* Kepler's equation M -> E is solved by Newton iteration to |dE| < 1e-15.

Systems are ragged: ``n_body[s]`` bodies each, body ``b`` of system ``s``
sits at flat index ``off[s] + b`` with ``off`` the exclusive prefix sum.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Ensemble:
    """Host-side ragged ensemble (flat, body-major arrays, float64)."""

    n_body: np.ndarray            # int32 [n_sys]
    mass: np.ndarray              # float64 [N]
    pos: np.ndarray               # float64 [N, 3]
    vel: np.ndarray               # float64 [N, 3]
    meta: dict = field(default_factory=dict)

    @property
    def n_sys(self) -> int:
        return int(self.n_body.shape[0])

    @property
    def offsets(self) -> np.ndarray:
        off = np.zeros(self.n_sys + 1, dtype=np.int64)
        np.cumsum(self.n_body, out=off[1:])
        return off

    def system(self, s: int):
        off = self.offsets
        a, b = int(off[s]), int(off[s + 1])
        return self.mass[a:b].copy(), self.pos[a:b].copy(), self.vel[a:b].copy()

    def subset(self, idx) -> "Ensemble":
        idx = np.asarray(idx, dtype=np.int64)
        off = self.offsets
        rows = np.concatenate([np.arange(off[s], off[s + 1]) for s in idx]) if len(idx) else np.zeros(0, np.int64)
        return Ensemble(self.n_body[idx].astype(np.int32), self.mass[rows].copy(),
                        self.pos[rows].copy(), self.vel[rows].copy(), dict(self.meta))


def _log_uniform(rng, lo, hi, size):
    return 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size)


def _solve_kepler(M, e):
    """Eccentric anomaly E with E - e sin E = M (elliptic, e < 1), vectorised Newton."""
    M = np.asarray(M, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(100):
        f = E - e * np.sin(E) - M
        dE = -f / (1.0 - e * np.cos(E))
        E = E + dE
        if np.all(np.abs(dE) < 1e-15):
            break
    return E


def elements_to_cartesian(mu, a, e, inc, node, peri, M):
    """Astrocentric Keplerian elements -> position and velocity (vectorised)."""
    E = _solve_kepler(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = a * np.sqrt(1.0 - e * e)
    X = a * (cE - e)
    Y = b * sE
    Edot = np.sqrt(mu / a ** 3) / (1.0 - e * cE)
    VX = -a * sE * Edot
    VY = b * cE * Edot
    cO, sO = np.cos(node), np.sin(node)
    cw, sw = np.cos(peri), np.sin(peri)
    ci, si = np.cos(inc), np.sin(inc)
    # rows of R = Rz(node) Rx(inc) Rz(peri), first two columns only
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si], axis=-1)
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si], axis=-1)
    pos = X[..., None] * P + Y[..., None] * Q
    vel = VX[..., None] * P + VY[..., None] * Q
    return pos, vel


def _assemble(n_body, m_pl, a, e, inc, node, peri, M, m0=1.0):
    """Padded planet element arrays [n_sys, n_max-1] -> barycentric ragged Ensemble."""
    n_sys, npl_max = m_pl.shape
    npl = n_body - 1
    valid = np.arange(npl_max)[None, :] < npl[:, None]
    mu = m0 + m_pl
    a_safe = np.where(valid, a, 1.0)
    e_safe = np.where(valid, e, 0.0)
    pos_pl, vel_pl = elements_to_cartesian(mu, a_safe, e_safe, inc, node, peri, M)
    m_full = np.zeros((n_sys, npl_max + 1))
    m_full[:, 0] = m0
    m_full[:, 1:] = np.where(valid, m_pl, 0.0)
    pos_full = np.zeros((n_sys, npl_max + 1, 3))
    vel_full = np.zeros((n_sys, npl_max + 1, 3))
    pos_full[:, 1:] = np.where(valid[..., None], pos_pl, 0.0)
    vel_full[:, 1:] = np.where(valid[..., None], vel_pl, 0.0)
    mtot = m_full.sum(axis=1)
    com = (m_full[..., None] * pos_full).sum(axis=1) / mtot[:, None]
    vcom = (m_full[..., None] * vel_full).sum(axis=1) / mtot[:, None]
    pos_full -= com[:, None, :]
    vel_full -= vcom[:, None, :]
    keep = np.arange(npl_max + 1)[None, :] < n_body[:, None]
    return Ensemble(n_body.astype(np.int32), m_full[keep].copy(),
                    pos_full[keep].copy(), vel_full[keep].copy())


def _hill_spaced(rng, m_pl, valid, k_lo, k_hi, m0=1.0):
    """a_1 = 1; a_{k+1} = a_k (1+h)/(1-h), h = (K/2) ((m_k+m_{k+1})/(3 m0))^(1/3), K ~ U[k_lo,k_hi]."""
    n_sys, npl_max = m_pl.shape
    a = np.ones((n_sys, npl_max))
    K = rng.uniform(k_lo, k_hi, (n_sys, max(npl_max - 1, 0)))
    for k in range(1, npl_max):
        h = 0.5 * K[:, k - 1] * np.cbrt((m_pl[:, k - 1] + m_pl[:, k]) / (3.0 * m0))
        a[:, k] = a[:, k - 1] * (1.0 + h) / (1.0 - h)
    return np.where(valid, a, 1.0)


def _draw_planets(rng, n_body, mlo, mhi, e_hi, inc_deg_hi, spacing):
    n_sys = n_body.shape[0]
    npl_max = int(n_body.max()) - 1
    valid = np.arange(npl_max)[None, :] < (n_body - 1)[:, None]
    shape = (n_sys, npl_max)
    m_pl = np.where(valid, _log_uniform(rng, mlo, mhi, shape), 0.0)
    if spacing == "two-planet":
        a = np.ones(shape)
        a[:, 1] = rng.uniform(1.5, 3.0, n_sys)
    elif spacing[0] == "annulus":
        a = rng.uniform(spacing[1], spacing[2], shape)
    else:
        a = _hill_spaced(rng, m_pl, valid, *spacing)
    e = rng.uniform(0.0, e_hi, shape)
    inc = np.radians(rng.uniform(0.0, inc_deg_hi, shape))
    node = rng.uniform(0.0, TWO_PI, shape)
    peri = rng.uniform(0.0, TWO_PI, shape)
    M = rng.uniform(0.0, TWO_PI, shape)
    return _assemble(n_body, m_pl, a, e, inc, node, peri, M)


def three_body(n_sys: int, seed: int) -> Ensemble:
    """Star + two planets: m ~ logU[1e-5,1e-3], a1 = 1, a2 ~ U[1.5,3], e ~ U[0,0.05], i ~ U[0,2 deg]."""
    rng = np.random.default_rng(seed)
    n_body = np.full(n_sys, 3, dtype=np.int32)
    ens = _draw_planets(rng, n_body, 1e-5, 1e-3, 0.05, 2.0, "two-planet")
    ens.meta = {"family": "three_body", "seed": seed}
    return ens


def ragged_hill(n_sys: int, seed: int, n_lo=3, n_hi=15, mlo=1e-6, mhi=1e-4,
                k_lo=8.0, k_hi=12.0, e_hi=0.03, inc_deg_hi=1.0) -> Ensemble:
    """Body counts uniform on n_lo..n_hi; Hill-spaced planets (a_1 = 1, K mutual Hill radii)."""
    rng = np.random.default_rng(seed)
    n_body = rng.integers(n_lo, n_hi + 1, n_sys).astype(np.int32)
    ens = _draw_planets(rng, n_body, mlo, mhi, e_hi, inc_deg_hi, (k_lo, k_hi))
    ens.meta = {"family": "ragged_hill", "seed": seed, "n_range": [n_lo, n_hi]}
    return ens


def planetesimal_disk(n_sys: int, n: int, seed: int, mlo=1e-9, mhi=1e-7, a_lo=1.0, a_hi=3.0,
                      e_hi=0.02, inc_deg_hi=1.0) -> Ensemble:
    """Star + (n-1) small bodies (large-n systems): m ~ logU[mlo, mhi], a ~ U[a_lo, a_hi],
    e ~ U[0, e_hi], i ~ U[0, inc_deg_hi deg], node/peri/M ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    n_body = np.full(n_sys, n, dtype=np.int32)
    ens = _draw_planets(rng, n_body, mlo, mhi, e_hi, inc_deg_hi, ("annulus", a_lo, a_hi))
    ens.meta = {"family": "planetesimal_disk", "seed": seed, "n": n}
    return ens


def paper_ics(n_sys: int, n: int, planet_mass=1e-3, alpha=0.4) -> Ensemble:
    """Section 5.1's standard set: equal-mass planets on circular coplanar orbits, a_i = (1+alpha)^(i-1)."""
    n_body = np.full(n_sys, n, dtype=np.int32)
    npl = n - 1
    shape = (n_sys, npl)
    m_pl = np.full(shape, planet_mass)
    a = np.broadcast_to((1.0 + alpha) ** np.arange(npl), shape).copy()
    z = np.zeros(shape)
    ens = _assemble(n_body, m_pl, a, z, z, z, z, z)
    ens.meta = {"family": "paper_ics", "n": n}
    return ens


# ---------------------------------------------------------------------------
# Named workloads (sizes and distributions of the benchmark configurations)
# ---------------------------------------------------------------------------

H_INNER_1000 = TWO_PI / 1000.0
H_INNER_2000 = TWO_PI / 2000.0


def workload(name: str, n_sys: int | None = None):
    """Return (Ensemble, params) for a named workload; n_sys trims the system count."""
    if name == "parity_1024x3":
        ens = three_body(n_sys or 1024, seed=0)
        return ens, {"dt": H_INNER_1000, "steps": 1000}
    if name == "homog_131072x3":
        ens = three_body(n_sys or 131072, seed=1)
        return ens, {"dt": H_INNER_1000, "steps": 100000}
    if name == "ragged_65536x3-15":
        ens = ragged_hill(n_sys or 65536, seed=2)
        return ens, {"dt": H_INNER_2000, "steps": 20000}
    if name == "lifetimes_65536x4-8":
        ens = ragged_hill(n_sys or 65536, seed=3, n_lo=4, n_hi=8, mlo=1e-5, mhi=1e-3,
                          k_lo=3.0, k_hi=6.0, e_hi=0.2, inc_deg_hi=1.0)
        return ens, {"eta": 0.01, "t_end": TWO_PI * 1e4, "r_eject": 100.0}
    if name.startswith("disk_"):          # disk_<n_sys>x<n>: large-n planetesimal disks
        ns, n = (int(v) for v in name[5:].split("x"))
        ens = planetesimal_disk(n_sys or ns, n, seed=5)
        return ens, {"dt": H_INNER_1000, "steps": 1000}
    raise KeyError(name)


@dataclass
class Request:
    arrival: float        # seconds since trace start
    ensemble: Ensemble
    t_end: float
    dt: float


def serving_trace(n_req: int = 2000, rate: float = 200.0, seed: int = 4,
                  max_sys: int = 4096, n_lo=3, n_hi=10) -> list[Request]:
    """Poisson arrivals; each request 1..max_sys systems (discrete log-uniform) of n_lo..n_hi
    bodies drawn per system with the ragged_hill parameters; t_end = 2 pi 10^U(1,3); dt = 2 pi/1000."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_req)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = np.floor(10.0 ** rng.uniform(0.0, math.log10(max_sys + 1), n_req)).astype(np.int64)
    sizes = np.clip(sizes, 1, max_sys)
    t_end = TWO_PI * 10.0 ** rng.uniform(1.0, 3.0, n_req)
    seeds = rng.integers(0, 2**63 - 1, n_req)
    out = []
    for r in range(n_req):
        ens = ragged_hill(int(sizes[r]), seed=int(seeds[r]), n_lo=n_lo, n_hi=n_hi)
        out.append(Request(float(arrivals[r]), ens, float(t_end[r]), H_INNER_1000))
    return out
