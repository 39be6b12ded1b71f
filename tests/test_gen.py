"""Seeded input generators: determinism and the stated distributions."""
import math

import numpy as np

from paper_1208_1157_amd import gen


def _astro_elements(ens):
    """Semi-major axis, eccentricity and inclination of each planet about its star."""
    off = ens.offsets
    out = []
    for s in range(ens.n_sys):
        m, x, v = ens.system(s)
        for i in range(1, len(m)):
            r = x[i] - x[0]
            u = v[i] - v[0]
            mu = m[0] + m[i]
            rn = np.linalg.norm(r)
            a = 1.0 / (2.0 / rn - (u @ u) / mu)
            h = np.cross(r, u)
            evec = np.cross(u, h) / mu - r / rn
            inc = math.degrees(math.acos(h[2] / np.linalg.norm(h)))
            out.append((s, i, a, np.linalg.norm(evec), inc, m[i]))
    return out


def test_three_body_distribution_and_frame():
    ens = gen.three_body(256, seed=0)
    assert ens.n_body.tolist() == [3] * 256
    el = _astro_elements(ens)
    for s, i, a, e, inc, m in el:
        if i == 1:
            assert abs(a - 1.0) < 1e-12
        else:
            assert 1.5 - 1e-12 <= a <= 3.0 + 1e-12
        assert e <= 0.05 + 1e-12
        assert inc <= 2.0 + 1e-9
        assert 1e-5 <= m <= 1e-3
    off = ens.offsets
    for s in range(ens.n_sys):
        sl = slice(off[s], off[s + 1])
        m = ens.mass[sl]
        assert np.abs((m[:, None] * ens.pos[sl]).sum(0)).max() < 1e-15
        assert np.abs((m[:, None] * ens.vel[sl]).sum(0)).max() < 1e-15
    assert ens.mass[0] == 1.0


def test_seeded_and_prefix_stable():
    a = gen.three_body(64, seed=3)
    b = gen.three_body(64, seed=3)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)
    c = gen.three_body(64, seed=4)
    assert not np.array_equal(a.pos, c.pos)


def test_ragged_hill_spacing():
    ens = gen.ragged_hill(200, seed=2)
    assert ens.n_body.min() >= 3 and ens.n_body.max() <= 15
    assert len(set(ens.n_body.tolist())) == 13
    el = _astro_elements(ens)
    by_sys = {}
    for s, i, a, e, inc, m in el:
        by_sys.setdefault(s, []).append((i, a, m, e, inc))
    for s, pl in by_sys.items():
        pl.sort()
        assert abs(pl[0][1] - 1.0) < 1e-12
        for (i0, a0, m0, _, _), (i1, a1, m1, _, _) in zip(pl, pl[1:]):
            rh = ((m0 + m1) / 3.0) ** (1 / 3) * (a0 + a1) / 2
            k = (a1 - a0) / rh
            assert 8.0 - 1e-9 <= k <= 12.0 + 1e-9
        for (_, _, m, e, inc) in pl:
            assert 1e-6 <= m <= 1e-4 and e <= 0.03 + 1e-12 and inc <= 1.0 + 1e-9


def test_workloads_and_trace():
    ens, p = gen.workload("parity_1024x3")
    assert ens.n_sys == 1024 and p["steps"] == 1000 and p["dt"] == 2 * math.pi / 1000
    ens3, p3 = gen.workload("lifetimes_65536x4-8", n_sys=100)
    assert ens3.n_body.min() >= 4 and ens3.n_body.max() <= 8
    tr = gen.serving_trace(50, seed=4)
    arr = np.array([r.arrival for r in tr])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    for r in tr:
        assert 1 <= r.ensemble.n_sys <= 4096
        assert 3 <= r.ensemble.n_body.min() and r.ensemble.n_body.max() <= 10
        assert 2 * math.pi * 10 <= r.t_end <= 2 * math.pi * 1000


def test_paper_ics_circular():
    ens = gen.paper_ics(4, 5)
    for s, i, a, e, inc, m in _astro_elements(ens):
        assert abs(a - 1.4 ** (i - 1)) < 1e-9 * a
        assert e < 1e-9 and m == 1e-3
