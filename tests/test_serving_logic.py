"""Host-side serving arithmetic (no GPU): percentiles and step schedules."""
import math

import numpy as np

from paper_1208_1157_amd import serve


def test_nearest_rank():
    v = [5.0, 1.0, 4.0, 2.0, 3.0]
    assert serve.nearest_rank(v, 50) == 3.0
    assert serve.nearest_rank(v, 99) == 5.0
    assert serve.nearest_rank(v, 20) == 1.0
    assert serve.nearest_rank(list(range(1, 101)), 99) == 99
    assert math.isnan(serve.nearest_rank([], 50))


def test_request_steps_matches_stepping():
    rng = np.random.default_rng(0)
    dt = 2 * math.pi / 1000
    for _ in range(200):
        t_end = 2 * math.pi * 10 ** rng.uniform(-1, 1.5)
        n = serve.request_steps(t_end, dt)
        # whole steps k*dt <= t_end, plus one short step unless the remainder is negligible
        whole = int(math.floor(t_end / dt))
        while whole * dt > t_end:
            whole -= 1
        rem = t_end - whole * dt
        assert n == whole + (1 if rem > 1e-9 * dt else 0)
    assert serve.request_steps(5 * dt, dt) in (5, 6)
    assert serve.request_steps(0.0, dt) == 0
