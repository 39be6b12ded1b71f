"""Autotuner on the GPU: it installs one plan per body count and for the
persistent launch, leaves the ensemble's state untouched, and integration
with the installed plans still matches the oracle."""
import math
import sys

import numpy as np
import pytest

from paper_1208_1157_amd import gen
from tests.helpers import assert_parity, oracle_fixed

pytestmark = pytest.mark.gpu
H = 2 * math.pi / 2000


def test_autotune_restores_state_and_installs_plans(plans, ora):
    fb = plans
    ens = gen.ragged_hill(600, seed=13, n_lo=3, n_hi=9)
    print("[case] autotune 600 ragged", file=sys.stderr, flush=True)
    E = fb.from_gen(ens)
    E.integrate_steps(10, H)
    before = E.state()
    hb = E.hermite_state()
    entries = E.autotune(24, H)
    after = E.state()
    ha = E.hermite_state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    for x, y in zip(hb, ha):
        assert np.array_equal(x, y)
    present = sorted(set(int(n) for n in ens.n_body))
    for n in present:
        chosen = [e for e in entries if e["n"] == n and e["chosen"]]
        assert len(chosen) == 1, n
        m, w, _ = fb.get_plan(n)
        assert (m, w) == (chosen[0]["mapping"], chosen[0]["waves_per_group"])
        assert all(e["ms"] > 0 for e in entries if e["n"] == n)
    pers = [e for e in entries if e["n"] == 0 and e["chosen"]]
    assert len(pers) == 1
    assert fb.get_plan(0)[1:] == (pers[0]["waves_per_group"], pers[0]["groups_per_cu"])
    E.integrate_steps(190, H, fb.Opts(schedule=fb.SCHED_PERSISTENT, steps_per_quantum=64))
    st = E.state()
    E.close()
    X, V, _, _ = oracle_fixed(ora, ens, H, 200)
    assert_parity(ens.n_body, st["pos"], st["vel"], X, V, label="after autotune")
