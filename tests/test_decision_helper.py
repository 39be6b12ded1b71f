"""CPU checks of the adaptive-parity helper the GPU tests use to explain a
system whose discrete decisions differ: it must accept a flip at a last-bit
threshold (after verifying parity up to it) and reject a flip far from one.
The candidate side here is the oracle itself, run with a perturbed setting."""
import numpy as np
import pytest

from paper_1208_1157_amd import gen
from tests.helpers import explain_adaptive_mismatch


def test_clamp_flip_at_a_last_bit_threshold_is_explained(ora):
    ens, _ = gen.workload("lifetimes_65536x4-8", n_sys=4)
    m, x, v = ens.system(1)
    o50 = ora.integrate_adaptive(m, x, v, t_end=1e9, eta=0.01, stop_rules=0, max_steps=50)
    t_end = o50["t"] + o50["dt_next"]        # the 51st step lands exactly on t_end
    ref = ora.integrate_adaptive(m, x, v, t_end=t_end, eta=0.01, stop_rules=0)
    assert ref["status"] == ora.DONE and ref["steps"] == 51
    t_alt = t_end * (1 + 2e-15)              # the candidate's sum falls just short
    got = ora.integrate_adaptive(m, x, v, t_end=t_alt, eta=0.01, stop_rules=0)
    assert got["steps"] == 52

    def rerun(k):
        return ora.integrate_adaptive(m, x, v, t_end=t_alt, eta=0.01, stop_rules=0, max_steps=k)
    k1, crit, margin = explain_adaptive_mismatch(ora, (m, x, v), t_end, 0.01, 0, 100.0, False, rerun,
                                                 got["status"], got["steps"], ref)
    assert (k1, crit) == (51, "clamp") and margin <= 1e-15


def test_flip_far_from_its_threshold_is_rejected(ora):
    m = np.array([1.0, 1e-5, 1e-5])
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 3.0, 0]])
    v = np.array([[0.0, 0, 0], [0, 1.0, 0], [2.0, 0.0, 0]])    # planet 2 escapes
    ref = ora.integrate_adaptive(m, x, v, t_end=1e4, eta=0.01, r_eject=100.0)
    assert ref["status"] == ora.EJECTED
    got = ora.integrate_adaptive(m, x, v, t_end=1e4, eta=0.01, r_eject=50.0)   # a wrong radius
    assert got["status"] == ora.EJECTED and got["steps"] < ref["steps"]

    def rerun(k):
        return ora.integrate_adaptive(m, x, v, t_end=1e4, eta=0.01, r_eject=50.0, max_steps=k)
    with pytest.raises(AssertionError, match="eject"):
        explain_adaptive_mismatch(ora, (m, x, v), 1e4, 0.01, 3, 100.0, False, rerun,
                                  got["status"], got["steps"], ref)


def test_divergence_before_the_decision_is_rejected(ora):
    """A candidate whose trajectory differs beyond 1e-10 before its first
    differing decision fails the parity check, whatever the margins."""
    ens, _ = gen.workload("lifetimes_65536x4-8", n_sys=4)
    m, x, v = ens.system(2)
    ref = ora.integrate_adaptive(m, x, v, t_end=20.0, eta=0.01, stop_rules=0)
    got = ora.integrate_adaptive(m, x, v, t_end=20.0, eta=0.0101, stop_rules=0)   # a wrong eta
    assert got["steps"] != ref["steps"]

    def rerun(k):
        return ora.integrate_adaptive(m, x, v, t_end=20.0, eta=0.0101, stop_rules=0, max_steps=k)
    with pytest.raises(AssertionError, match="before the first differing decision"):
        explain_adaptive_mismatch(ora, (m, x, v), 20.0, 0.01, 0, 100.0, False, rerun,
                                  got["status"], got["steps"], ref)
