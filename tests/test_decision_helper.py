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


def test_clamp_flip_inside_a_continued_run_is_explained(ora):
    """The same planted clamp flip, in a run that continues from a carried
    state (the second leg of an integration to several times)."""
    ens, _ = gen.workload("lifetimes_65536x4-8", n_sys=4)
    m, x, v = ens.system(3)
    leg1 = ora.integrate_adaptive(m, x, v, t_end=2.0, eta=0.01, stop_rules=0)
    start = dict(t0=leg1["t"], acc=leg1["acc"], jerk=leg1["jerk"], dt_next=leg1["dt_next"],
                 steps=leg1["steps"])
    mid = ora.integrate_adaptive(m, leg1["pos"], leg1["vel"], t_end=1e9, eta=0.01, stop_rules=0,
                                 max_steps=leg1["steps"] + 30, **start)
    t_end = mid["t"] + mid["dt_next"]
    ref = ora.integrate_adaptive(m, leg1["pos"], leg1["vel"], t_end=t_end, eta=0.01, stop_rules=0, **start)
    assert ref["steps"] == leg1["steps"] + 31
    t_alt = t_end * (1 + 2e-15)
    got = ora.integrate_adaptive(m, leg1["pos"], leg1["vel"], t_end=t_alt, eta=0.01, stop_rules=0, **start)

    def rerun(k):
        return ora.integrate_adaptive(m, leg1["pos"], leg1["vel"], t_end=t_alt, eta=0.01, stop_rules=0,
                                      max_steps=k, **start)
    k1, crit, margin = explain_adaptive_mismatch(ora, (m, leg1["pos"], leg1["vel"]), t_end, 0.01, 0, 100.0,
                                                 False, rerun, got["status"], got["steps"], ref, start=start)
    assert (k1, crit) == (leg1["steps"] + 31, "clamp")


def test_rkck_clamp_flip_is_explained_and_a_wrong_tolerance_is_not(ora):
    from tests.helpers import explain_rkck_mismatch
    ens, _ = gen.workload("lifetimes_65536x4-8", n_sys=4)
    m, x, v = ens.system(0)
    eps, dt0 = 1e-10, 0.02
    k = ora.integrate_rkck_adaptive(m, x, v, 1e9, eps, dt0, max_steps=40)
    t_end = k["t"] + k["dt_next"]                  # step 41 lands exactly on t_end
    ref = ora.integrate_rkck_adaptive(m, x, v, t_end, eps, dt0)
    assert ref["steps"] == 41
    t_alt = t_end * (1 + 2e-15)
    got = ora.integrate_rkck_adaptive(m, x, v, t_alt, eps, dt0)
    assert got["steps"] == 42

    def rerun(kk):
        return ora.integrate_rkck_adaptive(m, x, v, t_alt, eps, dt0, max_steps=kk)
    kstar, crit, margin = explain_rkck_mismatch(ora, (m, x, v), t_end, eps, dt0, rerun, got["steps"], ref)
    assert (kstar, crit) == (41, "clamp") and margin <= 1e-15

    def rerun_loose(kk):                            # a tolerance 3x too loose
        return ora.integrate_rkck_adaptive(m, x, v, 20.0, 3 * eps, dt0, max_steps=kk)
    ref20 = ora.integrate_rkck_adaptive(m, x, v, 20.0, eps, dt0)
    loose = ora.integrate_rkck_adaptive(m, x, v, 20.0, 3 * eps, dt0)
    assert loose["steps"] != ref20["steps"]
    with pytest.raises(AssertionError):
        explain_rkck_mismatch(ora, (m, x, v), 20.0, eps, dt0, rerun_loose, loose["steps"], ref20)
