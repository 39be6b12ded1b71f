"""Continuous-batching server on the GPU: results alone vs in the mix,
admission by memory budget, cancellation, and a short Poisson trace."""
import math
import sys

import numpy as np
import pytest

from paper_1208_1157_amd import gen, serve
from tests.helpers import assert_parity, threads

pytestmark = pytest.mark.gpu
H = 2 * math.pi / 1000


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def small_requests(n_req, seed, max_sys=48, orbits=(0.3, 2.5)):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_req):
        ens = gen.ragged_hill(int(rng.integers(1, max_sys + 1)), seed=int(rng.integers(1 << 30)),
                              n_lo=3, n_hi=10)
        out.append((ens, 2 * math.pi * rng.uniform(*orbits)))
    return out


@pytest.mark.parametrize("cls,policy", [("bpl", 0), ("spl", 0), ("bpl", 1)])
def test_results_identical_alone_and_in_the_mix(plans, ora, cls, policy):
    """Systems of all requests share pool chunks and tiles; each request's
    results are bit-identical alone, in the mix and through an ensemble, in
    either fused-kernel class and under either scheduling policy."""
    fb = plans
    fb.set_plan(0, fb.MAP_SPL if cls == "spl" else fb.MAP_BPL, 2, 8)
    reqs = small_requests(16, seed=1)
    say("mix of", len(reqs), "requests", cls, "policy", policy)
    kw = dict(steps_per_quantum=300, policy=policy, chunk_slots=64,
              quantum_tiles=8 if policy == fb.POLICY_SRPT else 0)
    with fb.Server(**kw) as srv:
        ids = [srv.submit_gen(e, t, H) for e, t in reqs]
        mixed = []
        for rid in ids:
            assert srv.wait(rid, 120.0) == fb.REQ_DONE
            mixed.append(srv.result(rid))
        # continuous batching: later requests were admitted before earlier ones finished
        assert any(mixed[j]["t_admit"] < mixed[i]["t_done"] for i in range(len(mixed))
                   for j in range(i + 1, len(mixed)))
    for k, (ens, t_end) in enumerate(reqs):
        with fb.Server(**kw) as solo:
            rid = solo.submit_gen(ens, t_end, H)
            solo.wait(rid, 60.0)
            alone = solo.result(rid)
        assert np.array_equal(alone["pos"], mixed[k]["pos"]), k
        assert np.array_equal(alone["vel"], mixed[k]["vel"]), k
        assert np.all(mixed[k]["t"] == t_end) and np.all(mixed[k]["status"] == fb.DONE)
        assert np.all(mixed[k]["steps"] == serve.request_steps(t_end, H))
        # the same integration through an ensemble
        E = fb.from_gen(ens)
        E.integrate(t_end, H, fb.Opts(schedule=fb.SCHED_PERSISTENT, steps_per_quantum=300))
        st = E.state()
        E.close()
        assert np.array_equal(st["pos"], mixed[k]["pos"]), k
    # and against the oracle: whole steps then the shortened step
    for k, (ens, t_end) in enumerate(reqs[:4]):
        nfull = int(math.floor(t_end / H))
        X, V, A, J = ora.ensemble_fixed(ens.n_body, ens.mass, ens.pos, ens.vel, H, nfull, nthreads=threads())
        off = ens.offsets
        for s in range(ens.n_sys):
            sl = slice(off[s], off[s + 1])
            X[sl], V[sl], _, _ = ora.integrate_fixed(ens.mass[sl], X[sl], V[sl], t_end - nfull * H, 1,
                                                     acc=A[sl], jerk=J[sl])
        assert_parity(ens.n_body, mixed[k]["pos"], mixed[k]["vel"], X, V, label="serving vs oracle")


def test_idle_spread_is_bitwise_neutral(plans):
    """System-per-lane class: on a lightly loaded server the slowest
    system-per-lane tiles run body-per-lane (idle_spread); every request's
    results are bitwise those of a server that never spreads."""
    fb = plans
    fb.set_plan(0, fb.MAP_SPL, 2, 8)
    reqs = small_requests(6, seed=7, max_sys=200, orbits=(0.5, 1.5))
    # and systems the class always runs body-per-lane (11..16 bodies)
    reqs.append((gen.ragged_hill(90, seed=8, n_lo=11, n_hi=16), 2 * math.pi * 0.7))
    res = {}
    for spread in (-1, 1):
        say("idle spread", spread)
        with fb.Server(steps_per_quantum=250, chunk_slots=64, idle_spread=spread) as srv:
            ids = [srv.submit_gen(e, t, H) for e, t in reqs]
            out = []
            for rid in ids:
                assert srv.wait(rid, 120.0) == fb.REQ_DONE
                out.append(srv.result(rid))
            res[spread] = (out, srv.stats()["spread_quanta"])
    assert res[-1][1] == 0 and res[1][1] > 0
    for k, (off, on) in enumerate(zip(res[-1][0], res[1][0])):
        for key in ("pos", "vel", "t", "steps", "status"):
            assert np.array_equal(off[key], on[key]), (k, key)


def test_idle_spread_shortens_a_lone_request(plans):
    """A lone request of 10-body systems on an idle server: with idle spread
    its quanta run body-per-lane tiles, several times shorter per step (the
    single-tile step times are 9.3 us and 2.4 us), so it finishes well
    before the same request without it."""
    fb = plans
    fb.set_plan(0, fb.MAP_SPL, 2, 8)
    ens = gen.ragged_hill(256, seed=23, n_lo=10, n_hi=10)
    lat = {}
    for spread in (-1, 1):
        say("lone request, idle spread", spread)
        with fb.Server(steps_per_quantum=2000, idle_spread=spread) as srv:
            warm = srv.submit_gen(ens, 2 * math.pi * 2, H)    # first-launch costs
            assert srv.wait(warm, 120.0) == fb.REQ_DONE
            srv.result(warm)
            rid = srv.submit_gen(ens, 2 * math.pi * 30, H)    # 30000 steps, 15 quanta
            assert srv.wait(rid, 120.0) == fb.REQ_DONE
            r = srv.result(rid)
            lat[spread] = r["t_done"] - r["t_submit"]
    say("latency without / with idle spread", lat[-1], lat[1])
    assert lat[1] < 0.7 * lat[-1], lat


def test_admission_by_memory_budget(fb):
    """Requests that each fill a pool chunk cannot share one: with room for a
    single request, each waits until the one before it finishes."""
    slots = 64
    reqs = []
    for k in range(4):
        ens = gen.ragged_hill(slots, seed=20 + k, n_lo=5, n_hi=5)
        reqs.append((ens, 2 * math.pi * (1.0 + 0.1 * k)))
    need = fb.server_request_bytes(reqs[0][0].n_body, chunk_slots=slots)
    assert need > 0
    assert fb.server_request_bytes(reqs[0][0].n_body[:1], chunk_slots=slots) < need
    assert fb.server_request_bytes([1], chunk_slots=slots) == 0
    budget = int(1.5 * need)
    say("budget", budget)
    with fb.Server(budget_bytes=budget, steps_per_quantum=200, chunk_slots=slots) as srv:
        ids = [srv.submit_gen(e, t, H) for e, t in reqs]
        res = []
        for rid in ids:
            assert srv.wait(rid, 120.0) == fb.REQ_DONE
            res.append(srv.result(rid))
        st = srv.stats()
        assert st["peak_bytes"] <= budget
        assert st["completed"] == len(reqs)
    for i in range(1, len(res)):
        assert res[i]["t_admit"] >= res[i - 1]["t_done"], i
    # the same numbers as an unconstrained server
    with fb.Server(steps_per_quantum=200, chunk_slots=slots) as big:
        rid = big.submit_gen(*reqs[2], H)
        big.wait(rid, 60.0)
        assert np.array_equal(big.result(rid)["pos"], res[2]["pos"])
    with fb.Server(budget_bytes=max(4096, need - 256), chunk_slots=slots) as tiny:
        with pytest.raises(fb.FewbodyError) as ei:
            tiny.submit_gen(reqs[0][0], 1.0, H)
        assert ei.value.code == fb.E_BUDGET


def test_srpt_runs_least_remaining_work_first(fb):
    """One quantum holds one request (quantum_tiles = 1): the short requests
    submitted after a long one still finish before it."""
    long_ens = gen.ragged_hill(32, seed=30, n_lo=4, n_hi=6)
    short = [gen.ragged_hill(8, seed=31 + k, n_lo=3, n_hi=5) for k in range(4)]
    with fb.Server(steps_per_quantum=500, policy=fb.POLICY_SRPT, quantum_tiles=1) as srv:
        lid = srv.submit_gen(long_ens, 5000 * H, H)
        sids = [srv.submit_gen(e, 400 * H, H) for e in short]
        for rid in [lid] + sids:
            assert srv.wait(rid, 120.0) == fb.REQ_DONE
        lres = srv.result(lid)
        sres = [srv.result(r) for r in sids]
    assert max(r["t_done"] for r in sres) < lres["t_done"]
    assert np.all(lres["steps"] == serve.request_steps(5000 * H, H))


def test_cancel_and_errors(fb):
    ens = gen.ragged_hill(8, seed=3, n_lo=3, n_hi=6)
    with fb.Server(steps_per_quantum=100) as srv:
        rid = srv.submit_gen(ens, 2 * math.pi * 200, H)
        # not settled yet: it cannot be released
        with pytest.raises(fb.FewbodyError) as ei:
            srv.release(rid)
        assert ei.value.code == fb.E_STATE
        srv.cancel(rid)
        assert srv.wait(rid, 60.0) == fb.REQ_CANCELLED
        with pytest.raises(fb.FewbodyError) as ei:
            srv.result(rid)
        assert ei.value.code == fb.E_STATE
        # a settled request is forgotten on release
        srv.release(rid)
        for call in (srv.poll, srv.release):
            with pytest.raises(fb.FewbodyError) as ei:
                call(rid)
            assert ei.value.code == fb.E_NOTFOUND
        with pytest.raises(fb.FewbodyError) as ei:
            srv.poll(10 ** 9)
        assert ei.value.code == fb.E_NOTFOUND
        # a done request may be released instead of read
        rid = srv.submit_gen(ens, 2 * math.pi, H)
        assert srv.wait(rid, 60.0) == fb.REQ_DONE
        srv.release(rid)
        with pytest.raises(fb.FewbodyError) as ei:
            srv.result(rid)
        assert ei.value.code == fb.E_NOTFOUND


def test_short_poisson_trace(fb):
    trace = gen.serving_trace(60, rate=200.0, seed=5, max_sys=256)
    for r in trace:
        r.t_end = min(r.t_end, 2 * math.pi * 20)
    say("poisson trace", len(trace))
    rep = serve.run_trace(fb, trace, steps_per_quantum=1000)
    say({k: v for k, v in rep.items()})
    assert rep["requests"] == 60
    assert 0 < rep["p50_latency_s"] <= rep["p99_latency_s"] < 120
    assert rep["aggregate_system_steps_per_s"] > 0
