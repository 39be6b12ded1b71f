#!/usr/bin/env python3
"""Benchmark: FP64 Hermite P(EC)^2 system-steps/s on one MI355X.

One benchmark step is one pass of the whole hot path over the headline
ensemble (131072 independent star + two planet systems, seeded synthetic
inputs already resident in HBM): pack + set-up evaluation, 100000 fixed
Hermite steps of 2 pi/1000 in one launch, energy/angular-momentum
diagnostics, release.  value = system-steps per second of wall time over the
timed steps.

Printed as one JSON line, with
  roofline      achieved algorithmic FP64 FLOP/s of the integration kernel
                (HIP events on its launch stream) against the FP64 vector peak
                and against this device's measured FP64 FMA ceiling; the
                counter-derived FP64 FLOP/s and VALU occupancy where the
                kernel's hardware counters are on record; HBM traffic;
  p50/p99       solve latency of the serving trace (Poisson arrivals at
                200 req/s, 1..4096 systems of 3..10 bodies per request);
  load_store    HBM GB/s of the integration kernel's load and store phases:
                zero-step launches (state in, nothing integrated, state out);
  cpu_baseline  the CPU oracle timed on this host's cores on a bounded sample
                (all threads of the CPU share, and one thread);
  extras        the serving report (with the single-tile latency floor); the
                ragged 65536 x (3..15) batch with autotuned plans, plain
                per-bucket launches vs the fused persistent launch; uneven
                lifetimes 65536 x (4..8) with adaptive steps and stop rules on
                a bounded horizon, plain launches vs persistent quanta with
                compaction; with --extras also Section 5.1's initial
                conditions at Table 3's size, beside the paper's times; the
                MVS and Runge-Kutta Cash-Karp integrators on the headline
                ensemble, the ragged workload and the Section 5.1 systems.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 Hermite system-steps/s at 131072×3-body; p50/p99 solve latency"
KERNEL_SRC = os.path.join(ROOT, "paper_1208_1157_amd", "csrc", "fb_kernels.hip")
# HBM bytes per launch of the integration kernel on this workload, from the
# FETCH_SIZE / WRITE_SIZE counter passes (scaled by a 256 MiB copy kernel's
# reading) recorded in profiles/, keyed by the kernel source they measured.
MEASURED_TRAFFIC = {"f56593fdeadf867b": 92376093.0, "a3428dc18039eedc": 92445596.1,
                    "1c9dff3d544099cf": 92417308.4, "234f298587126ea3": 92405022.4,
                    "b0cf1370d8600140": 92417213.2, "d75718a170f1a208": 92400808.0,
                    "2e972ba6903455f7": 92417165.5, "b18c3be0358ab8a1": 92417237.0,
                    "1ed17940f99ee27b": 92404903.3, "0e3df7279f4c8f5d": 92412928.0,
                    "51a920369b9cae68": 92407561.1, "ad207609a06017a7": 92422664.6}
# Hardware counters of the same kernel on this workload from rocprofv3 runs
# (profiles/), keyed the same way: FP64 flop per system-step from
# SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes; the fraction of SIMD cycles issuing
# VALU (SQ_ACTIVE_INST_VALU x 4 over GRBM_GUI_ACTIVE per XCD x SIMDs); the
# shader clock those cycles implied on the profiled box.  They are records of
# those runs, reported as such, not measurements of this run.
PROFILED_COUNTERS = {
    "1c9dff3d544099cf": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9671,
                         "shader_clock_ghz": 2.018, "valu_insts_per_system_step": 388.01},
    "234f298587126ea3": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9753,
                         "shader_clock_ghz": 1.996, "valu_insts_per_system_step": 388.01},
    "b0cf1370d8600140": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9729,
                         "shader_clock_ghz": 1.977, "valu_insts_per_system_step": 388.01},
    "d75718a170f1a208": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9685,
                         "shader_clock_ghz": 1.999, "valu_insts_per_system_step": 388.01},
    "2e972ba6903455f7": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9725,
                         "shader_clock_ghz": 1.94, "valu_insts_per_system_step": 388.01},
    "b18c3be0358ab8a1": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9708,
                         "shader_clock_ghz": 2.025, "valu_insts_per_system_step": 388.01},
    "1ed17940f99ee27b": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9677,
                         "shader_clock_ghz": 1.939, "valu_insts_per_system_step": 388.01},
    "0e3df7279f4c8f5d": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9626,
                         "shader_clock_ghz": 2.114, "valu_insts_per_system_step": 388.0},
    "51a920369b9cae68": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9692,
                         "shader_clock_ghz": 2.066, "valu_insts_per_system_step": 388.0},
    "ad207609a06017a7": {"fp64_flops_per_system_step": 672.0, "valu_busy": 0.9556,
                         "shader_clock_ghz": 2.057, "valu_insts_per_system_step": 388.0},
}
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU
HBM_PEAK_GBPS = 8000.0           # MI355X HBM3E
PROFILE_SUMMARY = "profiles/k_plain_spl3_homog_131072x3.md"
# The oracle's threads: every CPU of the affinity set, up to the host share of
# one GPU on the GPU machines (16 threads).
HOST_THREAD_SHARE = 16
# Section 5.3, Table 3: seconds to integrate 131072 systems of the Section 5.1
# initial conditions for one time unit with the Hermite integrator, on the
# paper's four machines (context only: other hardware).
PAPER_TABLE3_SECONDS = {
    3: {"cluster1": 140.008, "cluster2": 35.951, "server1": 29.290, "workstation": 30.482},
    4: {"cluster1": 203.036, "cluster2": 65.284, "server1": 52.635, "workstation": 53.132},
    5: {"cluster1": 310.685, "cluster2": 100.800, "server1": 69.346, "workstation": 81.880},
    6: {"cluster1": 807.346, "cluster2": 121.908, "server1": 102.880, "workstation": 103.536},
    10: {"cluster1": 1874.480, "cluster2": 444.202, "server1": 577.674, "workstation": 362.020},
}


def kernel_source_hash() -> str:
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def flops_per_system_step(n: int) -> float:
    """Algorithmic FP64 work of one P(EC)^2 step of an n-body system:
    2 evaluations x 58 flop per pair + 120 flop per body for the predictor and
    two corrections (FMA = 2, add/mul/sqrt/div = 1)."""
    return 116.0 * n * (n - 1) / 2 + 120.0 * n


def affinity_cpus() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def host_threads() -> int:
    return max(1, min(HOST_THREAD_SHARE, affinity_cpus()))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(ens, h, target_s=15.0, single_s=5.0):
    """The oracle (plain FP64 C, one system per thread) on this host: all
    systems of the ensemble on every thread of the CPU share for a bounded
    number of steps, and a 2048-system subset on one thread."""
    import oracle
    nt = host_threads()

    def rate_of(e, threads, seconds):
        cal = e.subset(range(min(e.n_sys, 4096 * threads)))
        t0 = time.perf_counter()
        oracle.ensemble_fixed(cal.n_body, cal.mass, cal.pos, cal.vel, h, 20, nthreads=threads)
        r = cal.n_sys * 20 / (time.perf_counter() - t0)
        steps = max(10, int(r * seconds / e.n_sys))
        t0 = time.perf_counter()
        oracle.ensemble_fixed(e.n_body, e.mass, e.pos, e.vel, h, steps, nthreads=threads)
        dt = time.perf_counter() - t0
        return e.n_sys * steps / dt, steps, dt

    all_rate, all_steps, all_dt = rate_of(ens, nt, target_s)
    one = ens.subset(range(min(ens.n_sys, 2048)))
    one_rate, one_steps, one_dt = rate_of(one, 1, single_s)
    return {"value": all_rate, "unit": "system-steps/s", "cores": nt, "kind": "oracle",
            "sample": f"all {ens.n_sys} systems x {all_steps} steps (of the workload's 100000) on {nt} "
                      f"threads, {all_dt:.1f} s, pthreads with a static partition by system; single "
                      f"thread: {one.n_sys} systems x {one_steps} steps, {one_dt:.1f} s",
            "single_core_value": one_rate, "all_core_value": all_rate,
            "threads_used": nt, "os_cpu_count": os.cpu_count(), "affinity_cpus": affinity_cpus(),
            "thread_cap": HOST_THREAD_SHARE, "cpu_model": cpu_model()}


def load_store_probe(fb, ens, h, reps=10, scales=(1, 16)):
    """HBM rate of the integration kernel's load and store phases: launches
    of the headline kernel that load every system's state, take zero steps
    (the step cap is already reached) and store it back, timed by the
    library's kernel timer.  Algorithmic bytes per system: in 104 per body
    (m, x, v, a0, j0) + 68 of clock, out 96 per body + 36 of clock.  The
    headline ensemble, and the same systems tiled 16 times to amortise the
    launch latency."""
    import numpy as np
    out = {}
    for k in scales:
        nb = np.tile(ens.n_body, k)
        E = fb.Ensemble(nb, np.tile(ens.mass, k), np.tile(ens.pos, (k, 1)), np.tile(ens.vel, (k, 1)))
        E.integrate_steps(1, h)
        E.integrate_steps(1, h, fb.Opts(max_steps=1))     # warm: zero steps
        fb.profile_read()
        fb.profile_enable(True)
        for _ in range(reps):
            E.integrate_steps(1, h, fb.Opts(max_steps=1))
        E.synchronize()
        fb.profile_enable(False)
        ms, n = fb.profile_read()
        st = E.state()
        E.close()
        assert (st["steps"] == 1).all() and (st["status"] == fb.MAXSTEPS).all()
        n_sys, n_bodies = int(nb.shape[0]), int(nb.sum())
        nbytes = n_bodies * (104 + 96) + n_sys * (68 + 36)
        avg = ms / 1e3 / max(n, 1)
        out[f"{n_sys}x3"] = {"kernel": "k_plain_spl<3>, zero steps", "bytes_per_launch": nbytes,
                             "kernel_avg_ms": avg * 1e3, "launches": n, "achieved_gbps": nbytes / avg / 1e9,
                             "peak_gbps": HBM_PEAK_GBPS, "frac": nbytes / avg / 1e9 / HBM_PEAK_GBPS}
    return out


def timed(fb, torch, ens, fn):
    E = fb.from_gen(ens)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn(E)
    E.synchronize()
    dt = time.perf_counter() - t0
    st = E.state()
    E.close()
    return dt, st


def ragged_extras(fb, gen, torch, log):
    """Ragged 65536 x (3..15) batch: autotuned plans, then plain (one launch
    per body-count bucket, sequential) vs the fused persistent launch."""
    from paper_1208_1157_amd import autotune
    ens, p = gen.workload("ragged_65536x3-15")
    nsteps = p["steps"]
    tune = autotune.tune(fb, ens, p["dt"], use_cache=False, log=log)
    out = {"workload": f"ragged_65536x3-15: {ens.n_sys} systems, n uniform 3..15, "
                       f"{nsteps} fixed steps of 2pi/2000",
           "autotune_seconds": tune["seconds"], "plans": tune["plans"],
           "calibration_steps": tune.get("calibration_steps")}
    useful = ens.n_sys * nsteps
    flops = float(sum(flops_per_system_step(int(n)) for n in ens.n_body)) * nsteps
    for name, opts in [("plain", fb.Opts()),
                       ("persistent", fb.Opts(schedule=fb.SCHED_PERSISTENT))]:
        dt, st = timed(fb, torch, ens, lambda E: E.integrate_steps(nsteps, p["dt"], opts))
        assert (st["status"] == fb.DONE).all()
        out[name] = {"system_steps_per_s": useful / dt, "seconds": dt,
                     "fp64_tflops_algorithmic": flops / dt / 1e12}
        log(f"[bench] ragged {name}: {useful / dt:.3e} system-steps/s")
    out["persistent_over_plain"] = out["persistent"]["system_steps_per_s"] / out["plain"]["system_steps_per_s"]
    return out


def lifetimes_extras(fb, gen, torch, log, orbits=100.0, quantum=2000):
    """Uneven lifetimes 65536 x (4..8): adaptive steps (eta 0.01) with the
    close-encounter and ejection rules, on a horizon of `orbits` inner orbits
    (100 by default, a bounded sample of the workload's 1e4, which takes about
    23 s persistent and 83 s plain).  Plain: one launch per bucket, retired
    lanes idle until their wave's last system ends; persistent: quanta with
    in-kernel compaction of retired systems, the fused-kernel class chosen
    automatically (body-per-lane, then the tail mode once the survivors'
    waves no longer fill the device); and, for comparison, the body-per-lane
    class throughout."""
    import numpy as np
    ens, p = gen.workload("lifetimes_65536x4-8")
    t_end = 2 * math.pi * orbits
    base = dict(adaptive=True, eta=p["eta"], stop_rules=3, r_eject=p["r_eject"])
    out = {"workload": f"lifetimes_65536x4-8: {ens.n_sys} systems, n uniform 4..8, adaptive eta={p['eta']}, "
                       f"stop rules, bounded horizon t = 2pi*{orbits:g} (workload horizon 2pi*1e4)"}
    pers = fb.Opts(schedule=fb.SCHED_PERSISTENT, steps_per_quantum=quantum, compact=True, **base)
    saved = fb.get_plan(0)
    for name, opts, cls in [("plain", fb.Opts(**base), None),
                            ("persistent_compact", pers, None),
                            ("persistent_compact_body_per_lane_class", pers, fb.MAP_BPL)]:
        if cls is not None:
            fb.set_plan(0, cls, saved[1], saved[2])
        try:
            dt, st = timed(fb, torch, ens, lambda E: E.integrate(t_end, 0.0, opts))
        finally:
            fb.set_plan(0, *saved)
        useful = float(st["steps"].sum())
        flops = float(sum(flops_per_system_step(int(n)) * float(k) for n, k in zip(ens.n_body, st["steps"])))
        hist = {str(k): int(v) for k, v in zip(*np.unique(st["status"], return_counts=True))}
        out[name] = {"useful_system_steps_per_s": useful / dt, "seconds": dt, "system_steps": useful,
                     "fp64_tflops_algorithmic": flops / dt / 1e12, "status_histogram": hist}
        log(f"[bench] lifetimes {name}: {useful / dt:.3e} useful system-steps/s in {dt:.2f} s")
    out["compaction_over_plain"] = (out["persistent_compact"]["useful_system_steps_per_s"]
                                    / out["plain"]["useful_system_steps_per_s"])
    return out


def step_latency(fb, gen, n, mapping, h=2 * math.pi / 1000, steps=20000):
    """Seconds per step of a single tile (64 systems system-per-lane, or
    floor(64/n) body-per-lane) with the device otherwise idle: the floor of
    any request's latency per step."""
    k = 64 if mapping == fb.MAP_SPL else 64 // n
    ens = gen.ragged_hill(k, seed=9, n_lo=n, n_hi=n)
    saved = fb.get_plan(n)
    fb.set_plan(n, mapping, 1, 0)
    try:
        E = fb.from_gen(ens)
        E.integrate_steps(100, h)
        E.synchronize()
        t0 = time.perf_counter()
        E.integrate_steps(steps, h)
        E.synchronize()
        dt = time.perf_counter() - t0
        E.close()
    finally:
        fb.set_plan(n, *saved)
    return dt / steps


def paper_ic_extras(fb, gen, torch, log, n_sys=131072, h=1e-3, t_end=1.0):
    """Section 5.1's initial conditions at Table 3's size and length (one
    time unit at h = 1e-3), next to the paper's seconds on its machines."""
    rows = []
    steps = int(round(t_end / h))
    for n in sorted(PAPER_TABLE3_SECONDS):
        ens = gen.paper_ics(n_sys, n)
        dt, st = timed(fb, torch, ens, lambda E: E.integrate_steps(steps, h))
        assert (st["status"] == fb.DONE).all()
        rows.append({"n": n, "seconds": dt, "system_steps_per_s": n_sys * steps / dt,
                     "fp64_tflops_algorithmic": n_sys * steps * flops_per_system_step(n) / dt / 1e12,
                     "paper_table3_seconds": PAPER_TABLE3_SECONDS[n]})
        log(f"[bench] paper ICs n={n}: {dt:.4f} s")
    return {"workload": f"paper ICs (Section 5.1): {n_sys} systems, equal planet masses 1e-3, circular, "
                        f"coplanar, a_i = 1.4^(i-1); {steps} steps of h = {h:g} (one time unit); default plans",
            "rows": rows}


def mvs_extras(fb, gen, torch, log, dt=1e-2, steps=20000):
    """The mixed-variable symplectic integrator (Section 2.2.3) at the paper's
    step for it (Section 5.2.2: dt = 1e-2): the headline ensemble for `steps`
    steps, and Section 5.1's initial conditions at 131072 systems for one
    time unit.  Work unit: system-steps (each planet takes one Kepler drift,
    every planet pair one acceleration evaluation)."""
    out = {"dt": dt}
    ens, _ = gen.workload("homog_131072x3")
    t, st = timed(fb, torch, ens, lambda E: E.integrate_mvs(steps, dt))
    assert (st["status"] == fb.DONE).all()
    out["homog_131072x3"] = {"steps": steps, "seconds": t, "system_steps_per_s": ens.n_sys * steps / t}
    log(f"[bench] MVS homog_131072x3: {ens.n_sys * steps / t:.3e} system-steps/s")
    rows = []
    n_steps = int(round(1.0 / dt))
    for n in (3, 4, 5, 6, 8):
        e = gen.paper_ics(131072, n)
        t, st = timed(fb, torch, e, lambda E: E.integrate_mvs(n_steps, dt))
        assert (st["status"] == fb.DONE).all()
        rows.append({"n": n, "seconds": t, "system_steps_per_s": e.n_sys * n_steps / t})
    out["paper_ics_one_time_unit"] = rows
    # larger systems, one body per lane across a workgroup
    for name, nsteps in (("ragged_65536x3-15", 2000), ("disk_4096x64", 1000)):
        e, _ = gen.workload(name)
        t, st = timed(fb, torch, e, lambda E: E.integrate_mvs(nsteps, dt))
        done = float((st["status"] == fb.DONE).mean())
        out[name] = {"steps": nsteps, "seconds": t, "system_steps_per_s": e.n_sys * nsteps / t,
                     "fraction_done": done}
        log(f"[bench] MVS {name}: {e.n_sys * nsteps / t:.3e} system-steps/s ({100 * done:.1f}% done)")
    return out


def rkck_extras(fb, gen, torch, log, steps=2000):
    """The Runge-Kutta Cash-Karp integrator (Sections 2.2.2 and 4.3.2): fixed
    steps on the headline ensemble (dt 2pi/1000) and on the ragged workload
    (dt 2pi/2000), and adaptive steps (eps 1e-10, one inner orbit) on
    Section 5.1's three-body systems.  Work unit: system-steps (six
    acceleration evaluations each); adaptive counts accepted steps."""
    out = {}
    ens, _ = gen.workload("homog_131072x3")
    t, st = timed(fb, torch, ens, lambda E: E.integrate_rkck_steps(steps, 2 * math.pi / 1000))
    assert (st["status"] == fb.DONE).all()
    out["homog_131072x3_fixed"] = {"steps": steps, "seconds": t, "system_steps_per_s": ens.n_sys * steps / t}
    log(f"[bench] RKCK homog_131072x3: {ens.n_sys * steps / t:.3e} system-steps/s")
    rg, p = gen.workload("ragged_65536x3-15")
    t, st = timed(fb, torch, rg, lambda E: E.integrate_rkck_steps(steps, p["dt"]))
    assert (st["status"] == fb.DONE).all()
    out["ragged_65536x3-15_fixed"] = {"steps": steps, "seconds": t, "system_steps_per_s": rg.n_sys * steps / t}
    pi3 = gen.paper_ics(131072, 3)
    t, st = timed(fb, torch, pi3, lambda E: E.integrate_rkck(2 * math.pi, 0.01, 1e-10))
    assert (st["status"] == fb.DONE).all()
    acc = float(st["steps"].sum())
    out["paper_ics_n3_adaptive"] = {"eps": 1e-10, "t_end": 2 * math.pi, "seconds": t,
                                    "accepted_steps_per_system": acc / pi3.n_sys,
                                    "system_steps_per_s": acc / t}
    return out


def logging_extras(fb, gen, torch, log, steps=20000, every=200):
    """The monitor with on-device data reduction (Sections 4.3 and 4.4) on
    the headline ensemble: records every `every` steps of the star's
    line-of-sight velocity, or of energy and angular momentum, against the
    unlogged run.  The run leaves its records in a device buffer; their copy
    to pinned host memory is timed on its own."""
    ens, p = gen.workload("homog_131072x3")
    t0, _ = timed(fb, torch, ens, lambda E: E.integrate_steps(steps, p["dt"]))
    records = 1 + steps // every
    out = {"steps": steps, "every": every, "records_per_system": records, "unlogged_seconds": t0}
    full_state = 8 * (1 + 6 * 3)   # bytes of one full-state record of a 3-body system
    for name, kind in (("rv", fb.LOG_RV), ("energy", fb.LOG_ENERGY)):
        held = {}
        t, _ = timed(fb, torch, ens, lambda E: held.update(
            buf=E.integrate_steps_logged(steps, p["dt"], every, kind=kind, to_host=False)[0]))
        buf = held["buf"]
        host = torch.empty(buf.numel(), dtype=torch.uint8, pin_memory=True)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        host.copy_(buf)
        copy_s = time.perf_counter() - c0
        down = buf.numel()
        out[name] = {"seconds": t, "overhead": t / t0 - 1.0, "bytes_to_host": down,
                     "host_copy_seconds": copy_s, "host_copy_gb_per_s": down / copy_s / 1e9,
                     "bytes_as_full_states": ens.n_sys * records * full_state,
                     "records_per_s": ens.n_sys * records / t}
        log(f"[bench] logging {name}: {t:.4f} s vs {t0:.4f} s unlogged; {down / 1e6:.0f} MB of records "
            f"({ens.n_sys * records * full_state / down:.1f}x less than full states) copied in {copy_s:.4f} s")
        del buf, host, held
    return out


def table1_extras(fb, gen, torch, log, tau=1.7e-2, horizons=(0.45e6, 0.9e6, 1.3e6, 1.8e6)):
    """Table 1's adaptive Hermite energy test: Section 5.1's three-body
    systems (64 copies), Eq. 5 steps with step scale tau, |dE/E| at the
    table's times (Section 5.2.2).  Minutes of GPU time; not part of
    --extras."""
    import numpy as np
    ens = gen.paper_ics(64, 3)
    E = fb.from_gen(ens)
    e0, _ = E.diagnostics()
    rows = []
    t0 = time.perf_counter()
    for T in horizons:
        E.integrate(T, 0.0, fb.Opts(adaptive=2, eta=tau))
        e1, _ = E.diagnostics()
        st = E.state()
        err = float(np.max(np.abs(e1 / e0 - 1.0)))
        rows.append({"t": T, "steps": int(st["steps"][0]), "max_frac_energy_error": err,
                     "seconds": time.perf_counter() - t0})
        log(f"[bench] table1 tau={tau:g} t={T:.3g}: |dE/E| = {err:.3e}")
    E.close()
    return {"tau": tau, "rows": rows,
            "paper_table1_hermite_adaptive": [2.9e-11, 6.3e-11, 9.2e-11, 14.1e-11]}


def large_n_extras(fb, gen, torch, log):
    """The large-n gravitation (systems of 17..512 bodies, Section 4.2's
    second variant): fixed Hermite steps (dt 2pi/1000) on planetesimal disks.
    Algorithmic FP64 work counts each pair once per evaluation (the kernel
    evaluates every pair from both sides, twice that)."""
    out = {}
    for name, steps in (("disk_16384x17", 20000), ("disk_4096x64", 5000), ("disk_2048x128", 2000),
                        ("disk_512x512", 500)):
        ens, p = gen.workload(name)
        n = int(ens.n_body[0])
        timed(fb, torch, ens.subset(range(64)), lambda E: E.integrate_steps(2, p["dt"]))   # code load
        t, st = timed(fb, torch, ens, lambda E: E.integrate_steps(steps, p["dt"]))
        assert (st["status"] == fb.DONE).all()
        sps = ens.n_sys * steps / t
        alg = sps * flops_per_system_step(n) / 1e12
        out[name] = {"steps": steps, "seconds": t, "system_steps_per_s": sps,
                     "pair_interactions_per_s": sps * 2 * n * (n - 1) / 2,
                     "fp64_tflops_algorithmic": alg, "frac_fp64_peak": alg / FP64_VECTOR_PEAK_TFLOPS}
        log(f"[bench] large-n {name}: {sps:.3e} system-steps/s, {alg:.1f} TFLOP/s algorithmic")
    return out


def serving_report(fb, gen, log, n_req=2000, max_resident=4096, quantum=2000, policy="srpt",
                   cls="spl", quantum_tiles=0, long_steps=300000, idle_spread=0):
    from paper_1208_1157_amd import serve
    trace = gen.serving_trace(n_req, rate=200.0, seed=4)
    saved = fb.get_plan(0)
    fb.set_plan(0, fb.MAP_SPL if cls == "spl" else fb.MAP_BPL, saved[1], saved[2])
    try:
        rep = serve.run_trace(fb, trace, max_resident=max_resident, steps_per_quantum=quantum, log=log,
                              policy=fb.POLICY_SRPT if policy == "srpt" else fb.POLICY_FAIR,
                              quantum_tiles=quantum_tiles, long_steps=long_steps,
                              idle_spread=idle_spread)
    finally:
        fb.set_plan(0, *saved)
    rep["max_resident"] = max_resident
    rep["steps_per_quantum"] = quantum
    rep["policy"] = policy
    rep["fused_class"] = "system-per-lane" if cls == "spl" else "body-per-lane"
    rep["quantum_tiles"] = quantum_tiles
    rep["long_steps"] = long_steps
    rep["idle_spread"] = idle_spread >= 0
    rep["workload"] = (f"serving: {n_req} requests, Poisson 200 req/s, 1..4096 systems (log-uniform) of 3..10 "
                       f"bodies, t_end 2pi*10^U(1,3), dt 2pi/1000")
    lat = {"n3_system_per_lane": step_latency(fb, gen, 3, fb.MAP_SPL),
           "n10_system_per_lane": step_latency(fb, gen, 10, fb.MAP_SPL),
           "n10_body_per_lane": step_latency(fb, gen, 10, fb.MAP_BPL)}
    rep["single_tile_step_latency_s"] = lat
    rep["min_latency_1e6_steps_s"] = {k: v * 1e6 for k, v in lat.items()}
    return rep


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed benchmark steps")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--hermite-steps", type=int, default=100000,
                    help="Hermite steps per benchmark step (the workload's 100000)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--extras", action="store_true",
                    help="also run every other extra workload (paper ICs, MVS, Runge-Kutta, large n, logging)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the ragged (autotuned, plain vs persistent) and uneven-lifetimes "
                         "(plain vs compaction) comparisons that run by default")
    ap.add_argument("--extra", action="append", default=[],
                    choices=["ragged", "lifetimes", "paper_ics", "mvs", "rkck", "large_n", "logging",
                             "table1"],
                    help="run only this extra workload (repeatable; table1 only this way)")
    ap.add_argument("--table1-tau", type=float, default=1.7e-2,
                    help="Eq. 5 step scale of the table1 extra (the paper's 1.7e-2)")
    ap.add_argument("--lifetimes-orbits", type=float, default=100.0,
                    help="horizon of the uneven-lifetimes extra in inner orbits (the workload's is 1e4)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-max-resident", type=int, default=4096)
    ap.add_argument("--serve-quantum", type=int, default=2000)
    ap.add_argument("--serve-policy", choices=["fair", "srpt"], default="srpt",
                    help="server scheduling: every resident request per quantum, or least remaining work first")
    ap.add_argument("--serve-class", choices=["bpl", "spl"], default="spl",
                    help="fused-kernel class the server runs")
    ap.add_argument("--serve-quantum-tiles", type=int, default=0,
                    help="SRPT tiles per quantum (0: the server's default)")
    ap.add_argument("--serve-long-steps", type=int, default=300000,
                    help="SRPT: requests with at least this many steps left run every quantum")
    ap.add_argument("--serve-no-idle-spread", action="store_true",
                    help="keep every system-per-lane tile in its mapping, however light the load")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported (the path would "
              "shard by system across GPUs, which is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1208_1157_amd import fewbody as fb
    from paper_1208_1157_amd import gen

    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    ens, p = gen.workload("homog_131072x3")
    h = p["dt"]
    K = args.hermite_steps
    dev = torch.device("cuda", 0)
    m_d = torch.from_numpy(ens.mass).to(dev)
    x_d = torch.from_numpy(ens.pos).to(dev)
    v_d = torch.from_numpy(ens.vel).to(dev)
    torch.cuda.synchronize()

    default_plans = {n: fb.get_plan(n) for n in [0] + list(range(2, 17))}

    def restore_plans():
        for n, pl in default_plans.items():
            fb.set_plan(n, *pl)

    # the headline launch: system per lane, four waves per workgroup
    fb.set_plan(3, fb.MAP_SPL, 4, 0)

    def one_step():
        E = fb.Ensemble(ens.n_body, m_d, x_d, v_d)
        E.integrate_steps(K, h)
        energy, _ = E.diagnostics()
        E.close()
        return energy

    for w in range(args.warmup):
        one_step()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    fb.profile_read()
    fb.profile_enable(True)
    torch.cuda.synchronize()
    per_launch_ms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        energy = one_step()
        ms_k, n_k = fb.profile_read()   # this step's launch (the step has synchronised)
        per_launch_ms.append(ms_k / max(n_k, 1))
        print(f"[bench] step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fb.profile_enable(False)
    kernel_ms, launches = sum(per_launch_ms), len(per_launch_ms)
    assert np.all(np.isfinite(energy))

    sys_steps = ens.n_sys * K * args.steps
    value = sys_steps / elapsed
    kern_avg_s = kernel_ms / 1e3 / max(launches, 1)
    flops_per_launch = ens.n_sys * K * flops_per_system_step(3)
    achieved = flops_per_launch / kern_avg_s / 1e12
    m, w, _ = fb.get_plan(3)
    probe = fb.fp64_fma_ceiling()
    src_hash = kernel_source_hash()
    counters = PROFILED_COUNTERS.get(src_hash)
    profiled = None
    if counters:
        profiled = dict(counters, source=PROFILE_SUMMARY, kernel_source=src_hash,
                        note="hardware counters of a rocprofv3 run of this kernel source on another box "
                             "(records, not measured in this run)",
                        counter_tflops_at_this_runs_time=counters["fp64_flops_per_system_step"] * ens.n_sys * K
                        / kern_avg_s / 1e12)
    half = max(1, len(per_launch_ms) // 4)
    sustained = {"per_launch_ms": per_launch_ms,
                 "first_quarter_avg_ms": sum(per_launch_ms[:half]) / half,
                 "last_quarter_avg_ms": sum(per_launch_ms[-half:]) / half}
    sustained["last_over_first"] = sustained["last_quarter_avg_ms"] / sustained["first_quarter_avg_ms"]
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "system-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded star + 2 planet systems)",
        "config": {"workload": f"homog_131072x3: {ens.n_sys} systems x 3 bodies, {K} fixed Hermite "
                               f"P(EC)^2 steps of 2pi/1000 per benchmark step, one launch",
                   "n_sys": ens.n_sys, "n_body": 3, "hermite_steps": K, "dt": h,
                   "schedule": "plain", "mapping": "system-per-lane" if m == fb.MAP_SPL else "body-per-lane",
                   "waves_per_group": w},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": MEASURED_TRAFFIC.get(src_hash),
                     "kernel": "k_plain_spl<3>", "kernel_avg_ms": kern_avg_s * 1e3,
                     "kernel_launches": launches,
                     "flops_per_launch": flops_per_launch,
                     "fma_probe_tflops": probe, "frac_of_fma_probe": achieved / probe if probe else None,
                     "fma_probe_clock_ghz_lower_bound": probe / (256 * 128 * 1e-3) if probe else None,
                     "sustained": sustained, "profiled": profiled},
        "pair_interactions_per_s": value * 2 * 3,
    }
    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    extras = {}
    restore_plans()
    result["roofline"]["load_store"] = load_store_probe(fb, ens, h)
    restore_plans()
    if not args.no_serve:
        rep = serving_report(fb, gen, log, args.serve_requests, args.serve_max_resident, args.serve_quantum,
                             args.serve_policy, args.serve_class, args.serve_quantum_tiles,
                             args.serve_long_steps, -1 if args.serve_no_idle_spread else 0)
        result["p50_latency_s"] = rep["p50_latency_s"]
        result["p99_latency_s"] = rep["p99_latency_s"]
        extras["serving"] = rep
    runs = [
        ("ragged", lambda: ragged_extras(fb, gen, torch, log)),
        ("lifetimes", lambda: lifetimes_extras(fb, gen, torch, log, orbits=args.lifetimes_orbits)),
        ("paper_ics", lambda: paper_ic_extras(fb, gen, torch, log)),
        ("mvs", lambda: mvs_extras(fb, gen, torch, log)),
        ("rkck", lambda: rkck_extras(fb, gen, torch, log)),
        ("large_n", lambda: large_n_extras(fb, gen, torch, log)),
        ("logging", lambda: logging_extras(fb, gen, torch, log)),
    ]
    default_runs = () if args.no_compare else ("ragged", "lifetimes")
    for name, fn in runs:
        if args.extras or name in args.extra or name in default_runs:
            extras[name] = fn()
            restore_plans()
    if "ragged" in extras:
        result["ragged_persistent_over_plain"] = extras["ragged"]["persistent_over_plain"]
    if "lifetimes" in extras:
        result["lifetimes_compaction_over_plain"] = extras["lifetimes"]["compaction_over_plain"]
    if "table1" in args.extra:
        extras["table1"] = table1_extras(fb, gen, torch, log, tau=args.table1_tau)
    if extras:
        result["extras"] = extras
    if not args.no_cpu:
        ens_cpu = ens
        result["cpu_baseline"] = cpu_baseline(ens_cpu, h)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
