"""Launch-plan autotuning with a JSON plan cache.

The search itself is native (fb_autotune): for every body count of a
calibration ensemble it times each lane mapping x waves-per-group of the
plain schedule, then the fused persistent launch's waves-per-group x
groups-per-CU, and installs the fastest.  This module chooses the
calibration length, stores the chosen plans keyed by (GPU architecture, body
count) and re-applies them without re-timing.
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fewbody", "plans.json")


def arch_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def load_cache(path=DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply_plans(fb, plans: dict) -> list:
    """Install cached plans {"<n>": {...}, "persistent": {...}}; returns the body counts set."""
    done = []
    for key, p in plans.items():
        if key == "persistent":
            fb.set_plan(0, p.get("mapping", fb.MAP_AUTO), p["waves_per_group"], p["groups_per_cu"])
        else:
            fb.set_plan(int(key), p["mapping"], p["waves_per_group"], 0)
            done.append(int(key))
    return done


def tune(fb, ens, dt, target_ms=20.0, cache_path=DEFAULT_CACHE, use_cache=True, log=None):
    """Choose plans for the body counts in `ens` (a gen.Ensemble).

    With use_cache and every body count (and the persistent shape) cached for
    this architecture, the cached plans are applied and nothing is timed.
    Otherwise a short trial sizes the calibration run to about target_ms per
    candidate, fb_autotune measures every candidate, and the winners are
    cached.  Returns {"plans": ..., "entries": [...], "seconds": ...}."""
    arch = arch_name()
    cache = load_cache(cache_path) if use_cache else {}
    want = sorted({int(n) for n in ens.n_body})
    have = cache.get(arch, {})
    if use_cache and "persistent" in have and all(str(n) in have for n in want):
        apply_plans(fb, {k: have[k] for k in [str(n) for n in want] + ["persistent"]})
        return {"plans": have, "entries": [], "seconds": 0.0, "cached": True}
    t0 = time.perf_counter()
    E = fb.from_gen(ens)
    try:
        # size the calibration: time a short plain run first
        probe = 8
        E.synchronize()
        t1 = time.perf_counter()
        E.integrate_steps(probe, dt)
        E.synchronize()
        per_step_ms = max((time.perf_counter() - t1) * 1e3 / probe, 1e-4)
        steps = int(min(max(target_ms / per_step_ms, 16), 20000))
        entries = E.autotune(steps, dt)
    finally:
        E.close()
    plans = dict(have)
    for e in entries:
        if not e["chosen"]:
            continue
        if e["n"] == 0:
            plans["persistent"] = {"mapping": e["mapping"], "waves_per_group": e["waves_per_group"],
                                   "groups_per_cu": e["groups_per_cu"]}
        else:
            plans[str(e["n"])] = {"mapping": e["mapping"], "waves_per_group": e["waves_per_group"]}
    cache[arch] = plans
    if use_cache:
        save_cache(cache, cache_path)
    if log:
        log(f"[autotune] {len(entries)} candidates in {time.perf_counter() - t0:.1f} s, {steps} steps each")
    return {"plans": plans, "entries": entries, "seconds": time.perf_counter() - t0, "cached": False,
            "calibration_steps": steps}


def sweep(fb, gen, n_lo=3, n_hi=16, per_n=8192, steps=None, seed=21, log=print):
    """Per-body-count throughput of every candidate plan (no cache): an
    ensemble with `per_n` systems of each body count n_lo..n_hi (the
    ragged_hill distribution), timed by fb_autotune.  Returns rows of
    (n, mapping, waves_per_group, groups_per_cu, ms, algorithmic TFLOP/s,
    system-steps/s, chosen)."""
    import numpy as np
    parts = [gen.ragged_hill(per_n, seed=seed + n, n_lo=n, n_hi=n) for n in range(n_lo, n_hi + 1)]
    nb = np.concatenate([p.n_body for p in parts])
    ens = gen.Ensemble(nb, np.concatenate([p.mass for p in parts]), np.concatenate([p.pos for p in parts]),
                       np.concatenate([p.vel for p in parts]))
    dt = 2 * np.pi / 2000
    E = fb.from_gen(ens)
    try:
        if steps is None:
            E.integrate_steps(8, dt)
            E.synchronize()
            t0 = time.perf_counter()
            E.integrate_steps(32, dt)
            E.synchronize()
            per_step = (time.perf_counter() - t0) / 32
            steps = int(min(max(0.3 / per_step, 64), 20000))
        entries = E.autotune(steps, dt)
    finally:
        E.close()
    rows = []
    total_flops = float(sum(116.0 * n * (n - 1) / 2 + 120.0 * n for n in nb)) * steps
    for e in entries:
        n = e["n"]
        if n > 0:
            flops = per_n * (116.0 * n * (n - 1) / 2 + 120.0 * n) * steps
            sys_steps = per_n * steps
        else:
            flops, sys_steps = total_flops, len(nb) * steps
        s = e["ms"] / 1e3
        rows.append((n, e["mapping"], e["waves_per_group"], e["groups_per_cu"], e["ms"],
                     flops / s / 1e12, sys_steps / s, e["chosen"]))
    return rows, steps


if __name__ == "__main__":
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_1208_1157_amd import fewbody as fb_mod
    from paper_1208_1157_amd import gen as gen_mod
    ap = argparse.ArgumentParser(description="per-body-count plan sweep (prints a markdown table)")
    ap.add_argument("--per-n", type=int, default=8192)
    ap.add_argument("--n-lo", type=int, default=3)
    ap.add_argument("--n-hi", type=int, default=16)
    ap.add_argument("--steps", type=int, default=None)
    a = ap.parse_args()
    rows, steps = sweep(fb_mod, gen_mod, a.n_lo, a.n_hi, a.per_n, a.steps)
    names = {0: "auto", 1: "system/lane", 2: "body/lane"}
    # for the persistent rows the mapping is the fused kernel's class
    print(f"plan sweep: {a.per_n} systems per body count, {steps} fixed steps of 2pi/2000 per candidate")
    print("| n | mapping | waves/group | groups/CU | ms | algorithmic TFLOP/s | system-steps/s | chosen |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        n = "all (persistent)" if r[0] == 0 else str(r[0])
        print(f"| {n} | {names.get(r[1], r[1])} | {r[2]} | {r[3]} | {r[4]:.2f} | {r[5]:.2f} | {r[6]:.3e} | {'*' if r[7] else ''} |")
