"""Plan-cache logic of the autotuner (no GPU: a recording stand-in for the
binding's set_plan)."""
import json

from paper_1208_1157_amd import autotune


class RecordingPlans:
    MAP_AUTO, MAP_SPL, MAP_BPL = 0, 1, 2

    def __init__(self):
        self.calls = []

    def set_plan(self, n, mapping, waves, groups=0):
        self.calls.append((n, mapping, waves, groups))


def test_apply_plans_installs_every_entry():
    fb = RecordingPlans()
    plans = {"3": {"mapping": 1, "waves_per_group": 2}, "9": {"mapping": 2, "waves_per_group": 4},
             "persistent": {"mapping": 1, "waves_per_group": 4, "groups_per_cu": 8}}
    done = autotune.apply_plans(fb, plans)
    assert sorted(done) == [3, 9]
    assert (3, 1, 2, 0) in fb.calls and (9, 2, 4, 0) in fb.calls
    assert (0, 1, 4, 8) in fb.calls


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "plans.json")
    assert autotune.load_cache(path) == {}
    cache = {"gfx950": {"3": {"mapping": 1, "waves_per_group": 2}}}
    autotune.save_cache(cache, path)
    assert autotune.load_cache(path) == cache
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune.load_cache(path) == {}
    json.dumps(cache)
