"""The autotuner's choice and cache, with a stand-in trial function."""
import json

from paper_2203_14362_amd.autotune import Autotuner, signature


def test_picks_fastest_and_caches(tmp_path):
    calls = []

    def trial(ppv):
        calls.append(ppv)
        return (ppv - 100.0) ** 2 / 100.0 + 1.0      # fastest near 100

    path = str(tmp_path / "tune.json")
    t = Autotuner(path, candidates=(25, 50, 100, 200, 400), repeats=2, preset=None)
    key = signature("count", 260, 80436, 100_000_000)
    ppv, times = t.tune(key, trial)
    assert ppv == 100.0 and set(times) == {25.0, 50.0, 100.0, 200.0, 400.0}
    assert len(calls) == 5 * 3                      # warm + 2 repeats per candidate
    # cached: no further trials, also from a fresh tuner reading the file
    ppv2, times2 = t.tune(key, trial)
    assert ppv2 == 100.0 and times2 == {} and len(calls) == 15
    t2 = Autotuner(path, preset=None)
    assert t2.lookup(key) == 100.0
    assert json.load(open(path))[key]["ppv"] == 100.0
    # forced re-tune measures again
    t2.candidates = (50.0, 200.0)
    ppv3, _ = t2.tune(key, trial, force=True)
    assert ppv3 in (50.0, 200.0) and len(calls) == 15 + 2 * 4


def test_signature_buckets():
    assert signature("count", 260, 80000, 100_000_000) == signature("count", 250, 90000, 120_000_000)
    assert signature("count", 260, 80000, 100_000_000) != signature("select", 260, 80000, 100_000_000)


def test_preset_is_read_only_and_overridden(tmp_path):
    key = signature("count", 260, 80436, 100_000_000)
    preset = tmp_path / "preset.json"
    preset.write_text(json.dumps({key: {"ppv": 40.0}}))
    cache = str(tmp_path / "cache.json")
    calls = []

    def trial(ppv):
        calls.append(ppv)
        return abs(ppv - 64.0) + 1.0

    t = Autotuner(cache, candidates=(32, 64), repeats=1, preset=str(preset))
    assert t.tune(key, trial) == (40.0, {}) and calls == [] and t.last_source == "preset"
    ppv, times = t.tune(key, trial, force=True)          # measured, written to the cache only
    assert ppv == 64.0 and t.last_source == "measured"
    assert json.loads(preset.read_text())[key]["ppv"] == 40.0
    t2 = Autotuner(cache, preset=str(preset))
    assert t2.tune(key, trial) == (64.0, {}) and t2.last_source == "cache"


def test_shipped_preset_loads():
    from paper_2203_14362_amd.autotune import PRESET_PATH
    t = Autotuner(None)
    for k, e in json.load(open(PRESET_PATH)).items():
        assert t.lookup(k) == float(e["ppv"]) and float(e["ppv"]) > 0
