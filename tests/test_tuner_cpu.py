"""The option tuner picks the fastest candidate, skips candidates the
library rejects, times only after a warm-up call, and caches by class."""
import time

import pytest

from paper_2505_04431_amd import kc, tuner


def fake_run(delays, calls):
    def run(o):
        key = tuple(sorted(o.items()))
        calls.append(key)
        if o.get("bad"):
            raise kc.KcError(-1, "rejected")
        time.sleep(delays[key])
    return run


def test_tune_picks_fastest_and_skips_rejected(tmp_path, monkeypatch):
    monkeypatch.setenv("KC_TUNE_CACHE", str(tmp_path / "cache.json"))
    cands = [{}, {"leaf_target": 2560}, {"leaf_target": 3500}, {"bad": 1}]
    delays = {(): 0.02, (("leaf_target", 2560),): 0.005, (("leaf_target", 3500),): 0.03}
    calls = []
    out = tuner.tune("k1", fake_run(delays, calls), candidates=cands, reps=2)
    assert out["options"] == {"leaf_target": 2560}
    assert [t["options"] for t in out["timings"]][0] == {"leaf_target": 2560}
    assert len(out["timings"]) == 3
    # each accepted candidate: one warm-up call, then the timed repetitions
    assert calls.count(()) == 3 and calls.count((("leaf_target", 3500),)) == 3
    # cached: no further calls for the same class
    calls.clear()
    again = tuner.tune("k1", fake_run(delays, calls), candidates=cands, reps=2)
    assert again["options"] == {"leaf_target": 2560} and calls == []
    # a different class is timed afresh; use_cache=False never reads the cache
    tuner.tune("k2", fake_run(delays, calls), candidates=cands[:2], reps=1)
    assert calls
    calls.clear()
    tuner.tune("k1", fake_run(delays, calls), candidates=cands[:1], reps=1, use_cache=False)
    assert calls


def test_tune_raises_when_nothing_runs(tmp_path, monkeypatch):
    monkeypatch.setenv("KC_TUNE_CACHE", str(tmp_path / "c.json"))
    with pytest.raises(RuntimeError):
        tuner.tune("k3", fake_run({}, []), candidates=[{"bad": 1}], reps=1)
