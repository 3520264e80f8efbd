"""Autotuner search and cache logic, with an injected measurement (no GPU)."""
import json

import pytest


def fake_mix(cand):
    # pretend larger ticket groups and more lanes are faster; remap slower;
    # one configuration fails like a refused create
    if cand["ticket_group"] == 512 and cand["lanes"] == 1 << 17:
        raise RuntimeError("refused")
    ms = 10.0 / cand["ticket_group"] * (1 << 19) / cand["lanes"]
    if cand["slot_mode"] == "remap":
        ms *= 1.5
    return ms, 1 << 24


def test_tune_mix_picks_fastest_and_records_failures(tmp_path):
    from paper_2606_01693_amd import autotune as at
    path = str(tmp_path / "cache.json")
    r = at.tune_mix("lfq", 1 << 20, cache_path=path, measure=fake_mix)
    assert r.best == {"ticket_group": 1024, "lanes": 1 << 19, "slot_mode": "linear",
                      "patience": None}
    assert r.best_ms == min(t["ms"] for t in r.table if "ms" in t)
    assert any("error" in t for t in r.table)
    assert len(r.table) == 4 * 3 * 2
    data = json.load(open(path))
    assert r.key in data and data[r.key]["best"] == r.best


def test_cache_hit_skips_measurement(tmp_path):
    from paper_2606_01693_amd import autotune as at
    path = str(tmp_path / "cache.json")
    first = at.tune_mix("wfq", 1 << 16, cache_path=path, measure=fake_mix)
    calls = []

    def never(c):
        calls.append(c)
        return 1.0, 1

    again = at.tune_mix("wfq", 1 << 16, cache_path=path, measure=never)
    assert calls == [] and again.best == first.best
    forced = at.tune_mix("wfq", 1 << 16, cache_path=path, measure=never, force=True)
    assert len(calls) == len(forced.table)
    # other keys in the file survive a store
    at.tune_mix("lfq", 1 << 12, cache_path=path, measure=fake_mix)
    data = json.load(open(path))
    assert len(data) == 2


def test_lane_options_must_divide_the_work():
    from paper_2606_01693_amd import autotune as at
    r = at.tune_mix("lfq", 1 << 10, total_ops=3 << 16, lanes_options=(1 << 17, 3 << 15),
                    ticket_groups=(64,), slot_modes=("linear",), measure=fake_mix)
    assert [t["lanes"] for t in r.table] == [3 << 15]


def test_all_failing_raises():
    from paper_2606_01693_amd import autotune as at

    def bad(c):
        raise RuntimeError("no")

    with pytest.raises(RuntimeError):
        at.tune_mix("lfq", 1 << 10, measure=bad)


def test_multi_lanes_arithmetic():
    from paper_2606_01693_amd.autotune import multi_lanes
    caps = [256, 1024, 65536]
    lanes, ops = multi_lanes(caps, 1, 4)
    assert lanes[0] == 64 and lanes[1] == 256
    assert sum(lanes) % 256 == 0
    assert ops == 4 * 65536 // lanes[2] or lanes[2] > 64 * 256  # padded queue gets the pad
    lanes_half, _ = multi_lanes(caps, 0.5, 4)
    assert lanes_half[0] == 64  # at least one wavefront per queue


def test_tune_multi_with_fake_measure(tmp_path):
    from paper_2606_01693_amd import autotune as at

    def meas(c):
        return 1.0 / c["waves_per_256_slots"] + c["waves_per_256_slots"], 1000

    r = at.tune_multi("lfq", [256, 512, 1024], cache_path=str(tmp_path / "c.json"), measure=meas)
    assert r.best == {"waves_per_256_slots": 1}


def test_tune_prodcons_keeps_only_completed_runs(tmp_path):
    """Runs that time out or break conservation raise inside the measure and
    are recorded as failed; the fastest completed one wins."""
    from paper_2606_01693_amd import autotune as at

    def fake(c):
        pe, pd = c["patience"]
        if pe == 16:
            raise RuntimeError("run did not complete")
        return 100.0 / pe + c["help_delay"] / 1000.0, 1 << 24

    path = str(tmp_path / "pc.json")
    r = at.tune_prodcons(cache_path=path, measure=fake)
    assert r.best == {"patience": [256, 1024], "help_delay": 16}
    assert sum("error" in t for t in r.table) == 3 and len(r.table) == 9
    assert at.cached(path, r.key).best == r.best
