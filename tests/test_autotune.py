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
    ms *= {1: 1.2, 2: 1.0, 4: 1.1}[cand.get("capacity_factor", 1)]
    return ms, 1 << 24


def test_tune_mix_picks_fastest_and_records_failures(tmp_path):
    from paper_2606_01693_amd import autotune as at
    path = str(tmp_path / "cache.json")
    r = at.tune_mix("lfq", 1 << 20, cache_path=path, measure=fake_mix)
    assert r.best == {"ticket_group": 1024, "lanes": 1 << 19, "slot_mode": "linear",
                      "capacity_factor": 2, "patience": None}
    assert r.best_ms == min(t["ms"] for t in r.table if "ms" in t)
    assert any("error" in t for t in r.table)
    assert len(r.table) == 4 * 3 * 2 * 3
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
                    ticket_groups=(64,), slot_modes=("linear",), capacity_factors=(1,),
                    measure=fake_mix)
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


def test_mix_conservation_checksums_match_oracle():
    """The tuner's conservation check uses the same (count, S1, S2) the oracle
    defines (sums of v and v * v modulo 2^64), and it tells apart a multiset
    that lost one item and gained another of the same sum."""
    import numpy as np

    import oracle
    from paper_2606_01693_amd import autotune as at
    rng = np.random.default_rng(5)
    v = rng.integers(0, 1 << 63, 1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    assert at.checksums(v) == oracle.multiset_checksums(v)
    w = v.copy()
    w[0] += np.uint64(3)
    w[1] -= np.uint64(3)  # same count, same S1
    assert at.checksums(w)[:2] == at.checksums(v)[:2] and at.checksums(w) != at.checksums(v)
    a, b = at.checksums(v[:400]), at.checksums(v[400:])
    assert at._csum_add(a, b) == at.checksums(v)
