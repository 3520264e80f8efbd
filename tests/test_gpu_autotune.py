"""Autotuner on the device: the chosen configuration is the fastest one it
measured, and the cache returns it without measuring again."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
def test_tune_mix_conserves(kind):
    """The conservation check passes for every queue kind on a real run."""
    from paper_2606_01693_amd import autotune as at
    r = at.tune_mix(kind, 1 << 12, total_ops=1 << 18, ticket_groups=(256,),
                    lanes_options=(1 << 12,), slot_modes=("linear",), capacity_factors=(2,),
                    reps=2)
    assert all("mops" in t for t in r.table), r.table


def test_tune_mix_small(tmp_path):
    from paper_2606_01693_amd import autotune as at
    path = str(tmp_path / "tune.json")
    r = at.tune_mix("lfq", 1 << 12, total_ops=1 << 18, ticket_groups=(64, 1024),
                    lanes_options=(1 << 12, 1 << 13), slot_modes=("linear",),
                    capacity_factors=(1, 4), reps=2, cache_path=path)
    good = [t for t in r.table if "mops" in t]
    # every configuration ran and conserved its items (a failed check is an "error" row)
    assert len(good) == 8, [t for t in r.table if "error" in t]
    assert r.best_mops == max(t["mops"] for t in good)
    assert at.cached(path, r.key).best == r.best


def test_tune_multi_small():
    from paper_2606_01693_amd import autotune as at
    caps = [1 << e for e in (8, 9, 10, 11, 12, 13, 14, 15)] * 2
    r = at.tune_multi("lfq", caps, waves_per_256_slots=(0.5, 1, 2), reps=2)
    assert r.best["waves_per_256_slots"] in (0.5, 1, 2)
    assert all("mops" in t for t in r.table)


def test_tune_prodcons_small():
    """A 64-wavefront 8:56 polling run: every measured configuration either
    completes with conservation or is recorded as failed, and the best is a
    completed one."""
    from paper_2606_01693_amd import autotune as at
    r = at.tune_prodcons("wfq", capacity=1 << 10, waves=64, prod_waves=8, log2_inv_p=0,
                         items=1 << 16, patience_options=((16, 64), (64, 256)),
                         help_delays=(64,), time_limit_ms=10000)
    good = [t for t in r.table if "mops" in t]
    assert good and r.best_mops == max(t["mops"] for t in good)
