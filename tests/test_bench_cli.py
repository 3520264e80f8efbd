"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a device, and the sections can be listed."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    line = r.stdout.strip().splitlines()[-1]
    assert "one GPU" in json.loads(line)["error"]


def test_help_lists_the_section_switches():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0
    for flag in ("--no-c2", "--no-timed", "--no-c3", "--no-serve", "--no-rt", "--no-bfs",
                 "--no-multi", "--no-cpu"):
        assert flag in r.stdout


def test_step_plan_does_not_grow_with_steps():
    """The driver's --steps 20 --warmup 5 (and any longer run) fits: every step
    starts from a reset queue, so G-WFQ-YMC's pool holds one step's cells."""
    sys.path.insert(0, ROOT)
    import bench
    for steps, warmup in ((20, 5), (5, 2), (1000, 100)):
        p = bench.step_plan(steps, warmup)
        assert p["reset_each_step"] and p["fits"]
        assert p["launches"] == steps + warmup
        assert p["ymc_cells_needed_per_step"] == bench.LANES * bench.OPS_PER_LANE + bench.CAP // 2
        assert p["ymc_cells_needed_per_step"] <= p["ymc_pool_cells"]


def test_checksums_of_a_split_multiset_add_up():
    """The bench's per-step conservation check: checksums of a union are the
    wrapping sums of the parts' checksums."""
    sys.path.insert(0, ROOT)
    import numpy as np

    import bench
    rng = np.random.default_rng(3)
    v = rng.integers(0, 2**64, size=1000, dtype=np.uint64)
    a, b = v[:377], v[377:]
    assert bench.csum_add(bench.checksums(a), bench.checksums(b)) == bench.checksums(v)
    # a lost item and a duplicated one change the sums
    w = v.copy()
    w[5] = w[6]
    assert bench.checksums(w) != bench.checksums(v)


def test_step_shape_follows_residency():
    """A variant's step uses the most lanes, up to 2^19 and a power of two,
    that the device holds at once in 1024-lane workgroups; the work per step
    stays 2^26 attempts.  The per-wavefront form keeps 2^19 lanes."""
    sys.path.insert(0, ROOT)
    import bench

    class FakeGq:
        def __init__(self, blocks):
            self.blocks = blocks

        def resident_blocks(self, kernel, kind, block):
            assert kernel == "mix_group" and block == 1024
            return self.blocks[kind]

    g = FakeGq({"lfq": 512, "wfq": 256, "ymc": 300})
    assert bench.step_shape(g, "lfq", 0) == (1 << 19, 128)
    assert bench.step_shape(g, "wfq", 1024) == (1 << 18, 256)
    assert bench.step_shape(g, "ymc", 0) == (1 << 18, 256)  # 300 blocks: 2^18 is the largest power
    assert bench.step_shape(FakeGq({"lfq": 4096}), "lfq", 0) == (1 << 19, 128)
    assert bench.step_shape(g, "wfq", 64) == (1 << 19, 128)
    for kind in ("lfq", "wfq", "ymc"):
        lanes, ops = bench.step_shape(g, kind, 0)
        assert lanes * ops == 1 << 26
