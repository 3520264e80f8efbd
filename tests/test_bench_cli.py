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
