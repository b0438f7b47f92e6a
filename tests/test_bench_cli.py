"""bench.py command-line contract checks that need no GPU."""
import json
import os
import subprocess
import sys

from tests.helpers import ROOT


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_stored_counters_are_used_only_for_the_current_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(path):
        data = json.load(open(path))
        for key, ent in data.items():
            if key.startswith("_"):  # description, not a kernel entry
                assert bench.measured_counters(key) is None
                continue
            got = bench.measured_counters(key)
            assert (got is not None) == (ent.get("source_hash") == h)


def test_cpu_baseline_helpers_time_the_oracle():
    sys.path.insert(0, ROOT)
    import bench
    rate, wall, used, done = bench._oracle_rate("brio_wu", 400, 5, 1)
    assert used == 1 and done == 5 and rate > 0 and wall > 0
    assert isinstance(bench.cpu_model(), (str, type(None)))
