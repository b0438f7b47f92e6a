"""The benchmark line's contract, run in-process on a small grid (128^3, 3
timed steps, the extra legs off): one JSON line with the fields the line
promises, and numbers that agree with each other (value from ms_per_step and
the grid; the roofline's achieved bandwidth from its algorithmic bytes and
event-timed launch duration; frac = achieved / peak)."""
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_contract(capsys, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    n, steps, warmup = 128, 3, 1
    monkeypatch.setattr(sys, "argv", ["bench.py", "--n", str(n), "--steps", str(steps), "--warmup",
                                      str(warmup), "--no-fp64", "--no-cpu-baseline", "--no-paper-scheme",
                                      "--no-ct", "--no-adjoint"])
    bench.main()
    d = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["metric"] == bench.METRIC and d["unit"] == "Mcell-updates/s"
    assert (d["n_gpus"], d["steps"], d["warmup"]) == (1, steps, warmup)
    assert d["higher_is_better"] is True and d["scaling"] == "weak" and d["vs_baseline"] is None
    assert d["dtype"] == "f32" and d["data"] == "synthetic"
    assert f"{n}^3" in d["config"]["workload"] and d["config"]["n"] == [n] * 3
    cells = n ** 3
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert abs(d["value"] / (cells / (d["ms_per_step"] * 1e-3) / 1e6) - 1) < 2e-3
    r = d["roofline"]
    assert (r["bound"], r["unit"], r["peak"]) == ("hbm", "GB/s", bench.HBM_PEAK_GBS)
    assert r["alg_bytes_per_launch"] == 27 * 4 * cells
    assert 0 < r["avg_launch_ms"] < d["ms_per_step"]
    assert abs(r["achieved"] / (r["alg_bytes_per_launch"] / (r["avg_launch_ms"] * 1e-3) / 1e9) - 1) < 2e-3
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-4
    assert r["traffic"] is None or r["traffic"] > 0
    assert r["meets_target"] == (r["frac"] >= 0.6)
