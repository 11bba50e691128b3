"""The benchmark's one JSON line, from a short run on the GPU: the fields its readers rely on, the
roofline and CPU-baseline objects, and a value consistent with the step time."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.gpu


def test_bench_line_fields(tmp_path):
    env = dict(os.environ, UTC_AUTOTUNE_CACHE=str(tmp_path / "tune.json"))
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "12", "--warmup", "2",
           "--workload", "realistic", "--also", "tiny", "--cpu-seconds", "1", "--cpu-events", "50",
           "--no-per-event", "--no-fitgrad", "--no-copy-bandwidth", "--no-compact"]
    print("[bench line]", " ".join(cmd[1:]), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=300, env=env, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 12 and d["warmup"] == 2
    assert d["unit"] == "events/s" and d["higher_is_better"] is True and d["dtype"] == "f32"
    assert d["config"]["workload"].startswith("realistic: 1000 events")
    assert d["config"]["streams"] in (1, 2, 3)
    assert d["value"] == pytest.approx(1000 / (d["ms_per_step"] * 1e-3), rel=1e-3)
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    assert r["traffic"] is None or r["traffic"] > 0
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["unit"] == "events/s" and 1 <= c["cores"] <= 16 and c["value"] > 0
    assert c["sample"].startswith("the first 50 of the 1000 events")
    assert c["single_thread"]["cores"] == 1 and c["single_thread"]["value"] > 0
    assert c["host"]["nproc"] >= 1 and c["host"]["model"]
    assert d["found_fraction"] > 0.99
    o = d["other_workloads"]["tiny"]
    assert o["workload"].startswith("tiny: 100 events")
    assert o["events_per_s"] == pytest.approx(100 / (o["ms_per_step"] * 1e-3), rel=1e-3)
    assert set(o["calls_ms"]) == {"ut_decode", "compass_find", "compass_fit_grad"}
