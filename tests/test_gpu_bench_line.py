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
           "--cpu-seconds", "1", "--no-per-event", "--no-fitgrad", "--no-copy-bandwidth", "--no-compact"]
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
    assert c["kind"] == "oracle" and c["unit"] == "events/s" and c["cores"] == 1 and c["value"] > 0
    assert c["sample"]
    assert d["found_fraction"] > 0.99
