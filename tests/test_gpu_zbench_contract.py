"""The benchmark's one JSON line on the GPU (a short run, no CPU baseline, no
companion figures): the keys and units it promises, the round-trip rate from
its own step time, and a roofline entry consistent with itself."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_contract_line():
    print("case: bench.py --steps 10 --warmup 2 --no-cpu-baseline --no-forms", flush=True)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "10", "--warmup", "2",
                        "--no-cpu-baseline", "--no-forms"], capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, p.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 10 and d["warmup"] == 2
    assert d["unit"] == "MP/s" and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert "workload" in d["config"]
    # one step is the round trip of one 4096 x 4096 image
    assert d["value"] == pytest.approx(4096 * 4096 / 1e6 / (d["ms_per_step"] * 1e-3), rel=1e-3)
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    assert 0.0 < r["frac"] < 1.0
    assert r["traffic"] is None or abs(r["traffic"] / r["bytes_per_launch"] - 1.0) < 0.05
    # the roofline rate is the dominant kernel's bytes over its time in the loop
    t = d[r["kernel"] + "_ms"]
    assert t == max(d["frag_ms"], d["defrag_ms"]) and t < d["ms_per_step"]
    assert r["achieved"] == pytest.approx(r["bytes_per_launch"] / (t * 1e-3) / 1e9, rel=1e-3)
    assert d["frag_burst_ms"] > 0 and d["defrag_burst_ms"] > 0
    assert d["warm_ms_per_step"] > 0 and d["graph_replay_ms_per_step"] > 0
    assert 0 < d["median_ms_per_step"] < 10 * d["ms_per_step"]
