"""Host-side parts of the benchmark contract (no GPU): the one-GPU guard, the
algorithmic bytes of a launch, and the rule that HBM traffic is reported from
the committed counter summary only while the compiled kernels match it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_algorithmic_bytes_of_the_headline_workload():
    # 4096^2 RGB, DC + 5 AC private: every sample once, 58 FP32 public and 6
    # int16 private values per 8x8 block
    n = 4096 * 4096 * 3
    nb = n // 64
    assert bench.algorithmic_bytes(4096, 4096, 3, 6) == n + nb * 58 * 4 + nb * 6 * 2 == 242221056
    # the precision form stores 16-bit public values
    assert bench.algorithmic_bytes(8192, 8192, 1, 10, pub_elt=2) == 8192 * 8192 * (1 + 54 * 2 / 64 + 10 * 2 / 64)


def _profile_fields():
    with open(bench.PROFILE) as f:
        line = [l for l in f if l.startswith("traffic_bytes_per_launch")][-1]
    return dict(kv.split("=") for kv in line.split()[1:])


def test_traffic_follows_the_kernel_fingerprint(monkeypatch):
    fields = _profile_fields()
    assert set(fields) >= {"frag", "defrag", "code_sha1"}
    monkeypatch.setattr(bench, "code_sha1", lambda: fields["code_sha1"])
    assert bench.measured_traffic("frag") == int(fields["frag"])
    assert bench.measured_traffic("defrag") == int(fields["defrag"])
    # counters taken on other machine code say nothing about this build
    monkeypatch.setattr(bench, "code_sha1", lambda: "0" * 40)
    assert bench.measured_traffic("frag") is None
    monkeypatch.setattr(bench, "code_sha1", lambda: None)
    assert bench.measured_traffic("frag") is None


def test_committed_counters_match_the_built_kernels():
    """The built headline kernels are the ones the committed counters were
    taken on (skipped when the library has not been built here)."""
    code = bench.code_sha1()
    if code is None:
        pytest.skip("library not built")
    assert code == _profile_fields()["code_sha1"]
