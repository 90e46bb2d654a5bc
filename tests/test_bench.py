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


def test_tile_index_matches_the_oracle_layout():
    import numpy as np

    import oracle
    for nb, P in ((64, 58), (150, 54), (7, 3)):
        b = np.arange(nb).repeat(P)
        j = np.tile(np.arange(P), nb)
        got = bench._tile_index(nb, P, b, j)
        assert np.array_equal(got, [oracle.tile_offset(nb, P, int(bb), int(jj)) for bb, jj in zip(b, j)])


def test_reduced_precision_index_hand_example_and_permutation():
    import numpy as np
    # 100 blocks, P = 2: tile 0 in halves of 32 and 32 blocks, tile 1 (36 blocks) in 32 and 4
    f = bench._lp_tile_index
    assert [int(f(100, 2, b, j)) for b, j in ((0, 0), (31, 1), (32, 0), (33, 1), (64, 1), (96, 0), (99, 1))] == \
        [0, 63, 64, 97, 160, 192, 199]
    for nb, P in ((64, 54), (150, 54), (7, 3), (33, 5)):
        idx = f(nb, P, np.arange(nb).repeat(P), np.tile(np.arange(P), nb))
        assert np.array_equal(np.sort(idx), np.arange(nb * P))


def test_accuracy_of_sampled_blocks_against_the_oracle(monkeypatch):
    """The cpu_baseline leg's comparison: exact public values give 0; moving
    one value of one block by d gives d / |block|_2 for that block."""
    import numpy as np

    import oracle
    import synth
    x = synth.image(8, 8 * 40, 1, 2, 3).numpy()
    mask = (1 << 6) - 1
    ref = oracle.frag(x, mask)
    xb = oracle.blocks_of(x)
    pub = oracle.tile_unpack(ref["public"], 40, 58)
    monkeypatch.setattr(bench, "ACCURACY_SAMPLES", {"a": (xb, pub.copy(), mask)})
    assert bench.oracle_accuracy()["a"]["max"] == 0.0
    pub[5, 7] += 0.25
    monkeypatch.setattr(bench, "ACCURACY_SAMPLES", {"a": (xb, pub, mask)})
    r = bench.oracle_accuracy()["a"]
    assert r["max"] == pytest.approx(0.25 / np.linalg.norm(xb[5].astype(float)), rel=1e-3)
    assert r["median"] == 0.0


def test_cpu_baseline_fields():
    r = bench.cpu_baseline(budget_s=0.5)
    assert r["kind"] == "oracle" and r["unit"] == "MP/s" and r["cores"] >= 1
    assert r["value"] > 0 and r["frag_MP/s"] > 0 and r["defrag_MP/s"] > 0
    assert r["single_thread"]["MP/s"] > 0 and r["cpu_model"]


def test_cpu_fast_context_fields():
    r = bench.cpu_fast_context()
    assert r["frag_MP/s"] > 0 and r["defrag_MP/s"] > 0 and r["threads"] >= 1
    assert "not exact" in r["kind"]
    # rounding the private coefficients moves a sample by at most 1
    assert r["samples_off_by_more_than_1"] == 0
