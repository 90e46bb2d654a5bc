"""Runs the plain C consumer of the C ABI (tests/c_abi_roundtrip.c) on the
GPU as a child process: plain form, fp16 precision form, pixel-domain strong
level and wavelet round trips through include/sefrag.h alone, every sample
compared, and the exact integer fields of the security statistics against
host sums."""
import subprocess

import pytest

from c_abi_build import build_c_program

pytestmark = pytest.mark.gpu


def test_c_program_round_trips(tmp_path):
    exe = build_c_program(str(tmp_path))
    print("case: C consumer", exe, flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c abi round trips ok" in r.stdout
    assert r.stdout.count(": 0 of") == 7
