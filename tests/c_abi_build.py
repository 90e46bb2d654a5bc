"""Builds tests/c_abi_roundtrip.c against include/sefrag.h and the in-tree
library (gcc, HIP runtime); used by the C ABI tests."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1512_02951_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_c_program(out_dir: str) -> str:
    exe = os.path.join(out_dir, "c_abi_roundtrip")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_abi_roundtrip.c"), "-o", exe,
           "-L", PKG, "-lsefrag", "-Wl,-rpath," + PKG, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C consumer did not build:\n" + r.stdout + r.stderr)
    return exe
