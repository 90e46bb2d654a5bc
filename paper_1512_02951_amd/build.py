"""Build the HIP library in-tree: paper_1512_02951_amd/libsefrag.so (gfx950).

Run ``python -m paper_1512_02951_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsefrag.so")

HIPCC_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    # every FMA in the kernels is explicit; no implicit contraction
    "-ffp-contract=off",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    if verbose and proc.stderr:
        # hipcc's host pass warns about the GPU-only target feature; show the rest
        lines = [l for l in proc.stderr.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")


def build(verbose: bool = False, extra=(), out: str | None = None, jobs: int | None = None) -> str:
    """Compile every HIP source (in parallel) and link libsefrag.so; always
    recompiles.  ``extra`` adds compiler flags (e.g. -D tuning knobs); ``out``
    writes the library elsewhere."""
    lib = out or LIB
    tmp = lib + ".tmp%d" % os.getpid()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    jobs = jobs or min(8, len(sources()), os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="sefrag_build_") as objdir:
        objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in sources()]
        cmds = [[hipcc(), *HIPCC_FLAGS, *extra, *inc, "-c", "-o", o, src] for src, o in zip(sources(), objs)]
        with ThreadPoolExecutor(jobs) as pool:
            list(pool.map(lambda c: _run(c, verbose), cmds))
        _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
