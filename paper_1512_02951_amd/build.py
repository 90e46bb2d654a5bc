"""Build the HIP library in-tree: paper_1512_02951_amd/libsefrag.so (gfx950).

Run ``python -m paper_1512_02951_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import glob
import json
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


CODE_HASH = os.path.join(PKG, "kernel_code_sha1.json")
# translation units whose machine code is fingerprinted at build time
HASHED_UNITS = ("plain.hip", "lp.hip")


def _llvm_tool(name):
    for d in ("/opt/rocm/llvm/bin", os.path.dirname(hipcc())):
        p = os.path.join(d, name)
        if os.path.exists(p):
            return p
    return shutil.which(name)


def code_sha1(obj: str) -> str | None:
    """SHA-1 of the .text and .rodata sections (instructions and kernel
    descriptors) of the gfx950 code object inside a compiled object file.
    Unlike a hash of the sources it changes only when the generated code does."""
    import hashlib
    tools = [_llvm_tool(n) for n in ("llvm-objcopy", "clang-offload-bundler")]
    if not all(tools):
        return None
    objcopy, bundler = tools
    with tempfile.TemporaryDirectory(prefix="sefrag_hash_") as d:
        fat, co = os.path.join(d, "fat.bin"), os.path.join(d, "code.o")
        steps = [[objcopy, "--dump-section=.hip_fatbin=" + fat, obj, os.path.join(d, "host.o")],
                 [bundler, "--unbundle", "--type=o", "--input=" + fat,
                  "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--output=" + co]]
        for sec in (".text", ".rodata"):
            steps.append([objcopy, "-O", "binary", "--only-section=" + sec, co, os.path.join(d, sec[1:])])
        for cmd in steps:
            if subprocess.run(cmd, capture_output=True).returncode != 0:
                return None
        h = hashlib.sha1()
        for sec in ("text", "rodata"):
            with open(os.path.join(d, sec), "rb") as f:
                h.update(f.read())
        return h.hexdigest()


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
        hashes = {os.path.basename(src): code_sha1(o) for src, o in zip(sources(), objs)
                  if os.path.basename(src) in HASHED_UNITS}
    os.replace(tmp, lib)
    if out is None:
        with open(CODE_HASH, "w") as f:
            json.dump(hashes, f, indent=1, sort_keys=True)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
