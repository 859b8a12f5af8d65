"""Compile the HIP library ``libmphf.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SOURCES = ["kernels.hip", "partition.hip", "batch.hip", "kmer.hip", "stream.hip", "server.hip", "noalloc.hip", "probes.hip", "api.hip"]
LIB = os.path.join(PKG, "libmphf.so")
OBJ_DIR = os.path.join(PKG, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed FP32 instructions are disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    return r.returncode, msgs


def build(verbose: bool = False) -> str:
    """Every source compiled to an object in parallel (the kernels of one file call no device code
    of another), then linked into the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
        jobs.append((obj, [hipcc(), *compile_flags, *inc, "-c", "-o", obj, os.path.join(CSRC, src)]))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    for (obj, _), (rc, msgs) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(obj)}:\n" + msgs)
        if verbose and msgs:
            print(msgs)
    tmp = LIB + ".tmp"
    rc, msgs = _run([hipcc(), *HIPCC_FLAGS, "-o", tmp, *(o for o, _ in jobs)], verbose)
    if rc != 0:
        raise RuntimeError("hipcc link failed:\n" + msgs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
