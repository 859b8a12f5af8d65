"""ctypes wrapper of the multithreaded CPU baseline (``threaded_baseline.cpp``).

TEST INFRASTRUCTURE ONLY: used by the tests and by the cpu_baseline leg of ``bench.py``, never by
the product.  The library is the paper-style parallel build (keys split over threads, atomic
fetch-or on the shared bit arrays, Section 3.2) and lookup, compiled with g++ for the host.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "threaded_baseline.cpp")
LIB = os.path.join(HERE, "libthreaded_baseline.so")

_lib = None


def compile_lib() -> str:
    """g++ build of the baseline (portable x86-64 code plus popcnt, so it runs on any host)."""
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O3", "-mpopcnt", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", tmp, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("g++ failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            compile_lib()
        L = C.CDLL(LIB)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        L.tb_build.restype = vp
        L.tb_build.argtypes = [vp, u64, C.c_double, u64, u32, u32, C.POINTER(C.c_int)]
        L.tb_lookup.restype = None
        L.tb_lookup.argtypes = [vp, vp, u64, vp, u32]
        L.tb_sizes.restype = None
        L.tb_sizes.argtypes = [vp, vp]
        L.tb_export.restype = None
        L.tb_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.tb_free.restype = None
        L.tb_free.argtypes = [vp]
        _lib = L
    return _lib


def host_threads() -> int:
    """Threads the baseline uses: the CPUs this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


class Threaded:
    """A function built by the threaded baseline."""

    def __init__(self, keys: np.ndarray, gamma: float, seed: int = 0, max_levels: int = 25,
                 threads: int | None = None):
        self.threads = threads or host_threads()
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        st = C.c_int(0)
        self._h = lib().tb_build(k.ctypes.data, len(k), float(gamma), seed & (2**64 - 1), max_levels,
                                 self.threads, C.byref(st))
        if not self._h:
            raise ValueError("duplicate keys" if st.value == 3 else "invalid arguments")

    def sizes(self):
        s = np.zeros(4, dtype=np.uint64)
        lib().tb_sizes(self._h, s.ctypes.data)
        return [int(v) for v in s]

    def export(self) -> dict:
        L, nw, nr, nf = self.sizes()
        w, r, f = (np.zeros(x, dtype=np.uint64) for x in (nw, nr, nf))
        ln, lm, lo = (np.zeros(64, dtype=np.uint64) for _ in range(3))
        lib().tb_export(self._h, w.ctypes.data, r.ctypes.data, f.ctypes.data, ln.ctypes.data, lm.ctypes.data,
                        lo.ctypes.data)
        return {"words": w, "rank": r, "fallback_keys": f, "level_n": ln[:L].tolist(),
                "level_m": lm[:L].tolist(), "level_offset": lo[:L].tolist()}

    def lookup(self, queries: np.ndarray) -> np.ndarray:
        q = np.ascontiguousarray(queries, dtype=np.uint64)
        out = np.zeros(len(q), dtype=np.uint64)
        lib().tb_lookup(self._h, q.ctypes.data, len(q), out.ctypes.data, self.threads)
        return out

    def close(self):
        if self._h:
            lib().tb_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
