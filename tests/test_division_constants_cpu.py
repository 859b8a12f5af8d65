"""The exact division by an invariant integer that the kernels derive on the device (Granlund and
Montgomery 1994, Figure 4.1, for the levels sized inside a kernel): the same source compiled for the
host must give floor(n / m) for every m from 1 to 2^64 - 1, including m above 2^63 where 2^l - m
wraps, and numerators near 2^64.  No GPU: the constants are __host__ __device__ code."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1702_03154_amd", "csrc")

PROG = r"""
#include <cstdio>
#include <cstdint>
#include "device.h"
int main() {
    const uint64_t ms[] = {1ull, 2ull, 3ull, 7ull, 480ull, 1000003ull, (1ull << 32) - 1, 1ull << 32,
                           (1ull << 32) + 1, 6000000001ull, (1ull << 62) + 1, (1ull << 63) - 1, 1ull << 63,
                           (1ull << 63) + 1, 0xFFFFFFFFFFFFFFFFull, 0xFFFFFFFFFFFFFFFEull,
                           0xC000000000000001ull};
    uint64_t x = 0x9E3779B97F4A7C15ull, bad = 0, checked = 0;
    for (uint64_t m : ms) {
        const mphfk::LevelHash L = mphfk::device_level_hash(7, m, 0);
        for (int i = 0; i < 100000; ++i) {
            x ^= x << 13; x ^= x >> 7; x ^= x << 17;
            const uint64_t n = i < 64 ? ~0ull - (uint64_t)i : (i < 128 ? (uint64_t)(i - 64) : x);
            const uint64_t t = (uint64_t)(((unsigned __int128)L.magic * n) >> 64);
            const uint64_t q = (t + ((n - t) >> L.sh1)) >> L.sh2;
            bad += q != n / m;
            ++checked;
        }
    }
    printf("%llu %llu\n", (unsigned long long)checked, (unsigned long long)bad);
    return bad != 0;
}
"""


def test_device_division_constants_are_exact(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("no hipcc")
    src = tmp_path / "t.cpp"
    src.write_text(PROG)
    exe = tmp_path / "t"
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip", "-I", CSRC, "-o", str(exe),
                    str(src)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    checked, bad = (int(v) for v in r.stdout.split())
    assert r.returncode == 0 and checked == 1_700_000 and bad == 0
