"""The lookup's in-sector rank (device.h sector_count, both its forms), compiled for the host,
against a plain bit-by-bit count: random sectors (and all-ones, all-zeros, single-bit ones) at every bit position
0..479 of the 480 data bits."""
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
    uint64_t x = 0x243F6A8885A308D3ull, bad = 0, checked = 0;
    auto next = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    for (int t = 0; t < 3000; ++t) {
        uint32_t w[16];
        for (int k = 0; k < 16; ++k) {
            const uint32_t r = (uint32_t)next();
            w[k] = t == 0 ? 0xFFFFFFFFu : t == 1 ? 0u : t < 500 ? (1u << (r & 31)) : r;
        }
        w[0] = (uint32_t)(next() >> 40);   // the counter
        uint4 v[4];
        for (int c = 0; c < 4; ++c) v[c] = make_uint4(w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3]);
        for (uint32_t r = 0; r < 480; ++r) {
            const uint32_t word = 1 + r / 32, bit = r % 32;
            const bool set = (w[word] >> bit) & 1u;
            uint32_t want = w[0];
            for (uint32_t q = 0; q < r; ++q) want += (w[1 + q / 32] >> (q % 32)) & 1u;
            uint32_t got = 0xDEADBEEFu, got2 = 0xDEADBEEFu;
            const bool hit = mphfk::sector_count<true>(v, r, &got);
            const bool hit2 = mphfk::sector_count<false>(v, r, &got2);
            bad += hit != set || (set && got != want);
            bad += hit2 != set || (set && got2 != want);
            ++checked;
        }
    }
    printf("%llu %llu\n", (unsigned long long)checked, (unsigned long long)bad);
    return bad != 0;
}
"""


def test_sector_count_matches_a_bitwise_count(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    src = tmp_path / "t.cpp"
    src.write_text(PROG)
    exe = tmp_path / "t"
    subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", CSRC, "-o", str(exe),
                    str(src)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    checked, bad = (int(v) for v in r.stdout.split())
    assert r.returncode == 0 and checked == 3000 * 480 and bad == 0
