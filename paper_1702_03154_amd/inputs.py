"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds none of the method's arithmetic: no level hash, no bit
arrays, no rank.  It only produces the workloads the paper measures on:

* distinct pseudo-random 64-bit integer keys (paper, Section 4, results setup:
  unique random integers in [0, 2^64)), drawn here as the outputs of a
  SplitMix64 stream (Steele, Lea and Flood, OOPSLA 2014).  Output i of the
  stream is a bijective mix of ``seed + (i + 1) * golden``, so the first N
  outputs are distinct for any N below 2^64 and no de-duplication is needed;
* many independent key sets of log-uniform sizes (the batched workload): the
  size of set j is floor(lo * (hi/lo)^u_j) with u_j the top 53 bits of output
  j of a SplitMix64 stream over 2^53, and set j holds the first size_j outputs
  of the SplitMix64 stream seeded with output j of a second stream;
* a DNA sequence for the k-mer workload: 2 bits per base (A=0, C=1, G=2, T=3),
  32 bases per SplitMix64 output, the first base in the two most significant bits;
* a seeded permutation of [0, N) for the shuffled query order: a 4-round
  balanced Feistel network on 2h bits (2^(2h) >= N) with cycle walking
  (Black and Rogaway, CT-RSA 2002), so it is a bijection of [0, N).

Everything is computed with int64 torch ops (two's-complement wraparound holds
the uint64 bit pattern), so the same code runs on the CPU for the oracle and
on the GPU for the large workloads, and both sides see identical keys.
"""
from __future__ import annotations

import torch

_GOLDEN = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


def _s64(c: int) -> int:
    """uint64 constant -> the int64 with the same bit pattern."""
    c &= (1 << 64) - 1
    return c - (1 << 64) if c >= (1 << 63) else c


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor holding uint64 bits."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _s64(_MIX1)
    z = (z ^ _srl(z, 27)) * _s64(_MIX2)
    return z ^ _srl(z, 31)


def splitmix64(seed: int, count: int, start: int = 0, device="cpu",
               chunk: int = 1 << 27) -> torch.Tensor:
    """Outputs start .. start+count-1 of the SplitMix64 stream seeded with ``seed``.

    Returns an int64 tensor whose bits are the uint64 outputs.  Output i is
    mix(seed + (i + 1) * 0x9E3779B97F4A7C15).
    """
    out = torch.empty(count, dtype=torch.int64, device=device)
    for lo in range(0, count, chunk):
        hi = min(count, lo + chunk)
        z = torch.arange(start + lo + 1, start + hi + 1, dtype=torch.int64, device=device)
        z = z * _s64(_GOLDEN) + _s64(seed)
        out[lo:hi] = _mix(z)
    return out


def splitmix64_py(seed: int, count: int, start: int = 0) -> list:
    """Pure-Python SplitMix64 (same stream as :func:`splitmix64`), for tiny cases."""
    m = (1 << 64) - 1
    res = []
    for i in range(start, start + count):
        z = (seed + (i + 1) * _GOLDEN) & m
        z = ((z ^ (z >> 30)) * _MIX1) & m
        z = ((z ^ (z >> 27)) * _MIX2) & m
        res.append(z ^ (z >> 31))
    return res


def keys(n: int, seed: int = 1, device="cpu") -> torch.Tensor:
    """The key set used everywhere: the first n SplitMix64 outputs of ``seed``."""
    return splitmix64(seed, n, 0, device)


def feistel_permutation(n: int, seed: int = 2, device="cpu", rounds: int = 4) -> torch.Tensor:
    """A seeded bijection of [0, n) as an int64 index tensor (position j -> pi(j))."""
    if n <= 1:
        return torch.zeros(n, dtype=torch.int64, device=device)
    bits = max(2, (n - 1).bit_length())
    h = (bits + 1) // 2
    mask = (1 << h) - 1
    round_keys = splitmix64_py(seed, rounds)

    def perm(x: torch.Tensor) -> torch.Tensor:
        left = _srl(x, h) & mask
        right = x & mask
        for rk in round_keys:
            f = _mix(right ^ _s64(rk)) & mask
            left, right = right, left ^ f
        return (left << h) | right

    x = perm(torch.arange(n, dtype=torch.int64, device=device))
    while True:
        out = x >= n
        if not bool(out.any()):
            return x
        x[out] = perm(x[out])


def shuffled_queries(k: torch.Tensor, seed: int = 2) -> torch.Tensor:
    """The keys of ``k`` in a seeded Feistel-shuffled order."""
    pi = feistel_permutation(k.numel(), seed, device=k.device)
    return k[pi]


def log_uniform_sizes(nsets: int, lo: int = 16, hi: int = 65536, seed: int = 3) -> torch.Tensor:
    """Set sizes floor(lo * (hi/lo)^u_j), u_j = (output j of SplitMix64(seed)) >> 11 over 2^53.

    Computed on the CPU in float64 (int64 tensor); a size never exceeds ``hi``."""
    z = splitmix64(seed, nsets)
    u = _srl(z, 11).to(torch.float64) / float(1 << 53)
    sizes = torch.floor(float(lo) * torch.pow(torch.tensor(float(hi) / float(lo), dtype=torch.float64), u))
    return sizes.to(torch.int64).clamp_(max=hi)


def set_offsets(sizes: torch.Tensor) -> torch.Tensor:
    """Exclusive prefix of the set sizes, nsets + 1 entries, int64 on the sizes' device."""
    off = torch.zeros(sizes.numel() + 1, dtype=torch.int64, device=sizes.device)
    torch.cumsum(sizes, 0, out=off[1:])
    return off


def set_keys(sizes: torch.Tensor, seed: int = 4, device="cpu", chunk: int = 1 << 26) -> torch.Tensor:
    """Concatenated keys of the sets: set j is the first sizes[j] outputs of SplitMix64 seeded
    with output j of SplitMix64(seed), so each set's keys are distinct."""
    sizes = sizes.to(device)
    nsets = sizes.numel()
    set_seeds = splitmix64(seed, nsets, device=device)
    off = set_offsets(sizes)
    total = int(off[-1])
    out = torch.empty(total, dtype=torch.int64, device=device)
    set_of = torch.repeat_interleave(torch.arange(nsets, device=device), sizes)
    for lo in range(0, total, chunk):
        hi = min(total, lo + chunk)
        j = set_of[lo:hi]
        i = torch.arange(lo, hi, dtype=torch.int64, device=device) - off[j]
        z = (i + 1) * _s64(_GOLDEN) + set_seeds[j]
        out[lo:hi] = _mix(z)
    return out


def dna_sequence(nbases: int, seed: int = 5, device="cpu") -> torch.Tensor:
    """A uniform random ACGT sequence of nbases bases, 2-bit packed (32 per word, first base in the
    top two bits): the first ceil(nbases/32) SplitMix64 outputs of ``seed``."""
    return splitmix64(seed, (nbases + 31) // 32, 0, device)
