"""Full-size checks (1e9 keys, the benchmark's workload) of the HIP build and lookup.

The CPU oracle cannot build 1e9 keys in seconds, so at this size the structure is checked against
the method's definition restated with plain torch operations on the GPU, written independently of
the HIP kernels (its own fmix64 and exact mod, a bincount per level, a filter per level), fed only
with the seeded keys, gamma and the level seeds of the oracle's generator -- never with anything the
HIP path computed:

* level d: n_d keys F_d, m_d = ceil(gamma n_d); A_d[i] = [exactly one key of F_d at i],
  C_d[i] = [two or more]; F_{d+1} = the keys of F_d whose position holds two or more
  (Section 2.2, Algorithms 1 and 2); every word of every A_d and C_d must match;
* the leftovers after the last level are the fallback keys, ascending (Section 3, "Termination");
* the rank table holds the ones before every 512th position (Section 3.1);
* every key's label is in [1, N] and no two keys share one (Section 1), and a sample of labels
  equals the ones of A before the key's bit plus one (Section 2.1, Algorithm 3).
"""
import math

import numpy as np
import pytest
import torch

from oracle import mphf_oracle as O
from paper_1702_03154_amd import inputs as I

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 1_000_000_000


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_03154_amd import mphf
    mphf.lib()
    return mphf


def _s64(c):
    c &= (1 << 64) - 1
    return c - (1 << 64) if c >= (1 << 63) else c


def _srl(z, s):
    return (z >> s) & ((1 << (64 - s)) - 1)


def t_fmix64(x):
    x = x ^ _srl(x, 33)
    x = x * _s64(0xFF51AFD7ED558CCD)
    x = x ^ _srl(x, 33)
    x = x * _s64(0xC4CEB9FE1A85EC53)
    return x ^ _srl(x, 33)


def t_pos(keys, seed, m):
    """fmix64(key ^ seed) mod m for m < 2^31, in int64 arithmetic: ((hi mod m) 2^32 + lo) mod m."""
    assert 0 < m < 2**31
    h = t_fmix64(keys ^ _s64(seed))
    hi = _srl(h, 32)
    lo = h & 0xFFFFFFFF
    return torch.remainder(torch.remainder(hi, m) * (1 << 32) + lo, m)


def t_popcount64(x):
    x = x - (_srl(x, 1) & 0x5555555555555555)
    x = (x & 0x3333333333333333) + (_srl(x, 2) & 0x3333333333333333)
    x = (x + _srl(x, 4)) & 0x0F0F0F0F0F0F0F0F
    return _srl(x * 0x0101010101010101, 56)


def t_pack(bits):
    """bool[64k] -> int64[k] words, bit i of word j = bits[64j + i]."""
    b = bits.view(-1, 64).to(torch.int64)
    shifts = torch.arange(64, device=bits.device, dtype=torch.int64)
    return (b << shifts).sum(dim=1)   # distinct powers of two: the sum is the bitwise or


def definition_check(M, gamma):
    keys = I.keys(N, seed=1, device="cuda")
    h = M.build(keys, gamma, 0, keep_collisions=True)
    st = h.stats()
    v = h.device_views()
    seeds = O.level_seeds(0, 25)
    assert st["level_seed"] == seeds[:st["num_levels"]]
    alive = keys
    off = 0
    for d in range(st["num_levels"]):
        n = alive.numel()
        m = math.ceil(gamma * n)
        assert (st["level_n"][d], st["level_m"][d], st["level_offset"][d]) == (n, m, off), d
        p = t_pos(alive, seeds[d], m)
        cnt = torch.bincount(p, minlength=m)
        wd = (m + 63) // 64
        pad = wd * 64 - m
        for got, want in ((v["words"], cnt == 1), (v["collisions"], cnt >= 2)):
            want = torch.cat([want, torch.zeros(pad, dtype=torch.bool, device="cuda")])
            for c0 in range(0, wd, 1 << 24):      # chunks of 2^24 words
                c1 = min(wd, c0 + (1 << 24))
                w = t_pack(want[c0 * 64:c1 * 64])
                assert torch.equal(got[off // 64 + c0: off // 64 + c1], w), (d, c0)
        assert st["level_weight"][d] == int((cnt == 1).sum())
        alive = alive[cnt[p] >= 2]
        del p, cnt
        off += 64 * wd
    assert st["total_bits"] == off
    left = torch.sort(alive).values
    assert st["n_fallback"] == left.numel()
    # fallback keys compare as unsigned: sort on the flipped sign bit
    flip = lambda t: t ^ _s64(1 << 63)
    assert torch.equal(flip(torch.sort(flip(alive)).values), v["fallback_keys"])
    # rank table
    pc = t_popcount64(v["words"])
    ones = torch.cumsum(pc, 0) - pc
    per = 512 // 64
    assert torch.equal(v["rank"], ones[::per])
    # labels: a bijection onto [1, N], and a sample equal to ones-before + 1
    q = I.shuffled_queries(keys, seed=2)
    lab = h.lookup(q)
    assert int(lab.min()) == 1 and int(lab.max()) == N
    seen = torch.zeros(N + 1, dtype=torch.bool, device="cuda")
    seen[lab] = True
    assert bool(seen[1:].all())
    del seen
    sample = q[:: N // 1_000_000][:1_000_000].contiguous()
    want = torch.zeros(sample.numel(), dtype=torch.int64, device="cuda")
    todo = torch.ones(sample.numel(), dtype=torch.bool, device="cuda")
    for d in range(st["num_levels"]):
        g = st["level_offset"][d] + t_pos(sample, seeds[d], st["level_m"][d])
        word = v["words"][g >> 6]
        bit = (word >> (g & 63)) & 1
        hit = todo & (bit == 1)
        below = t_popcount64(word & ((torch.ones_like(g) << (g & 63)) - 1))
        want = torch.where(hit, ones[g >> 6] + below + 1, want)
        todo &= ~hit
    assert not bool(todo.any()) or st["n_fallback"] > 0
    got = h.lookup(sample)
    assert torch.equal(got[~todo], want[~todo])
    h.close()


@pytest.mark.parametrize("gamma", [2.0, 1.0])
def test_full_size_structure_equals_definition(M, gamma):
    definition_check(M, gamma)
