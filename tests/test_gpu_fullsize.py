"""Full-size checks (1e9 keys, the benchmark's workload, and a 4.5e8-key level of 4.5e9 positions)
of the HIP build and lookup.

The CPU oracle cannot build 1e9 keys in seconds, so at these sizes the structure is checked against
the method's definition restated with plain torch operations on the GPU, written independently of
the HIP kernels (its own fmix64, a long division for the mod, a bincount per level, a filter per
level), fed only with the seeded keys, gamma and the level seeds of the oracle's generator -- never
with anything the HIP path computed:

* level d: n_d keys F_d, m_d = ceil(gamma n_d); A_d[i] = [exactly one key of F_d at i],
  C_d[i] = [two or more]; F_{d+1} = the keys of F_d whose position holds two or more
  (Section 2.2, Algorithms 1 and 2); every word of every A_d and C_d must match;
* the leftovers after the last level are the fallback keys, ascending (Section 3, "Termination");
* the rank table holds the ones before every 512th position (Section 3.1);
* every query's label equals the ones of A before the key's first set bit plus one (Section 2.1,
  Algorithm 3), or its place in the fallback table; all of them, chunk by chunk.
"""
import math

import numpy as np
import pytest
import torch

from oracle import mphf_oracle as O
from paper_1702_03154_amd import inputs as I

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
    """fmix64(key ^ seed) mod m for m < 2^47, in int64 arithmetic: schoolbook long division of the
    64-bit hash by m in four 16-bit digits, r <- (r 2^16 + digit) mod m (every r 2^16 < 2^63)."""
    assert 0 < m < 2**47
    h = t_fmix64(keys ^ _s64(seed))
    r = torch.remainder(_srl(h, 48), m)
    for sh in (32, 16, 0):
        r = torch.remainder(r * (1 << 16) + ((h >> sh) & 0xFFFF), m)
    return r


def test_t_pos_is_the_unsigned_mod():
    """The torch restatement against the oracle's plain unsigned mod, on the CPU: hashes near 2^64
    and moduli across 2^31, 2^32 and beyond."""
    rng = np.random.default_rng(5)
    keys = rng.integers(-2**63, 2**63 - 1, size=4000, dtype=np.int64)
    keys[:4] = [-1, 0, 2**63 - 1, -2**63]
    kt = torch.from_numpy(keys)
    for m in (1, 3, 2**31 - 1, 2**31, 2**32 - 1, 2**32 + 7, 4_500_000_003, 2**46 + 5):
        for seed in (0, 0xE220A8397B1DCDAF):
            got = t_pos(kt, seed, m).numpy()
            want = O.level_positions(keys.view(np.uint64), seed, m).astype(np.int64)
            assert np.array_equal(got, want), (m, seed)


def test_t_words_and_popcount_on_the_cpu():
    """The packing and popcount helpers against numpy, bit 63 included."""
    pos = torch.tensor([0, 5, 63, 64, 127, 130], dtype=torch.int64)
    w = t_words(pos, 3).numpy().view(np.uint64)
    assert w.tolist() == [(1 << 0) | (1 << 5) | (1 << 63), (1 << 0) | (1 << 63), 1 << 2]
    x = torch.tensor([-1, 0, 1, -2**63, 0x0123456789ABCDEF], dtype=torch.int64)
    assert t_popcount64(x).tolist() == [64, 0, 1, 1, bin(0x0123456789ABCDEF).count("1")]


def t_popcount64(x):
    x = x - (_srl(x, 1) & 0x5555555555555555)
    x = (x & 0x3333333333333333) + (_srl(x, 2) & 0x3333333333333333)
    x = (x + _srl(x, 4)) & 0x0F0F0F0F0F0F0F0F
    return _srl(x * 0x0101010101010101, 56)


def t_words(pos, nwords):
    """int64 words with bit p % 64 of word p // 64 set for each of the distinct positions pos: the
    sum of distinct powers of two (in two's complement for bit 63) is their bitwise or."""
    w = torch.zeros(nwords, dtype=torch.int64, device=pos.device)
    return w.index_add_(0, pos >> 6, torch.ones_like(pos) << (pos & 63))


def _flip(t):
    """Unsigned order of int64 words: flip the sign bit."""
    return t ^ _s64(1 << 63)


def definition_check(M, n, gamma, key_seed=1):
    """Build n keys of the SplitMix64 stream key_seed and check the structure and every label
    against the definition.  Returns the build's stats."""
    keys = I.keys(n, seed=key_seed, device="cuda")
    h = M.build(keys, gamma, 0, keep_collisions=True)
    st = h.stats()
    v = h.device_views()
    seeds = O.level_seeds(0, 25)
    assert st["level_seed"] == seeds[:st["num_levels"]]
    alive = keys
    off = 0
    for d in range(st["num_levels"]):
        nd = alive.numel()
        m = math.ceil(gamma * nd)
        assert (st["level_n"][d], st["level_m"][d], st["level_offset"][d]) == (nd, m, off), d
        p = t_pos(alive, seeds[d], m)
        # keys per occupied position: the distinct positions (ascending) and how many keys each holds
        u, inv, c = torch.unique(p, return_inverse=True, return_counts=True)
        del p
        wd = (m + 63) // 64
        for got, want in ((v["words"], u[c == 1]), (v["collisions"], u[c >= 2])):
            assert torch.equal(got[off // 64: off // 64 + wd], t_words(want, wd)), d
        assert st["level_weight"][d] == int((c == 1).sum())
        alive = alive[c[inv] >= 2]
        del u, inv, c
        off += 64 * wd
    assert st["total_bits"] == off
    assert st["n_fallback"] == alive.numel()
    fbk = v["fallback_keys"]
    assert torch.equal(_flip(torch.sort(_flip(alive)).values), fbk)
    # rank table
    pc = t_popcount64(v["words"])
    ones = torch.cumsum(pc, 0) - pc
    del pc
    per = 512 // 64
    assert torch.equal(v["rank"], ones[::per])
    # every label of the shuffled queries: the first level whose bit is set gives the ones before
    # it plus one; a key that finds none is in the fallback table (labels N - |L| + 1 ..)
    q = I.shuffled_queries(keys, seed=2)
    del keys
    lab = h.lookup(q)
    nfb = st["n_fallback"]
    fbs = _flip(fbk)
    QC = 1 << 25
    for q0 in range(0, n, QC):
        x = q[q0:q0 + QC]
        want = torch.zeros(x.numel(), dtype=torch.int64, device="cuda")
        idx = torch.arange(x.numel(), device="cuda")
        for d in range(st["num_levels"]):
            if not idx.numel():
                break
            g = st["level_offset"][d] + t_pos(x[idx], seeds[d], st["level_m"][d])
            word = v["words"][g >> 6]
            hit = ((word >> (g & 63)) & 1) == 1
            below = t_popcount64(word & ((torch.ones_like(g) << (g & 63)) - 1))
            want[idx[hit]] = (ones[g >> 6] + below + 1)[hit]
            idx = idx[~hit]
        if idx.numel():
            assert nfb > 0, q0
            xs = _flip(x[idx])
            pos = torch.searchsorted(fbs, xs)
            assert torch.equal(fbs[pos.clamp(max=nfb - 1)], xs), q0     # every query is a member
            want[idx] = n - nfb + 1 + pos
        assert torch.equal(lab[q0:q0 + QC], want), q0
    assert int(lab.min()) == 1 and int(lab.max()) == n
    h.close()
    return st


@pytest.mark.gpu
@pytest.mark.slow
@pytest.mark.parametrize("gamma", [2.0, 1.0])
def test_full_size_structure_equals_definition(M, gamma):
    st = definition_check(M, N, gamma)
    assert st["level_path"][0] == "two_pass"
    if gamma == 1.0:
        assert st["num_levels"] == 25 and st["n_fallback"] > 0


@pytest.mark.gpu
@pytest.mark.slow
def test_wide_partition_and_offsets_past_2_32_equal_definition(M):
    """4.5e8 keys at gamma 10: level 0 has 4.5e9 positions, ceil(4.5e9 / 2^16) = 68665 > 2^16
    buckets, so the second partition pass takes 2^9 buckets per coarse bin (the wide pass, as the
    4e9-key k-mer workload at gamma 2 does), and the concatenated A holds about 5e9 > 2^32 bits, so
    bit offsets, ranks and labels take 64-bit arithmetic."""
    st = definition_check(M, 450_000_000, 10.0, key_seed=3)
    assert st["level_path"][0] == "two_pass_wide"
    assert st["level_m"][0] > 2**32 and st["total_bits"] > 2**32
