"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
arithmetic: the brute force is a sequential state machine (Algorithm 2), the
worked example comes from the Figure 1 caption, and the statistics are the
closed forms of Section 2.3 and the textbook occupancy problem.
"""
import math
import os

import numpy as np
import pytest

from oracle import mphf_oracle as O
from paper_1702_03154_amd import inputs as I
from tests.brute import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _keys(n, seed=1):
    return I.keys(n, seed).numpy().view(np.uint64)


@pytest.fixture(scope="module")
def big():
    """N = 1e6 at gamma 1, 2 and 5 (the paper's gamma values, Table 1)."""
    k = _keys(1_000_000)
    return k, {g: O.build(k, g, 0) for g in (1.0, 2.0, 5.0)}


# ------------------------------------------------------------ hash family

def test_level_seeds_are_published_splitmix64_outputs():
    # SplitMix64 seeded with 0: the reference generator's first outputs.
    assert O.level_seeds(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_fmix64_is_a_bijection_with_the_expected_inverse():
    # x ^= x >> 33 is an involution on 64 bits; the multipliers are odd, so invertible mod 2^64.
    rng = np.random.default_rng(0)
    x = rng.integers(0, 2**63, size=4096, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    y = O.fmix64(x)
    inv1 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    inv2 = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)
    for xi, yi in zip(x.tolist()[:256], y.tolist()[:256]):
        z = yi ^ (yi >> 33)
        z = (z * inv2) & O.MASK64
        z ^= z >> 33
        z = (z * inv1) & O.MASK64
        z ^= z >> 33
        assert z == xi
    assert int(O.fmix64(np.array([0], np.uint64))[0]) == 0


def test_positions_are_plain_mod_of_the_hash():
    k = _keys(1000)
    for m in (1, 2, 3, 64, 1000, 2**33 + 1, 2**40 - 3):
        p = O.level_positions(k, 12345, m)
        assert int(p.max()) < m
        h = O.fmix64(k ^ np.uint64(12345))
        assert [int(a) % m for a in h[:50]] == [int(a) for a in p[:50]]


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("gamma", [1.0, 1.5, 2.0, 5.0])
def test_brute_force_agrees_with_oracle(gamma):
    for seed in range(12):
        for n in (0, 1, 2, 3, 5, 8, 17, 33, 64):
            keys = [int(v) for v in _keys(n, seed=100 + seed)]
            levels, left, labels, concat = brute(keys, gamma, seed)
            st = O.build(np.array(keys, dtype=np.uint64), gamma, seed)
            assert st.num_levels == len(levels)
            for lev, (m, A, C, F) in zip(st.levels, levels):
                assert lev.m == m and lev.n == len(F)
                assert lev.A.astype(int).tolist() == A
                assert lev.C.astype(int).tolist() == C
            assert [int(v) for v in st.fallback_keys] == left
            got = O.lookup(st, np.array(keys, dtype=np.uint64))
            assert [int(v) for v in got] == [labels[x] for x in keys]
            bits = np.unpackbits(st.words.view(np.uint8), bitorder="little")[:st.total_bits]
            assert bits.tolist() == concat


def test_brute_force_with_forced_fallback():
    keys = [int(v) for v in _keys(40, seed=7)]
    levels, left, labels, _ = brute(keys, 1.0, 3, max_levels=2)
    st = O.build(np.array(keys, dtype=np.uint64), 1.0, 3, max_levels=2)
    assert [int(v) for v in st.fallback_keys] == left and len(left) > 0
    got = O.lookup(st, np.array(keys, dtype=np.uint64))
    assert [int(v) for v in got] == [labels[x] for x in keys]


# ------------------------------------------------------------ worked example

def _fig1():
    rows = []
    with open(os.path.join(GOLDEN, "fig1_worked_example.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    keys = np.array([int(r[0][1:]) for r in rows], dtype=np.uint64)   # k1..k6 -> 1..6
    pos = {int(r[0][1:]): [None if v == "-" else int(v) for v in r[1:4]] for r in rows}
    level = [int(r[4]) for r in rows]
    label = [int(r[5]) for r in rows]
    return keys, pos, level, label


def test_figure1_worked_example_labels():
    keys, pos, level, label = _fig1()

    def positions(ks, d, m):
        out = []
        for x in ks.tolist():
            p = pos[int(x)][d]
            assert p is not None and p < m
            out.append(p)
        return np.array(out, dtype=np.uint64)

    st = O.build(keys, 1.0, 0, positions=positions)
    assert [lev.m for lev in st.levels] == [6, 4, 2]
    assert [lev.n for lev in st.levels] == [6, 4, 2]
    assert O.lookup(st, keys, positions=positions).tolist() == label
    # the brute force agrees on the same positions
    _, _, labels, _ = brute([int(k) for k in keys], 1.0, 0,
                            pos=lambda x, d, m: pos[x][d])
    assert [labels[int(k)] for k in keys] == label
    # levels: k3, k6 at level 0; k1, k5 at 1; k2, k4 at 2
    got_level = []
    for x in keys.tolist():
        for d in range(3):
            if st.levels[d].A[pos[int(x)][d]]:
                got_level.append(d)
                break
    assert got_level == level


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("gamma", [1.0, 2.0, 5.0])
def test_invariants(big, gamma):
    k, sts = big
    st = sts[gamma]
    N = len(k)
    for d, lev in enumerate(st.levels):
        assert not np.any(lev.A & lev.C)                      # footnote of Algorithm 2
        nxt = st.levels[d + 1].n if d + 1 < st.num_levels else len(st.fallback_keys)
        assert lev.weight == lev.n - nxt
        assert lev.m == math.ceil(gamma * lev.n)
    assert sum(lev.weight for lev in st.levels) + len(st.fallback_keys) == N
    lab = O.lookup(st, k)
    assert np.array_equal(np.sort(lab), np.arange(1, N + 1, dtype=np.uint64))   # bijection onto [1, N]
    # ordering the placed keys by their bit in the concatenated A gives 1 .. N - |L|
    lvl = O.level_of(st, k)
    g = np.full(N, -1, dtype=np.int64)
    for d, lev in enumerate(st.levels):
        sel = lvl == d
        g[sel] = lev.offset + O.level_positions(k[sel], lev.seed, lev.m).astype(np.int64)
    placed = lvl < st.num_levels
    order = np.argsort(g[placed], kind="stable")
    assert np.array_equal(lab[placed][order], np.arange(1, placed.sum() + 1, dtype=np.uint64))


@pytest.mark.parametrize("rank_sample", [512, 1024])
def test_rank_table_is_prefix_popcount(rank_sample):
    k = _keys(30_000)
    st = O.build(k, 2.0, 0, rank_sample=rank_sample)
    per = rank_sample // 64
    expect, acc = [], 0
    for i, w in enumerate(st.words.tolist()):     # textbook: popcount word by word
        if i % per == 0:
            expect.append(acc)
        acc += bin(w).count("1")
    assert st.rank.tolist() == expect
    assert acc == 30_000 - len(st.fallback_keys)


def test_labels_equal_rank_table_plus_in_block_popcount():
    # the label through the sampled counters is the same as the plain prefix count
    k = _keys(20_000)
    st = O.build(k, 1.0, 0)
    lab = O.lookup(st, k)
    words = st.words.tolist()
    lvl = O.level_of(st, k)
    for x, d, want in list(zip(k.tolist(), lvl.tolist(), lab.tolist()))[:3000]:
        if d == st.num_levels:
            continue
        lev = st.levels[d]
        p = int(O.level_positions(np.array([x], np.uint64), lev.seed, lev.m)[0])
        g = lev.offset + p
        b = g // 512
        r = int(st.rank[b]) + sum(bin(w).count("1") for w in words[b * 8:g // 64])
        r += bin(words[g // 64] & ((1 << (g % 64)) - 1)).count("1")
        assert r + 1 == want


# ------------------------------------------------------------ statistics (Section 2.3)

def _occupancy(n, m):
    """Singleton bins when n balls fall uniformly into m bins: mean and standard deviation."""
    e = n * math.exp((n - 1) * math.log1p(-1.0 / m))
    exx = (m - 1) / m * n * (n - 1) * math.exp((n - 2) * math.log1p(-2.0 / m)) if n > 1 else 0.0
    return e, math.sqrt(max(exx + e - e * e, 0.0))


@pytest.mark.parametrize("gamma", [1.0, 2.0, 5.0])
def test_placed_per_level_matches_occupancy(big, gamma):
    _, sts = big
    for lev in sts[gamma].levels:
        if lev.n < 200:
            continue
        e, s = _occupancy(lev.n, lev.m)
        assert abs(lev.weight - e) <= 6 * s + 1, (lev.n, lev.m, lev.weight, e, s)
    lev0 = sts[gamma].levels[0]
    assert abs(lev0.weight / lev0.n - math.exp(-1 / gamma)) < 0.005   # e^{-1/gamma}


@pytest.mark.parametrize("gamma", [1.0, 2.0, 5.0])
def test_total_size_matches_space_analysis(big, gamma):
    _, sts = big
    st = sts[gamma]
    S = sum(lev.m for lev in st.levels) / st.N
    assert abs(S / (gamma * math.exp(1 / gamma)) - 1) < 0.01      # gamma e^{1/gamma} N bits
    bpk = st.bits_per_key
    assert abs(bpk / (1.125 * gamma * math.exp(1 / gamma)) - 1) < 0.01   # (1 + 64/512) factor


def test_bits_per_key_round_to_table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_bits_per_key.txt"))
            if l.strip() and not l.startswith("#")]
    k = _keys(1_000_000)
    for g, rs, printed in rows:
        st = O.build(k, float(g), 0, rank_sample=int(rs))
        assert round(st.bits_per_key, 1) == float(printed), (g, rs, st.bits_per_key)


@pytest.mark.parametrize("gamma,printed", [(1.0, 1.03), (2.0, 0.55), (5.0, 0.21)])
def test_disk_ratio_of_first_two_levels(big, gamma, printed):
    # Section 3.4: |F_1| + |F_2| is about 1.03 N, 0.55 N, 0.21 N for gamma = 1, 2, 5
    _, sts = big
    st = sts[gamma]
    r = (st.levels[1].n + st.levels[2].n) / st.N
    assert abs(r - printed) < 0.006


@pytest.mark.parametrize("gamma", [1.0, 2.0, 5.0])
def test_mean_probes(big, gamma):
    # Section 4.1: the average level of a key is e^{1/gamma} (counting from 1)
    k, sts = big
    lvl = O.level_of(sts[gamma], k)
    assert abs((lvl.mean() + 1) / math.exp(1 / gamma) - 1) < 0.01


def test_fallback_size_after_25_levels(big):
    # Section 3.5: about 1e-5 N keys reach H at gamma = 1, practically none at gamma >= 2
    _, sts = big
    n1 = len(sts[1.0].fallback_keys)
    assert 1 <= n1 <= 40
    assert len(sts[2.0].fallback_keys) == 0 and len(sts[5.0].fallback_keys) == 0
    assert sts[1.0].num_levels == 25


@pytest.mark.parametrize("gamma,case", [(2.0, "decreasing"), (1.0, "increasing")])
def test_construction_memory_lemma1(big, gamma, case):
    # Lemma 1: m(d) = sum_{i<d}|A_i| + 2|A_d|; max is m(0) = 2 e^{-1/gamma} S when gamma > 1/ln 2,
    # and at most S when gamma <= 1/ln 2.
    _, sts = big
    st = sts[gamma]
    sizes = [lev.m for lev in st.levels]
    S = sum(sizes)
    mem = [sum(sizes[:d]) + 2 * sizes[d] for d in range(len(sizes))]
    if case == "decreasing":
        assert mem.index(max(mem)) == 0
        assert abs(max(mem) / S - 2 * math.exp(-1 / gamma)) < 0.01
    else:
        assert max(mem) / S <= 1.0 + 1e-3


# ------------------------------------------------------------ forced paths and edge cases

def test_forced_fallback_labels_in_key_order():
    k = _keys(5000)
    st = O.build(k, 2.0, 0, max_levels=1)
    L = st.fallback_keys
    assert len(L) > 1000 and np.all(L[1:] > L[:-1])
    lab = O.lookup(st, L)
    assert np.array_equal(lab, np.arange(5000 - len(L) + 1, 5001, dtype=np.uint64))
    assert np.array_equal(np.sort(O.lookup(st, k)), np.arange(1, 5001, dtype=np.uint64))


def test_duplicate_keys_rejected():
    k = _keys(1000)
    k[500] = k[17]
    with pytest.raises(O.DuplicateKeysError):
        O.build(k, 2.0, 0)


def test_degenerate_inputs():
    st = O.build(np.zeros(0, np.uint64), 2.0, 0)
    assert st.num_levels == 0 and st.total_bits == 0 and len(st.rank) == 0
    assert O.lookup(st, _keys(5)).tolist() == [0] * 5
    st = O.build(_keys(1), 2.0, 0)
    assert st.levels[0].m == 2 and O.lookup(st, _keys(1)).tolist() == [1]
    st = O.build(_keys(1), 1.0, 0)
    assert st.levels[0].m == 1 and O.lookup(st, _keys(1)).tolist() == [1]
    for bad in (0.5, float("nan"), -1.0):
        with pytest.raises(ValueError):
            O.build(_keys(4), bad, 0)


def test_non_members_get_a_deterministic_value_in_range():
    k = _keys(50_000)
    st = O.build(k, 2.0, 0)
    absent = _keys(20_000, seed=99)
    a = O.lookup(st, absent)
    assert int(a.max()) <= 50_000
    assert np.array_equal(a, O.lookup(st, absent))


def test_order_independence():
    k = _keys(20_000)
    st = O.build(k, 2.0, 0)
    perm = np.random.default_rng(5).permutation(len(k))
    st2 = O.build(k[perm], 2.0, 0)
    assert np.array_equal(st.words, st2.words) and np.array_equal(st.rank, st2.rank)
    assert np.array_equal(O.lookup(st, k), O.lookup(st2, k))
