"""GPU parity: the HIP path against the CPU oracle, element by element.

Every bit array A_d and C_d, the rank table, the fallback table, the level sizes
and every label must be identical (bit-exact: the method is integer work whose
result does not depend on the order of the atomics)."""
import math

import numpy as np
import pytest
import torch

from oracle import mphf_oracle as O
from paper_1702_03154_amd import inputs as I

pytestmark = pytest.mark.gpu

U64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_03154_amd import mphf
    mphf.lib()
    return mphf


from tests.parity import check_against_oracle, host, keys_np  # noqa: E402


# ------------------------------------------------------------ hash + exact mod

@pytest.mark.parametrize("m", [1, 2, 3, 7, 64, 1000, 1_000_003, 2**31 - 1, 2_000_000_000, 2**32 - 1,
                               2**32, 2**32 + 15, 6_000_000_001, 2**40 - 3, 2**52 + 7, 2**62 + 1,
                               2**63 - 1])
def test_device_positions_equal_plain_mod(M, m):
    rng = np.random.default_rng(m % 1000)
    k = np.concatenate([np.array([0, 1, 2, U64, U64 - 1, 2**63, 2**63 - 1, 2**32, 2**32 - 1],
                                 dtype=np.uint64),
                        keys_np(20_000, seed=m % 97),
                        rng.integers(0, 2**63, size=2000, dtype=np.uint64) * np.uint64(2)])
    for seed in (0, 0x9E3779B97F4A7C15, U64):
        got = host(M.positions(torch.from_numpy(k.view(np.int64)).cuda(), seed, m))
        assert np.array_equal(got, O.level_positions(k, seed, m)), (m, seed)


def test_device_mod_on_hash_values_near_the_top(M):
    # keys chosen so that fmix64(key ^ 0) covers h near 2^64 - 1 is not controllable; instead use
    # the bijection: invert fmix64 on the host for chosen h values.
    inv1 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    inv2 = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)

    def unfmix(y):
        z = y ^ (y >> 33)
        z = (z * inv2) & U64
        z ^= z >> 33
        z = (z * inv1) & U64
        return z ^ (z >> 33)

    hs = [U64 - i for i in range(64)] + [(1 << 63) + i for i in range(-32, 32)] + list(range(64))
    k = np.array([unfmix(h) for h in hs], dtype=np.uint64)
    assert np.array_equal(O.fmix64(k), np.array(hs, dtype=np.uint64))
    for m in (3, 1000, 2**32 + 1, 2**61 - 1, 2**63 - 25):
        got = host(M.positions(torch.from_numpy(k.view(np.int64)).cuda(), 0, m))
        assert np.array_equal(got, np.array([h % m for h in hs], dtype=np.uint64))


# ------------------------------------------------------------ whole structure

@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 64, 100, 1000, 4097, 33_333, 100_000])
@pytest.mark.parametrize("gamma", [1.0, 2.0])
def test_parity_small(M, n, gamma):
    absent = keys_np(3000, seed=77)
    check_against_oracle(M, keys_np(n), gamma, queries_np=absent)


@pytest.mark.parametrize("gamma", [1.5, 3.7, 5.0, 10.0])
def test_parity_other_gammas(M, gamma):
    check_against_oracle(M, keys_np(50_000, seed=3), gamma, seed=11)


@pytest.mark.parametrize("seed", [0, 1, 12345, U64])
def test_parity_seeds(M, seed):
    check_against_oracle(M, keys_np(20_000, seed=5), 2.0, seed=seed)


def test_parity_config1_1e6_gamma2(M):
    """1e6 SplitMix64 keys (seed 1), gamma 2, every key queried in input order."""
    k = keys_np(1_000_000)
    assert len(np.unique(k)) == len(k)
    st = check_against_oracle(M, k, 2.0)
    assert len(st.fallback_keys) == 0


def test_parity_1e6_gamma1_with_fallback(M):
    st = check_against_oracle(M, keys_np(1_000_000), 1.0, queries_np=keys_np(100_000, seed=9))
    assert st.num_levels == 25 and len(st.fallback_keys) > 0


def test_parity_minirank(M):
    check_against_oracle(M, keys_np(200_000), 1.0, rank_sample=1024)


@pytest.mark.parametrize("max_levels", [1, 2, 3])
def test_parity_forced_fallback(M, max_levels):
    st = check_against_oracle(M, keys_np(100_000, seed=4), 2.0, max_levels=max_levels)
    assert len(st.fallback_keys) > 1000


def test_parity_structured_keys(M):
    # dense small integers and a strided set: the hash must still spread them
    k = np.concatenate([np.arange(1, 50_001, dtype=np.uint64),
                        np.arange(50_001, dtype=np.uint64) * np.uint64(2**40) + np.uint64(2**63)])
    check_against_oracle(M, np.unique(k), 2.0)


def test_order_independence_on_gpu(M):
    k = keys_np(300_000)
    t = torch.from_numpy(k.view(np.int64)).cuda()
    a = M.build(t, 2.0, 0)
    perm = torch.randperm(len(k), generator=torch.Generator().manual_seed(3)).cuda()
    b = M.build(t[perm].contiguous(), 2.0, 0)
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["words"], eb["words"]) and np.array_equal(ea["rank"], eb["rank"])
    assert torch.equal(a.lookup(t), b.lookup(t))


def test_repeat_builds_identical(M):
    t = torch.from_numpy(keys_np(200_000).view(np.int64)).cuda()
    ref = M.build(t, 1.0, 0).export()["words"]
    for _ in range(3):
        assert np.array_equal(M.build(t, 1.0, 0).export()["words"], ref)


# ------------------------------------------------------------ errors and edge cases

def test_duplicate_keys(M):
    k = keys_np(10_000)
    k[9000] = k[10]
    with pytest.raises(M.DuplicateKeysError):
        M.build(torch.from_numpy(k.view(np.int64)).cuda(), 2.0)


def test_invalid_arguments(M):
    t = torch.from_numpy(keys_np(100).view(np.int64)).cuda()
    for g in (0.99, float("nan"), float("inf"), -2.0):
        with pytest.raises(M.MphfError) as e:
            M.build(t, g)
        assert e.value.status == M.E_INVALID
    for kw in ({"max_levels": 0}, {"max_levels": 65}, {"rank_sample": 256}):
        with pytest.raises(M.MphfError):
            M.build(t, 2.0, **kw)


def test_host_pointer_rejected(M):
    import ctypes
    k = keys_np(16)
    h = ctypes.c_void_p()
    st = M.lib().mphf_build_ex(k.ctypes.data, 16, 2.0, 0, None, None, ctypes.byref(h))
    assert st == M.E_INVALID and not h.value


def test_mem_budget(M):
    t = torch.from_numpy(keys_np(100_000).view(np.int64)).cuda()
    with pytest.raises(M.MphfError) as e:
        M.build(t, 2.0, mem_budget=4096)
    assert e.value.status == M.E_NOMEM
    h = M.build(t, 2.0, mem_budget=64 << 20)
    assert 0 < h.stats()["peak_bytes"] <= 64 << 20


def test_empty_and_single(M):
    e = torch.zeros(0, dtype=torch.int64, device="cuda")
    h = M.build(e, 2.0)
    assert h.stats()["num_levels"] == 0
    q = torch.from_numpy(keys_np(10).view(np.int64)).cuda()
    assert h.lookup(q).tolist() == [0] * 10
    one = q[:1].contiguous()
    h1 = M.build(one, 1.0)
    assert h1.lookup(one).tolist() == [1]


def test_concurrent_lookups_on_streams(M):
    k = keys_np(500_000)
    t = torch.from_numpy(k.view(np.int64)).cuda()
    h = M.build(t, 2.0)
    ref = h.lookup(t)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(4)]
    outs = []
    for i, s in enumerate(streams):
        with torch.cuda.stream(s):
            outs.append(h.lookup(t[i::4].contiguous(), stream=s))
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert torch.equal(o, ref[i::4])


# ------------------------------------------------------------ build strategies

def unfmix64(y):
    inv1 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    inv2 = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)
    z = y ^ (y >> 33)
    z = (z * inv2) & U64
    z ^= z >> 33
    z = (z * inv1) & U64
    return z ^ (z >> 33)


def test_parity_one_pass_partition_with_wide_digits(M):
    """N = 5e6 at gamma 2: level 0 has ceil(1e7 / 2^15) = 306 buckets of the default size, more
    than 256 and at most 1024, so one radix pass with 10-bit digits."""
    def want(p):
        assert p[0] == "one_pass" and p[-1] == "tail", p
    check_against_oracle(M, keys_np(5_000_000, seed=21), 2.0, paths=want)


@pytest.mark.parametrize("gamma", [1.0, 2.0])
def test_parity_two_pass_partition(M, gamma):
    """N = 2e7: level 0 has ceil(gamma 2e7 / 2^b) = 1221 buckets of the default size (b = 14 at
    gamma 1, 15 at gamma 2), more than 1024, so a pass into coarse bins and a second pass into the
    buckets; the later levels take one pass, then the one-workgroup tail."""
    def want(p):
        assert p[0] == "two_pass" and "one_pass" in p and p[-1] == "tail", p
    check_against_oracle(M, keys_np(20_000_000, seed=21), gamma, paths=want)


@pytest.mark.parametrize("n,gamma,bits,first", [
    (5_000_000, 2.0, 10, "two_pass"),          # 9766 buckets: 2^6 buckets per coarse bin
    (5_000_000, 1.0, 8, "two_pass"),           # 19532 buckets: 2^7 per coarse bin
    (10_000_000, 2.0, 8, "two_pass_wide"),     # 78125 buckets: 2^9 per coarse bin (10-bit pass)
    (10_000_000, 2.0, 7, "two_pass_wide"),     # 156250 buckets: 2^10 per coarse bin
    (10_000_000, 2.0, 6, "atomic"),            # 312500 > 2^18 buckets: global atomics
])
def test_parity_small_buckets(M, n, gamma, bits, first):
    """Buckets smaller than the default make the level of a small key set as many buckets as a
    level of 1e9-1e10 keys has: the two-pass partition with 2^9 and 2^10 buckets per coarse bin
    (which the default buckets need only past about 2.1e9 keys per level), and past 2^18 buckets
    the global-atomic levels.  Every bit, counter and label must still equal the oracle's."""
    def want(p):
        assert p[0] == first, p
        if first != "atomic":
            assert "one_pass" in p and p[-1] == "tail", p
        else:
            assert set(p) == {"atomic"}, p
    check_against_oracle(M, keys_np(n, seed=22 + bits), gamma, bucket_bits=bits, paths=want,
                         queries_np=keys_np(20_000, seed=99))


def test_bucket_bits_rejected_when_too_large(M):
    t = torch.from_numpy(keys_np(1000).view(np.int64)).cuda()
    for bits in (5, 17, 16):          # 2^16 positions at gamma 2: 32768 keys, more than fit
        with pytest.raises(M.MphfError) as e:
            M.build(t, 2.0, bucket_bits=bits)
        assert e.value.status == M.E_INVALID


@pytest.mark.parametrize("n,gamma", [(1000, 2.0), (100_000, 2.0), (1_000_000, 1.0)])
def test_parity_atomic_levels(M, n, gamma):
    """The global-atomic build (MPHF_FLAG_ATOMIC_LEVELS) gives the same structure."""
    k = keys_np(n, seed=8)
    t = torch.from_numpy(k.view(np.int64)).cuda()
    ha = M.build(t, gamma, 0, atomic_levels=True)
    assert set(ha.stats()["level_path"]) == {"atomic"}
    hb = M.build(t, gamma, 0)
    assert ha.stats()["level_n"] == hb.stats()["level_n"]
    assert np.array_equal(ha.export()["words"], hb.export()["words"])
    st_o = O.build(k, gamma, 0)
    assert np.array_equal(ha.export()["words"], st_o.words)
    assert np.array_equal(host(ha.lookup(t)), O.lookup(st_o, k))


def test_bucket_overflow_falls_back_to_atomic_levels(M):
    """Adversarial keys: 20000 of them land in the first 32768 positions of level 0, more than a
    bucket's LDS holds, so the level is redone with global atomics; the result must not change."""
    n, gamma = 60_000, 2.0
    m0 = math.ceil(gamma * n)
    s0 = O.level_seeds(0, 1)[0]
    rng = np.random.default_rng(4)
    pos = rng.integers(0, 32768, size=20_000)
    hs = set()
    out = []
    q = 0
    for p in pos.tolist():           # h = p + j * m0 has h mod m0 = p
        h = p + (int(rng.integers(1, 2**40)) * m0)
        if h not in hs and h <= U64:
            hs.add(h)
            out.append(unfmix64(h) ^ s0)
    rest = keys_np(n - len(out), seed=31)
    k = np.unique(np.concatenate([np.array(out, dtype=np.uint64), rest]))
    assert np.sum(O.level_positions(k, s0, math.ceil(gamma * len(k))) < 32768) > 18_000
    check_against_oracle(M, k, gamma)


def test_tail_only_sizes(M):
    # every size up to one workgroup's LDS is built by the single-workgroup kernel
    for n in (7, 1000, 16_000, 16_384, 16_385, 20_000):
        check_against_oracle(M, keys_np(n, seed=n), 2.0)


def test_level1_bucket_overflow_falls_back_with_hashed_survivors(M):
    """Keys crafted so that level 0 builds by partition but one bucket of level 1 (2^8 positions,
    room for 347 keys) receives more than 400: level 1 and the levels after it are redone with global
    atomics from level 0's partitioned survivors, and every bit, counter and label must still equal the
    oracle's."""
    gamma, bits = 2.0, 8
    rest = keys_np(100_000, seed=57)
    n_adv_groups, per_group = 20, 20
    N = len(rest) + n_adv_groups * per_group
    m0 = math.ceil(gamma * N)
    s0, s1 = O.level_seeds(0, 2)
    rng = np.random.default_rng(11)
    # level-0 positions of the groups: one per distinct bucket of 2^8 positions
    p0s = (rng.choice(m0 >> bits, size=n_adv_groups, replace=False).astype(np.int64) << bits) + 7
    # |F_1| does not depend on which keys of a group are chosen (each group collides at its p0), so
    # m1 follows from the random keys and the groups' positions alone
    pos_rest = O.level_positions(rest, s0, m0).astype(np.int64)
    cnt = np.bincount(np.concatenate([pos_rest, np.repeat(p0s, per_group)]), minlength=m0)
    n1 = int((cnt[pos_rest] >= 2).sum()) + n_adv_groups * per_group
    m1 = math.ceil(gamma * n1)
    inv1 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    inv2 = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)
    adv = []
    for p0 in p0s.tolist():
        found = 0
        while found < per_group:
            js = rng.integers(1, 2**40, size=4096).astype(object)
            hs = [p0 + int(j) * m0 for j in js]
            xs = np.array([unfmix64(h) ^ s0 for h in hs], dtype=np.uint64)
            ok = O.level_positions(xs, s1, m1) < (1 << bits)
            for x in xs[ok].tolist():
                if found < per_group:
                    adv.append(x)
                    found += 1
    k = np.concatenate([rest, np.array(adv, dtype=np.uint64)])
    assert len(np.unique(k)) == len(k) == N
    st = O.build(k, gamma, 0)
    assert st.levels[1].n == n1 and st.levels[1].m == m1
    # every crafted key survives level 0 and lands in level 1's first bucket: 400 > 347 keys
    assert np.all(O.level_positions(np.array(adv, dtype=np.uint64), s1, m1) < (1 << bits))

    def want(p):
        assert p[0] == "one_pass" and set(p[1:]) == {"atomic"}, p
    check_against_oracle(M, k, gamma, bucket_bits=bits, paths=want, queries_np=keys_np(5000, seed=58))


@pytest.mark.parametrize("mode", ["1", "0", "reject"])
@pytest.mark.parametrize("n,gamma", [(200_000, 2.0), (200_000, 1.0), (3_000_000, 2.0), (20_000_000, 2.0)])
def test_levels_queued_ahead(M, monkeypatch, mode, n, gamma):
    """A partitioned level is queued before the host knows its key count, sized for bounds on the
    survivors of the level before it, with its level hash derived on the device; a level whose count
    falls outside the bounds does nothing and is queued again exactly.  On (the default), off, and a
    mode whose bounds nearly every level misses (so the redo runs at every level after the first)
    must all give the oracle's structure and labels, on one-pass and two-pass levels."""
    monkeypatch.setenv("MPHF_LEVELS_AHEAD", mode)
    check_against_oracle(M, keys_np(n, seed=n + 3), gamma, queries_np=keys_np(3000, seed=99))


def test_levels_queued_ahead_after_a_level0_overflow(M, monkeypatch):
    """Adversarial keys overflow a level-0 bucket: the level queued ahead sees the overflow flag and
    does nothing, and the atomic redo from level 0 must equal the oracle."""
    monkeypatch.setenv("MPHF_LEVELS_AHEAD", "1")
    test_bucket_overflow_falls_back_to_atomic_levels(M)


def test_concurrent_builds_on_threads_and_streams(M):
    """Four host threads build at once, each on its own stream: one takes the device's cached
    workspace, the others private temporaries, each polls its own reports and queues its levels
    ahead.  Every function must equal the oracle's (bits, rank table, labels)."""
    import threading

    sets = [keys_np(300_000 + 20_000 * i, seed=70 + i) for i in range(4)]
    tens = [torch.from_numpy(k.view(np.int64)).cuda() for k in sets]
    streams = [torch.cuda.Stream() for _ in sets]
    torch.cuda.synchronize()
    built, errors = [None] * len(sets), []

    def run(i):
        try:
            with torch.cuda.stream(streams[i]):
                built[i] = M.build(tens[i], 2.0, seed=i, stream=streams[i])
        except Exception as e:   # reported below
            errors.append(e)

    ts = [threading.Thread(target=run, args=(i,)) for i in range(len(sets))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, k in enumerate(sets):
        st = O.build(k, 2.0, i)
        ex = built[i].export()
        assert np.array_equal(ex["words"], st.words), i
        assert np.array_equal(ex["rank"], st.rank), i
        assert built[i].stats()["level_n"] == [l.n for l in st.levels], i
        assert np.array_equal(host(built[i].lookup(tens[i])), O.lookup(st, k)), i
