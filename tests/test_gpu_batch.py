"""GPU parity of the batched build: every set of a batch against the oracle built on that set
alone, bit for bit (level sizes and offsets, the set's A words, its fallback keys, every label),
and against a standalone build of the same set through the plain entry point.

Sets are independent functions (Section 2: the levels of a key set depend only on its keys,
gamma and the level seeds), so a batch must reproduce each standalone result exactly."""
import math

import numpy as np
import pytest
import torch

from oracle import mphf_oracle as O
from paper_1702_03154_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_03154_amd import mphf
    mphf.lib()
    return mphf


def host(t):
    return t.cpu().numpy().view(np.uint64)


def make_sets(sizes, seed=4):
    sizes = torch.as_tensor(sizes, dtype=torch.int64)
    return sizes, I.set_keys(sizes, seed), I.set_offsets(sizes)


def sectors_from_words(words, total_bits):
    """The lookup sectors of a set laid out from its A words: 480 bits per sector, word 0 the ones
    of the set before the sector."""
    w32 = words.view(np.uint32) if len(words) else np.zeros(0, dtype=np.uint32)
    ns = (total_bits + 479) // 480
    out = np.zeros((ns, 16), dtype=np.uint32)
    run = 0
    for k in range(ns):
        chunk = w32[15 * k:15 * k + 15]
        out[k, 1:1 + len(chunk)] = chunk
        out[k, 0] = run
        run += int(sum(bin(int(v)).count("1") for v in chunk))
    return out


def check_set(b, s, ks, gamma, seed, max_levels, labels, sectors=True):
    st = O.build(ks, gamma, seed, max_levels=max_levels)
    info = b.set_info(s)
    assert info["n"] == len(ks)
    assert info["num_levels"] == st.num_levels, s
    assert info["level_n"] == [l.n for l in st.levels], s
    assert info["level_m"] == [l.m for l in st.levels], s
    assert info["level_offset"] == [l.offset for l in st.levels], s
    assert info["total_bits"] == st.total_bits, s
    assert info["n_fallback"] == len(st.fallback_keys), s
    ex = b.export_set(s)
    assert np.array_equal(ex["words"], st.words), s
    assert np.array_equal(ex["fallback_keys"], st.fallback_keys), s
    if sectors:
        assert np.array_equal(b.export_sectors(s), sectors_from_words(st.words, st.total_bits)), s
    assert np.array_equal(labels, O.lookup(st, ks)), s
    return st


def check_batch(M, sizes, gamma, seed=0, max_levels=25, check=None, absent=True, planned=False, launch=None):
    sizes, keys, off = make_sets(sizes)
    nsets = sizes.numel()
    if planned:
        b = M.Batch.plan(off.cuda(), gamma, seed, max_levels=max_levels, launch=launch).rebuild(keys.cuda()).status()
    else:
        b = M.build_batch(keys.cuda(), off.cuda(), gamma, seed, max_levels=max_levels, launch=launch)
    set_ids = torch.repeat_interleave(torch.arange(nsets), sizes)
    lab = host(b.lookup(set_ids.cuda(), keys.cuda()))
    knp = keys.numpy().view(np.uint64)
    offn = off.numpy()
    sets = range(nsets) if check is None else check
    for s in sets:
        ks = knp[offn[s]:offn[s + 1]]
        st = check_set(b, s, ks, gamma, seed, max_levels, lab[offn[s]:offn[s + 1]],
                       sectors=(s % 7 == 0) or len(ks) < 3000)
        if absent and len(ks):
            q = I.splitmix64(1000 + s, 300).numpy().view(np.uint64)
            got = host(b.lookup(torch.full((300,), s, dtype=torch.int64).cuda(),
                                torch.from_numpy(q.view(np.int64)).cuda()))
            assert np.array_equal(got, O.lookup(st, q)), s
    # every set's labels are a bijection onto [1, n_s]
    g = off[set_ids].numpy() + lab.astype(np.int64) - 1
    assert np.all(lab >= 1)
    assert np.array_equal(np.sort(g), np.arange(int(off[-1])))
    return b, keys, off


def test_batch_small_mixed_sizes(M):
    sizes = [0, 1, 2, 3, 16, 63, 64, 65, 100, 511, 512, 513, 1000, 4097, 20000, 0, 7, 65536]
    check_batch(M, sizes, 2.0)


@pytest.mark.parametrize("gamma", [1.0, 1.5, 2.0, 3.7])
def test_batch_log_uniform(M, gamma):
    sizes = I.log_uniform_sizes(400, 16, 8192, seed=30 + int(gamma * 10))
    check_batch(M, sizes, gamma, seed=0x1234)


def test_batch_more_sets_than_workgroups(M):
    # far more sets than the persistent grid: the work queue must hand every one out once
    sizes = I.log_uniform_sizes(6000, 1, 64, seed=5)
    check_batch(M, sizes, 2.0, seed=9, check=range(0, 6000, 37))


@pytest.mark.parametrize("max_levels", [1, 2, 3])
def test_batch_fallback_tables(M, max_levels):
    # few levels leave keys for every set's fallback table (sorted, labels n - |L| + 1 ..)
    sizes = [0, 1, 5, 50, 300, 1500, 2000, 999]
    check_batch(M, sizes, 2.0, seed=7, max_levels=max_levels)


def test_batch_largest_set_in_lds(M):
    # ceil(gamma n) = 2^19 exactly: A and C take 128 KiB of LDS
    check_batch(M, [1 << 18, 10, 1 << 17], 2.0, seed=11, absent=False)


@pytest.mark.parametrize("launch,planned", [
    ((128, 4, 0, 13, 2), False),    # levels of at most 512 keys in registers
    ((512, 16, 0, 1, 2), False),    # at most 8192 keys in registers; one queue
    ((256, 8, 2, 64, 1), True),     # every set small, every workgroup on the small queue; planned
])
def test_batch_largest_set_across_launches(M, launch, planned):
    """The largest set a batch takes streams its first levels from global memory and keeps its
    last ones in registers, at a threshold (threads x keys per thread) that depends on the launch;
    its levels, words, sectors and labels must equal the oracle's whichever launch and queue split
    builds it, beside sets that start in registers."""
    check_batch(M, [1 << 18, 10, 3000, 1 << 17, 700, 9000], 2.0, seed=12, absent=False, planned=planned,
                launch=launch)


def test_batch_equals_standalone_builds(M):
    sizes, keys, off = make_sets(I.log_uniform_sizes(64, 16, 65536, seed=12))
    b = M.build_batch(keys.cuda(), off.cuda(), 2.0, 77)
    for s in range(0, 64, 5):
        ks = keys[int(off[s]):int(off[s + 1])].cuda()
        h = M.build(ks, 2.0, 77)
        st = h.stats()
        info = b.set_info(s)
        assert info["level_n"] == st["level_n"][:st["num_levels"]]
        assert info["level_m"] == st["level_m"][:st["num_levels"]]
        ex, exb = h.export(), b.export_set(s)
        assert np.array_equal(ex["words"], exb["words"])
        assert np.array_equal(ex["fallback_keys"], exb["fallback_keys"])
        ids = torch.full((ks.numel(),), s, dtype=torch.int64, device="cuda")
        assert torch.equal(b.lookup(ids, ks), h.lookup(ks))
        h.close()


def test_batch_equal_keys_across_sets(M):
    # the same keys in two sets are two independent functions
    k = I.keys(3000, 21)
    keys = torch.cat([k, k[:1000], k])
    off = torch.tensor([0, 3000, 4000, 7000], dtype=torch.int64)
    b = M.build_batch(keys.cuda(), off.cuda(), 2.0, 3)
    e0, e2 = b.export_set(0), b.export_set(2)
    assert np.array_equal(e0["words"], e2["words"])
    ids = torch.repeat_interleave(torch.arange(3), torch.tensor([3000, 1000, 3000])).cuda()
    lab = host(b.lookup(ids, keys.cuda()))
    assert np.array_equal(lab[:3000], lab[4000:])
    st = O.build(k.numpy().view(np.uint64), 2.0, 3)
    assert np.array_equal(lab[:3000], O.lookup(st, k.numpy().view(np.uint64)))


def test_batch_set_id_out_of_range_gives_zero(M):
    sizes, keys, off = make_sets([100, 200])
    b = M.build_batch(keys.cuda(), off.cuda(), 2.0, 0)
    ids = torch.tensor([2, 5, -1], dtype=torch.int64).cuda()
    assert host(b.lookup(ids, keys[:3].cuda())).tolist() == [0, 0, 0]


def test_batch_duplicate_keys_rejected(M):
    k = I.keys(500, 5)
    keys = torch.cat([I.keys(100, 6), k, k[10:11]])
    off = torch.tensor([0, 100, 601], dtype=torch.int64)
    with pytest.raises(M.DuplicateKeysError):
        M.build_batch(keys.cuda(), off.cuda(), 2.0, 0)


def test_batch_rejects_bad_arguments(M):
    sizes, keys, off = make_sets([10, 20])
    with pytest.raises(M.MphfError):   # offsets not non-decreasing
        M.build_batch(keys.cuda(), torch.tensor([0, 20, 10], dtype=torch.int64).cuda(), 2.0, 0)
    with pytest.raises(M.MphfError):   # offsets[0] != 0
        M.build_batch(keys.cuda(), torch.tensor([1, 10, 30], dtype=torch.int64).cuda(), 2.0, 0)
    with pytest.raises(M.MphfError):   # gamma < 1
        M.build_batch(keys.cuda(), off.cuda(), 0.5, 0)
    big = I.keys((1 << 18) + 1, 8)
    with pytest.raises(M.MphfError):   # ceil(2 n) > 2^19
        M.build_batch(big.cuda(), torch.tensor([0, big.numel()], dtype=torch.int64).cuda(), 2.0, 0)
    many = I.keys(10000, 8)
    with pytest.raises(M.MphfError):   # one level leaves far more than 2048 keys
        M.build_batch(many.cuda(), torch.tensor([0, 10000], dtype=torch.int64).cuda(), 2.0, 0,
                      max_levels=1)
    with pytest.raises(ValueError):
        M.build_batch(keys.cuda(), off, 2.0, 0)   # host offsets


def test_batch_repeat_is_deterministic(M):
    sizes, keys, off = make_sets(I.log_uniform_sizes(300, 16, 4096, seed=13))
    kc, oc = keys.cuda(), off.cuda()
    b1 = M.build_batch(kc, oc, 2.0, 5)
    b2 = M.build_batch(kc, oc, 2.0, 5)
    for s in range(0, 300, 17):
        assert np.array_equal(b1.export_set(s)["words"], b2.export_set(s)["words"])
    ids = torch.repeat_interleave(torch.arange(300), sizes).cuda()
    assert torch.equal(b1.lookup(ids, kc), b2.lookup(ids, kc))


# ------------------------------------------------------------ planned batches and graph capture

@pytest.mark.parametrize("max_levels", [3, 25])
def test_planned_batch_equals_oracle(M, max_levels):
    sizes = [0, 1, 2, 17, 300, 4097, 20000, 5, 1200]
    check_batch(M, sizes, 2.0, seed=21, max_levels=max_levels, planned=True)


def test_planned_batch_rebuilds_with_new_keys(M):
    sizes = I.log_uniform_sizes(200, 16, 8192, seed=22)
    off = I.set_offsets(sizes)
    b = M.Batch.plan(off.cuda(), 2.0, 5)
    ids = torch.repeat_interleave(torch.arange(200), sizes).cuda()
    for seed in (31, 32, 33):
        keys = I.set_keys(sizes, seed)
        kc = keys.cuda()
        b.rebuild(kc).status()
        ref = M.build_batch(kc, off.cuda(), 2.0, 5)
        assert torch.equal(b.lookup(ids, kc), ref.lookup(ids, kc))
        for s in range(0, 200, 23):
            assert np.array_equal(b.export_set(s)["words"], ref.export_set(s)["words"])
            assert np.array_equal(b.export_sectors(s), ref.export_sectors(s))
        assert b.totals()["bits_per_key"] == ref.totals()["bits_per_key"]


def test_planned_batch_reports_duplicates_and_recovers(M):
    sizes = torch.tensor([100, 500], dtype=torch.int64)
    off = I.set_offsets(sizes)
    b = M.Batch.plan(off.cuda(), 2.0, 0)
    good = I.set_keys(sizes, 4)
    bad = good.clone()
    bad[150] = bad[120]
    with pytest.raises(M.DuplicateKeysError):
        b.rebuild(bad.cuda()).status()
    b.rebuild(good.cuda()).status()
    ids = torch.repeat_interleave(torch.arange(2), sizes).cuda()
    lab = host(b.lookup(ids, good.cuda()))
    st = O.build(good[100:].numpy().view(np.uint64), 2.0, 0)
    assert np.array_equal(lab[100:], O.lookup(st, good[100:].numpy().view(np.uint64)))


def test_rebuild_needs_a_plan(M):
    sizes, keys, off = make_sets([10, 20])
    b = M.build_batch(keys.cuda(), off.cuda(), 2.0, 0)
    with pytest.raises(M.MphfError):
        b.rebuild(keys.cuda())


def test_planned_batch_in_hip_graph(M):
    """Rebuild + lookup captured once in a graph and replayed on new keys: every replay must equal
    an eager one-shot build of the same keys."""
    sizes = I.log_uniform_sizes(300, 16, 16384, seed=40)
    off = I.set_offsets(sizes).cuda()
    ids = torch.repeat_interleave(torch.arange(300), sizes).cuda()
    keys_buf = I.set_keys(sizes, 41).cuda()
    out = torch.empty_like(keys_buf)
    b = M.Batch.plan(off, 2.0, 9)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up outside the capture
        b.rebuild(keys_buf).lookup(ids, keys_buf, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.rebuild(keys_buf)
        b.lookup(ids, keys_buf, out=out)
    for seed in (42, 43, 44, 42):
        keys_buf.copy_(I.set_keys(sizes, seed).cuda())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        b.status()
        ref = M.build_batch(keys_buf, off, 2.0, 9)
        assert torch.equal(out, ref.lookup(ids, keys_buf)), seed
        for s in range(0, 300, 37):
            assert np.array_equal(b.export_sectors(s), ref.export_sectors(s)), (seed, s)
        ref.close()


# ------------------------------------------------------------ launch configurations and the tuner

def test_every_launch_configuration_gives_the_same_batch(M):
    from paper_1702_03154_amd import autotune
    sizes, keys, off = make_sets(I.log_uniform_sizes(150, 1, 20000, seed=50))
    kc, oc = keys.cuda(), off.cuda()
    ids = torch.repeat_interleave(torch.arange(150), sizes).cuda()
    ref = M.build_batch(kc, oc, 2.0, 3)
    want = ref.lookup(ids, kc)
    secs = {s: ref.export_sectors(s) for s in range(0, 150, 11)}
    for launch in autotune.candidates():
        b = M.build_batch(kc, oc, 2.0, 3, launch=launch)
        assert torch.equal(b.lookup(ids, kc), want), launch
        for s, v in secs.items():
            assert np.array_equal(b.export_sectors(s), v), (launch, s)
        b.close()
    with pytest.raises(M.MphfError):
        M.build_batch(kc, oc, 2.0, 3, launch=(300, 8, 0))


@pytest.mark.parametrize("launch", [
    (256, 4, 0, 1, 1),       # no small sets: one queue, largest first
    (256, 4, 0, 64, 1),      # every set small, every workgroup on the small queue
    (256, 8, 0, 13, 1),      # every workgroup takes small sets first
    (128, 16, 2, 5, 3),      # small = below 16 keys
    (512, 4, 4, 17, 1000),   # one workgroup in 1000 takes small sets first
])
def test_work_queue_split_gives_the_same_batch(M, launch):
    """The two work queues (large sets first for most workgroups, small sets first for every k-th)
    only change which workgroup builds which set and when: every label and sector must equal the
    default build's, whatever the class threshold and share, including the degenerate splits."""
    sizes, keys, off = make_sets(I.log_uniform_sizes(400, 1, 30000, seed=52))
    kc, oc = keys.cuda(), off.cuda()
    ids = torch.repeat_interleave(torch.arange(400), sizes).cuda()
    ref = M.build_batch(kc, oc, 2.0, 5)
    b = M.build_batch(kc, oc, 2.0, 5, launch=launch)
    assert torch.equal(b.lookup(ids, kc), ref.lookup(ids, kc)), launch
    for s in range(0, 400, 13):
        assert np.array_equal(b.export_sectors(s), ref.export_sectors(s)), (launch, s)
    plan = M.Batch.plan(oc, 2.0, 5, launch=launch)
    plan.rebuild(kc).status()
    assert torch.equal(plan.lookup(ids, kc), ref.lookup(ids, kc)), launch
    for s in (0, 1, 2, 3, 399):
        assert np.array_equal(plan.export_sectors(s), ref.export_sectors(s)), (launch, s)
    for x in (b, plan, ref):
        x.close()
    with pytest.raises(M.MphfError):
        M.build_batch(kc, oc, 2.0, 5, launch=(256, 4, 0, 65, 2))


def test_tuner_picks_a_candidate_and_caches_it(M, tmp_path, monkeypatch):
    from paper_1702_03154_amd import autotune
    monkeypatch.setenv("MPHF_TUNE_CACHE", str(tmp_path / "tune.json"))
    sizes = I.log_uniform_sizes(500, 16, 4096, seed=51)
    off = I.set_offsets(sizes).cuda()
    launch = autotune.batch_launch(off, 2.0)
    assert launch in set(autotune.candidates())
    rec = autotune._load()[autotune.device_key()][autotune.workload_key(off, 2.0, 25)]
    assert tuple(rec["launch"]) == launch and rec["ms"] <= rec["default_ms"]
    assert autotune.batch_launch(off, 2.0) == launch   # from the cache
    keys = I.set_keys(sizes, 4).cuda()
    ids = torch.repeat_interleave(torch.arange(500), sizes).cuda()
    b = M.build_batch(keys, off, 2.0, 0, launch=launch)
    ref = M.build_batch(keys, off, 2.0, 0)
    assert torch.equal(b.lookup(ids, keys), ref.lookup(ids, keys))


def test_batch_set_outgrowing_its_expected_region(M):
    """Keys crafted so that every key collides at level 0 (pairs with equal level-0 positions): the
    set's levels then total about 2.65 m0 bits, more than the 1.5 e^(1/gamma) m0 the one-shot build
    reserves first, so the batch is redone with worst-case regions; the result must not change."""
    U64 = (1 << 64) - 1
    inv1 = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    inv2 = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)

    def unfmix64(y):
        z = y ^ (y >> 33)
        z = (z * inv2) & U64
        z ^= z >> 33
        z = (z * inv1) & U64
        return z ^ (z >> 33)

    n = 50_000
    m0 = 2 * n
    s0 = O.level_seeds(0, 1)[0]
    rng = np.random.default_rng(60)
    crafted = []
    for h in rng.integers(0, 1 << 62, size=n // 2, dtype=np.uint64).tolist():
        crafted += [unfmix64(h) ^ s0, unfmix64(h + m0) ^ s0]
    crafted = np.array(crafted, dtype=np.uint64)
    assert len(np.unique(crafted)) == n
    assert len(np.unique(O.level_positions(crafted, s0, m0))) <= n // 2
    other = I.keys(3000, 61).numpy().view(np.uint64)
    keys = np.concatenate([other[:1000], crafted, other[1000:]])
    off = torch.tensor([0, 1000, 1000 + n, 3000 + n], dtype=torch.int64)
    b = M.build_batch(torch.from_numpy(keys.view(np.int64)).cuda(), off.cuda(), 2.0, 0)
    ids = torch.repeat_interleave(torch.arange(3), off[1:] - off[:-1]).cuda()
    lab = host(b.lookup(ids, torch.from_numpy(keys.view(np.int64)).cuda()))
    offn = off.numpy()
    for s in range(3):
        ks = keys[offn[s]:offn[s + 1]]
        st = check_set(b, s, ks, 2.0, 0, 25, lab[offn[s]:offn[s + 1]])
        if s == 1:
            assert st.levels[1].n == n   # nothing placed at level 0
            assert st.total_bits > 1.5 * math.exp(0.5) * m0 + 64 * 25


def test_batch_full_config_65536_sets(M):
    """The benchmark's batch at full size (65,536 sets, log-uniform in [16, 65536], about 5.1e8
    keys): every set's labels are a bijection onto [1, n_s], and sampled sets, the largest among
    them, equal the oracle."""
    sizes = I.log_uniform_sizes(65536, 16, 65536, seed=3)
    off = I.set_offsets(sizes)
    keys = I.set_keys(sizes, seed=4, device="cuda")
    offc = off.cuda()
    b = M.build_batch(keys, offc, 2.0, 0)
    ids = torch.repeat_interleave(torch.arange(65536, device="cuda"), sizes.cuda())
    lab = b.lookup(ids, keys)
    g = offc[ids] + lab - 1
    assert bool((lab >= 1).all()) and bool((g < offc[ids + 1]).all())
    seen = torch.zeros(keys.numel(), dtype=torch.int8, device="cuda")
    seen[g] = 1
    assert bool(seen.all())
    big = int(torch.argmax(sizes))
    for s in sorted({0, 1, 777, 4095, 32768, 65535, big}):
        a, c = int(off[s]), int(off[s + 1])
        ks = keys[a:c].cpu().numpy().view(np.uint64)
        st = O.build(ks, 2.0, 0)
        assert np.array_equal(b.export_set(s)["words"], st.words), s
        assert np.array_equal(host(lab[a:c]), O.lookup(st, ks)), s
    t = b.totals()
    assert t["nsets"] == 65536 and t["nkeys"] == keys.numel()
    assert abs(t["bits_per_key"] - 3.6) < 0.1
