"""Shared parity check of the GPU tests: one build through the C ABI compared element by element
with the oracle built on the same keys (level sizes, offsets and seeds, every word of A and of every
C_d, the rank table, the fallback keys, bits/key, and the labels of the keys and of extra queries)."""
import numpy as np
import torch

from oracle import mphf_oracle as O
from paper_1702_03154_amd import inputs as I


def host(t):
    return t.cpu().numpy().view(np.uint64)


def check_against_oracle(M, keys_np, gamma, seed=0, max_levels=25, rank_sample=512,
                         queries_np=None, bucket_bits=0, paths=None):
    """Build on the GPU and with the oracle and compare everything; ``paths`` (if given) is called
    with the list of level paths the GPU build took (checks of which kernels ran)."""
    keys = torch.from_numpy(keys_np.view(np.int64)).cuda()
    h = M.build(keys, gamma, seed, max_levels=max_levels, rank_sample=rank_sample,
                keep_collisions=True, bucket_bits=bucket_bits)
    st = O.build(keys_np, gamma, seed, max_levels=max_levels, rank_sample=rank_sample)
    s = h.stats()
    assert s["num_levels"] == st.num_levels
    assert s["level_n"] == [l.n for l in st.levels]
    assert s["level_m"] == [l.m for l in st.levels]
    assert s["level_weight"] == [l.weight for l in st.levels]
    assert s["level_offset"] == [l.offset for l in st.levels]
    assert s["level_seed"] == [l.seed for l in st.levels]
    assert s["total_bits"] == st.total_bits
    assert s["n_fallback"] == len(st.fallback_keys)
    ex = h.export()
    assert np.array_equal(ex["words"], st.words)
    assert np.array_equal(ex["rank"], st.rank)
    assert np.array_equal(ex["fallback_keys"], st.fallback_keys)
    for d in range(st.num_levels):
        assert np.array_equal(h.export_collisions(d), O.collision_words(st, d)), d
    lab = host(h.lookup(keys))
    want = O.lookup(st, keys_np)
    assert np.array_equal(lab, want)
    if queries_np is not None:
        q = torch.from_numpy(queries_np.view(np.int64)).cuda()
        assert np.array_equal(host(h.lookup(q)), O.lookup(st, queries_np))
    assert abs(s["bits_per_key"] - st.bits_per_key) < 1e-9
    if paths is not None:
        paths(s["level_path"])
    h.close()
    return st


def keys_np(n, seed=1):
    return I.keys(n, seed).numpy().view(np.uint64)
