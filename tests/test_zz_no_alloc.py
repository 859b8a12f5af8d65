"""The allocation-free hash-set partition (mphf_partition_sets_noalloc) against mphf_partition_sets,
through the C ABI, on two calls in a row (the second smaller, so it runs over the first's scratch
contents), and both against the set of each key computed on the host from the oracle's fmix64."""
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


def per_set_sorted(keys, counts):
    seg = np.repeat(np.arange(len(counts)), counts)
    return keys[np.lexsort((keys, seg))]


def test_noalloc_partition_equals_partition_sets_twice(M):
    seed = 0x0DDB_A115_5EED_0001
    for n, bits in ((400_000, 14), (70_001, 9)):     # the second call smaller, over the first's scratch
        keys = I.keys(n, 60 + bits).cuda()
        out_a, off_a = M.partition_sets(keys, bits, seed=seed)
        out_b = torch.full_like(keys, -1)
        off_b = torch.full(((1 << bits) + 1,), -1, dtype=torch.int64, device=keys.device)
        M.partition_sets_noalloc(keys, bits, seed=seed, out=out_b, offsets=off_b)
        torch.cuda.synchronize()
        assert torch.equal(off_a, off_b), (n, bits)
        k = host(keys)
        sid = (O.fmix64(k ^ np.uint64(seed)) >> np.uint64(64 - bits)).astype(np.int64)
        counts = np.bincount(sid, minlength=1 << bits)
        assert np.array_equal(np.diff(off_b.cpu().numpy()), counts)
        want = per_set_sorted(k[np.argsort(sid, kind="stable")], counts)
        assert np.array_equal(per_set_sorted(host(out_a), counts), want)
        assert np.array_equal(per_set_sorted(host(out_b), counts), want)


def test_noalloc_partition_limits(M):
    keys = I.keys(1000, 3).cuda()
    with pytest.raises(M.MphfError) as e:
        M.partition_sets_noalloc(keys, 17)
    assert e.value.status == M.E_INVALID and "16" in str(e.value)
    out, off = M.partition_sets_noalloc(torch.zeros(0, dtype=torch.int64, device="cuda"), 16)
    torch.cuda.synchronize()
    assert int(off.abs().sum()) == 0
