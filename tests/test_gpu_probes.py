"""GPU tests of the roofline microbenchmarks (mphf_probe): every kind runs on small buffers and
reports the number of random operations it made; the host exchange copies pinned host memory
through a kernel (each word plus one); wrong buffers and sizes are rejected."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_03154_amd import mphf
    mphf.lib()
    return mphf


def test_device_probes_run(M):
    buf = torch.zeros(1 << 16, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(buf)
    nbytes = buf.numel() * 8
    assert M.probe("stream_read", buf, nbytes) == 0
    buf.fill_(7)
    assert M.probe("stream_copy", buf, nbytes, dst) == 0
    torch.cuda.synchronize()
    assert torch.equal(dst, buf)
    for kind in ("random_read8", "random_sector64", "random_atomic_or"):
        done = M.probe(kind, buf, nbytes, ops=1 << 20)
        assert done == M.lib().mphf_probe_ops(1 << 20) >= 1 << 20, kind
    assert M.probe("lds_atomic_or", None, 8192, ops=1 << 20) >= 1 << 20
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 1000, 1 << 20])
def test_host_exchange_copies_pinned_memory(M, n):
    src, dst = M.HostArray(n), M.HostArray(n)
    src.a[:] = np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    dst.a[:] = 0
    M.probe_host_exchange(src, dst, 8 * n)
    torch.cuda.synchronize()
    assert np.array_equal(dst.a, src.a + np.uint64(1))
    src.close()
    dst.close()


def test_probe_arguments_rejected(M):
    src, dst = M.HostArray(16), M.HostArray(16)
    dev = torch.zeros(16, dtype=torch.int64, device="cuda")
    lib = M.lib()
    k = M.PROBE_KINDS["host_exchange"]
    assert lib.mphf_probe(k, src._p.value, 12, dst._p.value, 0, 0, None) == M.E_INVALID   # not 8-byte words
    assert lib.mphf_probe(k, dev.data_ptr(), 128, dst._p.value, 0, 0, None) == M.E_INVALID   # device memory
    assert lib.mphf_probe(M.PROBE_KINDS["stream_read"], src._p.value, 128, 0, 0, 0, None) == M.E_INVALID
    assert lib.mphf_probe(99, dev.data_ptr(), 128, 0, 0, 0, None) == M.E_INVALID
    assert lib.mphf_probe(M.PROBE_KINDS["lds_atomic_or"], 0, 1 << 20, 0, 1, 0, None) == M.E_INVALID
    torch.cuda.synchronize()
    src.close()
    dst.close()
    with pytest.raises(ValueError):
        M.probe_host_exchange(M.HostArray(4), M.HostArray(8), 64)   # more than the arrays hold
