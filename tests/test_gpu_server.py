"""GPU tests of the serving loop: resident functions, requests admitted by HBM budget and batched as
they arrive.  A request's labels must be exactly those of a plain lookup on its function and of the
oracle built on that function's keys, whether it runs alone or in a mix with other requests."""
import threading

import numpy as np
import pytest
import torch

from oracle import mphf_oracle as O
from paper_1702_03154_amd import inputs as I

pytestmark = pytest.mark.gpu

SIZES = [1000, 7, 50_000, 300_000, 2_000_000, 123_457]


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_03154_amd import mphf
    mphf.lib()
    return mphf


@pytest.fixture(scope="module")
def fns(M):
    """Resident functions: (handle, host keys) per size; key stream seed 100 + index."""
    out = []
    for j, n in enumerate(SIZES):
        k = I.keys(n, 100 + j)
        out.append((M.build(k.cuda(), 2.0, 0), k.numpy().view(np.uint64)))
    return out


@pytest.fixture(scope="module")
def oracles(fns):
    """The oracle's build of every resident function (2.5e6 keys in all)."""
    return [O.build(keys, 2.0, 0) for _, keys in fns]


def make_requests(fns, count, seed, max_n=40_000):
    """(function, query array) pairs: sizes log-uniform in [1, max_n], 90% present keys, 10% absent."""
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        f = int(rng.integers(len(fns)))
        n = int(np.floor(max_n ** rng.random())) if rng.random() < 0.97 else 0
        keys = fns[f][1]
        q = keys[rng.integers(0, len(keys), size=n)]
        absent = rng.random(n) < 0.1
        q[absent] = I.splitmix64(900 + seed, int(absent.sum())).numpy().view(np.uint64)
        reqs.append((f, np.ascontiguousarray(q)))
    return reqs


def plain_labels(M, fns, f, q):
    if len(q) == 0:
        return np.zeros(0, dtype=np.uint64)
    t = torch.from_numpy(q.view(np.int64)).cuda()
    return fns[f][0].lookup(t).cpu().numpy().view(np.uint64)


def run(server, ids, reqs, pinned=None):
    outs, tickets = [], []
    for i, (f, q) in enumerate(reqs):
        out = np.zeros(len(q), dtype=np.uint64) if pinned is None else pinned[i]
        outs.append(out)
        tickets.append(server.submit(ids[f], q, out))
    infos = [server.poll(t, wait=True) for t in tickets]
    return outs, infos


def test_results_alone_and_in_the_mix(M, fns, oracles):
    """Every request's labels, served alone and in a mix of 240, equal a plain lookup on its function
    and the oracle's labels (members and the 10% non-members) for every function, up to 2e6 keys."""
    reqs = make_requests(fns, 240, seed=1)
    s = M.Server(hbm_budget=256 << 20, max_inflight=2)
    ids = [s.register(h) for h, _ in fns]
    alone = []
    for f, q in reqs[:40]:   # one at a time
        out = np.zeros(len(q), dtype=np.uint64)
        s.poll(s.submit(ids[f], q, out), wait=True)
        alone.append(out)
    mixed, infos = run(s, ids, reqs)   # everything at once
    for i, (f, q) in enumerate(reqs):
        want = plain_labels(M, fns, f, q)
        assert np.array_equal(mixed[i], want), i
        assert np.array_equal(mixed[i], O.lookup(oracles[f], q)), i
        if i < 40:
            assert np.array_equal(alone[i], want), i
    # continuous batching: requests shared batches, and batches overlapped on the device
    assert max(x["batch_requests"] for x in infos) > 1
    st = s.stats()
    assert st["requests"] == 280 and st["batches"] < 280
    s.close()


def test_small_functions_against_the_oracle(M, fns):
    s = M.Server(hbm_budget=64 << 20)
    ids = [s.register(h) for h, _ in fns]
    for f in (0, 1):
        keys = fns[f][1]
        st = O.build(keys, 2.0, 0)
        q = np.concatenate([keys, I.splitmix64(77, 500).numpy().view(np.uint64)])
        out = np.zeros(len(q), dtype=np.uint64)
        s.poll(s.submit(ids[f], q, out), wait=True)
        assert np.array_equal(out, O.lookup(st, q))
    s.close()


def test_admission_by_budget(M, fns):
    # 1 MiB budget over 2 batches: about 32k keys per batch, so large requests queue for memory
    s = M.Server(hbm_budget=1 << 20, max_inflight=2, max_batch_requests=64)
    ids = [s.register(h) for h, _ in fns]
    reqs = make_requests(fns, 150, seed=2, max_n=30_000)
    outs, infos = run(s, ids, reqs)
    for i, (f, q) in enumerate(reqs):
        assert np.array_equal(outs[i], plain_labels(M, fns, f, q)), i
    st = s.stats()
    assert st["peak_bytes_in_flight"] <= 1 << 20
    assert st["max_batch_requests_seen"] <= 64
    with pytest.raises(M.MphfError):
        s.submit(ids[4], fns[4][1][:100_000].copy(), np.zeros(100_000, dtype=np.uint64))
    s.close()


def test_concurrent_submitters_with_pinned_arrays(M, fns):
    s = M.Server(hbm_budget=512 << 20, max_inflight=3)
    ids = [s.register(h) for h, _ in fns]
    errors = []

    def client(seed):
        try:
            reqs = make_requests(fns, 60, seed=seed)
            pin_q = [M.HostArray(len(q)) for _, q in reqs]
            pin_o = [M.HostArray(len(q)) for _, q in reqs]
            for p, (_, q) in zip(pin_q, reqs):
                p.a[:] = q
            tickets = [s.submit(ids[f], p.a, o.a) for (f, _), p, o in zip(reqs, pin_q, pin_o)]
            for t in tickets:
                s.poll(t, wait=True)
            for (f, q), o in zip(reqs, pin_o):
                if not np.array_equal(o.a, plain_labels(M, fns, f, q)):
                    errors.append(seed)
            for p in pin_q + pin_o:
                p.close()
        except Exception as e:   # reported below
            errors.append(repr(e))

    ts = [threading.Thread(target=client, args=(10 + i,)) for i in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
    assert s.stats()["requests"] == 240
    s.close()


def test_overlap_and_arrival_order(M, fns):
    s = M.Server(hbm_budget=64 << 20, max_inflight=2, max_batch_requests=8)
    ids = [s.register(h) for h, _ in fns]
    reqs = make_requests(fns, 120, seed=3, max_n=200_000)
    _, infos = run(s, ids, reqs)
    nonempty = [x for x in infos if x["batch_requests"] > 0]
    batches = sorted({(x["batch"], x["start_us"], x["done_us"]) for x in nonempty})
    # batches are admitted in arrival order, and a later batch starts before an earlier one ends
    assert all(a[1] <= b[1] for a, b in zip(batches, batches[1:]))
    assert any(b[1] < a[2] for a, b in zip(batches, batches[1:]))
    order = [x["batch"] for x in nonempty]
    assert order == sorted(order)
    s.close()


def test_server_rejects_bad_requests(M, fns):
    s = M.Server(hbm_budget=16 << 20)
    i = s.register(fns[0][0])
    with pytest.raises(M.MphfError):
        s.submit(i + 5, np.zeros(4, dtype=np.uint64), np.zeros(4, dtype=np.uint64))
    t = s.submit(i, np.zeros(0, dtype=np.uint64), np.zeros(0, dtype=np.uint64))
    assert s.poll(t, wait=False)["done"]
    with pytest.raises(M.MphfError):
        s.poll(t, wait=False)   # a done request is forgotten once reported
    with pytest.raises(M.MphfError):
        M.Server(hbm_budget=1000)
    s.close()


def test_pinned_and_pageable_requests_in_one_batch(M, fns):
    """Pinned arrays are labelled in place over PCIe, pageable ones through the batch's device
    buffers; both kinds share batches and give the plain labels."""
    s = M.Server(hbm_budget=128 << 20, max_inflight=2)
    ids = [s.register(h) for h, _ in fns]
    reqs = make_requests(fns, 80, seed=7)
    pinned, outs, tickets = [], [], []
    for i, (f, q) in enumerate(reqs):
        if i % 2:
            pq, po = M.HostArray(len(q)), M.HostArray(len(q))
            pq.a[:] = q
            pinned += [pq, po]
            qa, oa = pq.a, po.a
        else:
            qa, oa = q, np.zeros(len(q), dtype=np.uint64)
        outs.append(oa)
        tickets.append(s.submit(ids[f], qa, oa))
    infos = [s.poll(t, wait=True) for t in tickets]
    assert max(x["batch_requests"] for x in infos) > 1
    for (f, q), o in zip(reqs, outs):
        assert np.array_equal(o, plain_labels(M, fns, f, q))
    for p in pinned:
        p.close()
    s.close()
