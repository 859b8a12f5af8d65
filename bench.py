"""Benchmark of the cascading-bit-array MPHF hot path on one MI355X.

Default workload (plain): one step = one build (every level, the fallback table
and the rank table) of N distinct 64-bit keys already resident in HBM, followed
by the lookup of all N keys in a seeded shuffled order.  The JSON line also
carries, each measured in the same run:

* roofline: the lookup (the dominant kernel) against HBM on its algorithmic
  bytes (16 per query), its random probes against the measured random-sector
  rate at the structure's footprint, and the lower bound T_lb over the measured
  time; build_roofline the same for the build;
* gamma1: the same build and lookup at gamma = 1;
* batched: 65,536 independent sets (log-uniform sizes in [16, 65536]) built in
  one launch and looked up, beside a loop of plain per-set builds and lookups;
* served: 64 resident functions answering Poisson-arriving requests from host
  memory through the serving loop, beside plain per-request lookups, with p50/p99
  latency at fractions of the served and of the plain capacity;
* cpu_baseline: the oracle (numpy, one core) on a sample, and the threaded CPU
  build and lookup in the paper's style on every host core on the whole workload.

--workload batch / serve: those parts alone (batch with the optional --tune).

--workload kmer: the first 4e9 distinct canonical 31-mers of a 4.2e9-base random
DNA sequence (32 GB of keys in HBM); plain build + lookup and the batched path
over 2^15 hash sets, with per-level sizes checked against the occupancy
statistics.

--workload stream: the streaming build over 1e10 keys generated on the fly (never
stored), levels re-scanning the stream while more than 2^31 keys survive; then the
lookup of every key, regenerated chunk by chunk.

--workload gamma: the plain build + lookup for gamma in 1..10 and with 1024-bit rank
sampling, beside the space analysis (bits/key, probes per query).

--workload roofline: the memory-system microbenchmarks (streaming read and copy,
random 8-byte and 64-byte-sector reads, random global and LDS atomicOr with
return) over footprints from LDS to 5 GB.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
LINE_BYTES = 128               # a random read on gfx950 moves one 128-byte line from HBM (measured)
LOOKUP_BYTES_PER_QUERY = 16.0  # the lookup's algorithmic bytes: the key read, the label written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_lookup_traffic.json")
BUILD_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "build_1e9_gamma2_traffic.json")
METRIC = "build keys/s + lookup queries/s (1e9 u64, gamma=2); batched/served vs plain"


def log(msg: str):
    print(f"# {msg}", file=sys.stderr, flush=True)


def mean_probes(st) -> float:
    """Levels a member query visits on average: a key placed at level d probes d+1 levels; a
    fallback key probes all of them (Algorithm 3)."""
    n = st["n"]
    if not n:
        return 0.0
    tot = sum((d + 1) * w for d, w in enumerate(st["level_weight"]))
    tot += st["n_fallback"] * st["num_levels"]
    return tot / n


def measured_traffic(n_queries: int):
    """HBM bytes of one k_lookup launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source and the same workload; else None."""
    from paper_1702_03154_amd.profsum import source_digest
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        sha = source_digest()
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != sha or t.get("queries") != n_queries:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def measured_build_traffic(n_keys: int):
    """HBM bytes of one plain build from the committed counter summary, if it was taken on the
    current build sources and the same key count; else None."""
    from paper_1702_03154_amd.profsum import BUILD_SOURCES, source_digest
    try:
        with open(BUILD_TRAFFIC_FILE) as f:
            t = json.load(f)
        sha = source_digest(BUILD_SOURCES)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != sha or t.get("keys") != n_keys:
        return None
    return t["bytes_per_build"]


def build_algorithmic_bytes(st) -> float:
    """Bytes the method itself moves in one build (the fused model of one pass per level): every
    key of F_d read once, every survivor written once, the concatenated A and the rank table
    written once (Sections 2.1, 2.2 and 3.1)."""
    nd = st["level_n"][:st["num_levels"]]
    survivors = sum(nd[1:]) + st["n_fallback"]
    return 8.0 * sum(nd) + 8.0 * survivors + st["total_bits"] / 8.0 + 8.0 * st["rank_entries"]


def build_random_ops(st) -> int:
    """The method's random accesses in one build: every key of every level is one test-and-set of
    its position (Algorithm 2) and one read of its bit by the filter (Algorithm 1)."""
    return 2 * sum(st["level_n"][:st["num_levels"]])


# ---------------------------------------------------------------- host description and CPU baselines

def host_info() -> dict:
    info = {"nproc": os.cpu_count()}
    try:
        info["usable_cpus"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            models = [l.split(":", 1)[1].strip() for l in f if l.startswith("model name")]
        if models:
            info["cpu_model"] = models[0]
            info["logical_cpus_listed"] = len(models)
    except OSError:
        pass
    try:
        with open("/proc/meminfo") as f:
            for l in f:
                if l.startswith("MemTotal"):
                    info["mem_total_gib"] = round(int(l.split()[1]) / 2**20, 1)
    except OSError:
        pass
    return info


def cpu_baseline(n: int, gamma: float):
    """The oracle as it stands, on a bounded sample of the same workload, one host core."""
    import numpy as np

    from oracle import mphf_oracle as O
    from paper_1702_03154_amd import inputs

    k = inputs.keys(n, seed=1).numpy().view(np.uint64)
    q = inputs.shuffled_queries(inputs.keys(n, seed=1), seed=2).numpy().view(np.uint64)
    t0 = time.perf_counter()
    st = O.build(k, gamma, 0)
    t1 = time.perf_counter()
    lab = O.lookup(st, q)
    t2 = time.perf_counter()
    assert int(lab.max()) == n
    return {"value": n / (t2 - t0), "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} keys, gamma={gamma}: build + lookup of all keys (shuffled)",
            "build_keys_per_s": n / (t1 - t0), "lookup_queries_per_s": n / (t2 - t1)}


def threaded_baseline(keys_host, queries_host, gamma: float):
    """The paper-style parallel CPU build (keys split over threads, atomic fetch-or on the shared
    bit arrays) and lookup on every usable host core, on the whole workload."""
    import numpy as np

    from oracle import threaded as T

    n = len(keys_host)
    t0 = time.perf_counter()
    f = T.Threaded(keys_host, gamma, 0)
    t1 = time.perf_counter()
    lab = f.lookup(queries_host)
    t2 = time.perf_counter()
    levels = f.sizes()[0]
    f.close()
    ok = int(lab.min()) == 1 and int(lab.max()) == n
    del lab
    return {"value": n / (t2 - t0), "unit": "keys/s", "cores": f.threads, "kind": "threaded",
            "sample": f"the whole workload: {n} keys, gamma={gamma}, build + shuffled lookup of all keys",
            "build_keys_per_s": n / (t1 - t0), "lookup_queries_per_s": n / (t2 - t1),
            "build_s": t1 - t0, "lookup_s": t2 - t1, "levels": levels, "labels_in_range": ok,
            "what": "std::thread over key chunks, __atomic_fetch_or on shared A_d and C_d (Section 3.2)"}


def calibrate_copy():
    """One plain 1 GiB device-to-device copy: a kernel of known traffic for scaling HBM counters."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


# ---------------------------------------------------------------- roofline probes

def probe_rate(kind: str, nbytes: int, ops: int = 0, reps: int = 5) -> dict:
    """Rate of one microbenchmark (bytes/s for the streaming kinds, operations/s for the random
    ones), timed with events on the stream it is launched on: the best of `reps` runs after one
    warm-up, since it stands for a ceiling (repeated runs of the random kinds spread by a few
    percent from box to box and within a process)."""
    import torch

    from paper_1702_03154_amd import mphf

    dev = torch.device("cuda:0")
    buf = dst = None
    if kind != "lds_atomic_or":
        buf = torch.zeros((nbytes + 63) // 8 + 8, dtype=torch.int64, device=dev)
        if kind == "stream_copy":
            dst = torch.empty_like(buf)
    s = torch.cuda.current_stream()
    times, done = [], 0
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        done = mphf.probe(kind, buf, nbytes, dst, ops, seed=r + 1)
        e1.record(s)
        torch.cuda.synchronize()
        if r:
            times.append(e0.elapsed_time(e1) / 1e3)
    t = min(times)
    del buf, dst
    if kind in ("stream_read", "stream_copy"):
        moved = nbytes * (2 if kind == "stream_copy" else 1)
        return {"kind": kind, "footprint_bytes": nbytes, "bytes_per_s": moved / t, "ms": t * 1e3}
    return {"kind": kind, "footprint_bytes": nbytes, "ops": done, "ops_per_s": done / t, "ms": t * 1e3}


def pcie_rate(nbytes: int = 1 << 30, reps: int = 3) -> dict:
    """The PCIe ceiling of a lookup fed from host memory: a kernel reading nbytes of pinned host
    memory and writing them to pinned host memory (mphf_probe, host exchange), bytes moved per
    second counting both directions."""
    import statistics

    import torch

    from paper_1702_03154_amd import mphf

    src, dst = mphf.HostArray(nbytes // 8), mphf.HostArray(nbytes // 8)
    src.a[:] = 1
    s = torch.cuda.current_stream()
    times = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        mphf.probe_host_exchange(src, dst, nbytes)
        e1.record(s)
        torch.cuda.synchronize()
        if r:
            times.append(e0.elapsed_time(e1) / 1e3)
    ok = bool(dst.a[0] == 2 and dst.a[-1] == 2)
    src.close(), dst.close()
    t = statistics.median(times)
    return {"kind": "host_exchange", "footprint_bytes": nbytes, "bytes_per_s": 2 * nbytes / t, "ms": t * 1e3,
            "checked": ok}


def bench_roofline(args):
    """The microbenchmark sweep: each random kind over LDS / L2 / MALL / HBM footprints."""
    foot = [("L2 (4 MiB)", 4 << 20), ("MALL (256 MiB)", 256 << 20), ("HBM (5 GiB)", 5 << 30)]
    rows = [probe_rate("stream_read", 8 << 30), probe_rate("stream_copy", 4 << 30)]
    for kind in ("random_read8", "random_sector64", "random_atomic_or"):
        for name, b in foot:
            r = probe_rate(kind, b, ops=1 << 29)
            r["footprint"] = name
            rows.append(r)
            log(f"{kind} over {name}: {r['ops_per_s']:.3e} ops/s")
    for b in (8192, 49152):
        r = probe_rate("lds_atomic_or", b, ops=1 << 32)
        r["footprint"] = f"LDS ({b // 1024} KiB per workgroup)"
        rows.append(r)
    r = pcie_rate()
    r["footprint"] = "pinned host memory over PCIe (1 GiB each way)"
    rows.append(r)
    log(f"host exchange over PCIe: {r['bytes_per_s'] / 1e9:.1f} GB/s (both directions)")
    res = {"metric": METRIC, "value": rows[1]["bytes_per_s"], "unit": "bytes/s",
           "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": rows[1]["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "memory-system microbenchmarks: streaming read and copy, random 8-byte and "
                                  "64-byte-sector reads, random atomicOr with return (global and LDS), "
                                  "a kernel exchanging pinned host memory over PCIe"},
           "rows": rows}
    print(json.dumps(res))


# ---------------------------------------------------------------- batched builds

def run_batch(args, steps: int, warmup: int, graph: bool = True) -> dict:
    """Batched build + lookup of many independent sets against a loop of plain per-set calls."""
    import statistics

    import torch

    from paper_1702_03154_amd import inputs, mphf

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nsets = int(args.sets)
    sizes = inputs.log_uniform_sizes(nsets, 16, 65536, seed=3)
    off_h = inputs.set_offsets(sizes)
    total = int(off_h[-1])
    keys = inputs.set_keys(sizes, seed=4, device=dev)
    off = off_h.to(dev)
    set_ids = torch.repeat_interleave(torch.arange(nsets, device=dev), sizes.to(dev))
    pi = inputs.feistel_permutation(total, seed=2, device=dev)
    q_ids, q_keys = set_ids[pi].contiguous(), keys[pi].contiguous()
    del pi
    out = torch.empty(total, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"batch inputs ready: {nsets} sets, {total} keys")

    launch, tune_rec = None, None
    if getattr(args, "tune", False):
        from paper_1702_03154_amd import autotune
        launch = autotune.batch_launch(off, args.gamma, verbose=True)
        cache = autotune._load()
        tune_rec = cache.get(autotune.device_key(), {}).get(autotune.workload_key(off, args.gamma, 25))
        log(f"tuned launch {launch}")

    s = torch.cuda.current_stream()
    build_ms, lookup_ms, step_ms = [], [], []
    tot = None
    for it in range(warmup + steps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(s)
        b = mphf.build_batch(keys, off, args.gamma, 0, launch=launch)
        e1.record(s)
        b.lookup(q_ids, q_keys, out=out)
        e2.record(s)
        torch.cuda.synchronize()
        if it >= warmup:
            build_ms.append(e0.elapsed_time(e1))
            lookup_ms.append(e1.elapsed_time(e2))
            step_ms.append(e0.elapsed_time(e2))
        if tot is None:
            tot = b.totals()
        b.close()
        log(f"batch step {it}: build {e0.elapsed_time(e1):.3f} ms lookup {e1.elapsed_time(e2):.3f} ms")
    graph_rec = None
    if graph:
        # the planned batch: rebuild + lookup captured once in a HIP graph and replayed
        plan = mphf.Batch.plan(off, args.gamma, 0, launch=launch)
        plan.rebuild(keys).lookup(q_ids, q_keys, out=out)
        plan.status()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.rebuild(keys)
            plan.lookup(q_ids, q_keys, out=out)
        graph_ms = []
        for it in range(warmup + steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(s)
            g.replay()
            e1.record(s)
            torch.cuda.synchronize()
            if it >= warmup:
                graph_ms.append(e0.elapsed_time(e1))
        plan.status()
        del g
        plan.close()
        gm = statistics.median(graph_ms)
        log(f"graph replay {gm:.3f} ms")
        graph_rec = {"value": total / (gm / 1e3), "unit": "keys/s", "ms": gm,
                     "what": "planned batch: rebuild + lookup captured in one HIP graph, replayed"}

    # labels of every set are a bijection onto [1, n_s]: offset + label - 1 covers [0, total)
    gidx = off[q_ids] + out - 1
    seen = torch.zeros(total, dtype=torch.int8, device=dev)
    ok = bool(((out >= 1) & (gidx < off[q_ids + 1])).all())
    seen[gidx] = 1
    ok = ok and bool(seen.all())
    del seen, gidx

    # the same work as a loop of plain one-set-per-launch calls, over a seeded sample of the sets
    sample = inputs.feistel_permutation(nsets, seed=6)[: int(args.plain_sample)].tolist()
    plain_keys = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in sample:
        a, c = int(off_h[j]), int(off_h[j + 1])
        ks = keys[a:c]
        h = mphf.build(ks, args.gamma, 0)
        h.lookup(ks, out=out[a:c])
        h.close()
        plain_keys += c - a
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0

    tb, tl = statistics.median(build_ms), statistics.median(lookup_ms)
    value = total * steps / (sum(step_ms) / 1e3)
    return {
        "value": value, "unit": "keys/s", "ms_per_step": sum(step_ms) / steps, "steps": steps, "warmup": warmup,
        "config": {"workload": f"batched build + shuffled lookup of {nsets} independent sets, sizes "
                               f"log-uniform in [16, 65536] (seed 3), keys SplitMix64 per set (seed 4), "
                               f"gamma={args.gamma}", "sets": nsets, "keys": total, "gamma": args.gamma},
        "build_keys_per_s": total / (tb / 1e3), "lookup_queries_per_s": total / (tl / 1e3),
        "build_ms": tb, "lookup_ms": tl,
        "labels_bijective_per_set": ok,
        "bits_per_key": tot["bits_per_key"],
        "graph_replay": graph_rec,
        "launch": list(launch) if launch else "default (256 threads, 8 keys in flight)",
        "tuning": tune_rec and {"ms": tune_rec["ms"], "default_ms": tune_rec["default_ms"]},
        "plain_loop": {"value": plain_keys / plain_s, "unit": "keys/s", "sets": len(sample),
                       "keys": plain_keys,
                       "sample": "seeded Feistel sample of the sets; per set one plain build and "
                                 "one lookup of its keys, host-timed including every launch"},
        "batched_over_plain": value / (plain_keys / plain_s),
    }


def bench_batch(args):
    r = run_batch(args, args.steps, args.warmup)
    res = {"metric": METRIC, "value": r["value"], "unit": "keys/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u64", "data": "synthetic", "config": r["config"]}
    res.update({k: v for k, v in r.items() if k not in res and k not in ("steps",)})
    print(json.dumps(res))


# ---------------------------------------------------------------- serving

def run_serve(args) -> dict:
    """Serving: many resident functions, Poisson-arriving lookup requests from host memory, batched
    as they arrive; throughput at saturation and p50/p99 latency at fractions of the served and of
    the plain capacity, beside plain per-request lookups."""
    import numpy as np
    import torch

    from paper_1702_03154_amd import inputs, mphf

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nfn = int(args.functions)
    u = inputs._srl(inputs.splitmix64(6, nfn), 11).double() / float(1 << 53)
    sizes = torch.floor(1e6 * torch.pow(torch.tensor(1000.0, dtype=torch.float64), u) * args.serve_scale)
    sizes = sizes.long().clamp(min=1).tolist()
    fn_seeds = [int(v) & ((1 << 64) - 1) for v in inputs.splitmix64(7, nfn).tolist()]
    fns, struct_bytes = [], 0
    t0 = time.perf_counter()
    for j in range(nfn):
        k = inputs.splitmix64(fn_seeds[j], sizes[j], device=dev)
        h = mphf.build(k, 2.0, 0)
        del k
        fns.append(h)
        struct_bytes += h.stats()["structure_bytes"]
    torch.cuda.synchronize()
    log(f"{nfn} functions built ({sum(sizes)} keys, {struct_bytes / 2**30:.2f} GiB) in "
        f"{time.perf_counter() - t0:.1f} s")

    # requests: sizes floor(1e6^u), function uniform, 90% present keys (a uniform index into the
    # function's key stream), 10% absent keys (a separate stream); all in pinned host memory
    R = int(args.requests)
    ru = inputs._srl(inputs.splitmix64(8, 3 * R), 11).double() / float(1 << 53)
    rsize = torch.floor(torch.pow(torch.tensor(1e6, dtype=torch.float64), ru[:R])).long().tolist()
    rfn = (ru[R:2 * R] * nfn).long().clamp(max=nfn - 1).tolist()
    gaps = (-torch.log1p(-ru[2 * R:])).tolist()   # unit-rate exponential inter-arrival gaps
    qs, outs = [], []
    absent_at = 0
    for i in range(R):
        n, f = rsize[i], rfn[i]
        idx = (inputs.splitmix64(10_000 + i, n, device=dev) & ((1 << 62) - 1)) % sizes[f]
        q = torch.empty(0, dtype=torch.int64, device=dev)
        if n:
            # key idx of the function's stream: mix(seed + (idx + 1) * golden)
            z = (idx + 1) * inputs._s64(inputs._GOLDEN) + inputs._s64(fn_seeds[f])
            q = inputs._mix(z)
            absent = (inputs.splitmix64(20_000 + i, n, device=dev) & 1023) < 102
            na = int(absent.sum())
            if na:
                q[absent] = inputs.splitmix64(9, na, start=absent_at, device=dev)
                absent_at += na
        hq, ho = mphf.HostArray(n), mphf.HostArray(n)
        if n:
            hq.a[:] = q.cpu().numpy().view(np.uint64)
        qs.append(hq)
        outs.append(ho)
    total_keys = sum(rsize)
    log(f"{R} requests, {total_keys} keys")

    # plain: one lookup per request, each copied in, labelled, copied out and waited for
    dq = torch.empty(max(rsize) + 1, dtype=torch.int64, device=dev)
    do = torch.empty_like(dq)
    plain_lab = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(R):
        n = rsize[i]
        if n:
            dq[:n].copy_(torch.from_numpy(qs[i].a.view(np.int64)), non_blocking=True)
            fns[rfn[i]].lookup(dq[:n], out=do[:n])
            outs[i].a.view(np.int64)[:] = do[:n].cpu().numpy()
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    plain_rps = R / plain_s
    for i in range(R):
        plain_lab.append(outs[i].a.copy())
    log(f"plain: {plain_rps:.0f} requests/s, {total_keys / plain_s:.3e} keys/s")

    server = mphf.Server(hbm_budget=int(args.hbm_budget), max_inflight=int(args.inflight))
    ids = [server.register(h) for h in fns]

    def run(rate):
        for o in outs:
            o.a[:] = 0
        tickets = [None] * R
        gc.collect()
        gc.disable()   # no collector pause inside the arrival loop
        start = time.perf_counter()
        t_next = start
        for i in range(R):
            if rate:
                t_next += gaps[i] / rate
                while time.perf_counter() < t_next:
                    pass
            tickets[i] = server.submit(ids[rfn[i]], qs[i].a, outs[i].a)
        infos = [server.poll(t, wait=True) for t in tickets]
        wall = time.perf_counter() - start
        gc.enable()
        lat = np.array([x["done_us"] - x["submit_us"] for x in infos])
        ok = all(np.array_equal(outs[i].a, plain_lab[i]) for i in range(R))
        return {"offered_requests_per_s": rate or None, "requests_per_s": R / wall, "keys_per_s": total_keys / wall,
                "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
                "max_us": float(lat.max()),
                "mean_batch_requests": float(np.mean([x["batch_requests"] for x in infos])),
                "equal_to_plain": ok}

    sat = run(0)
    sat_rps = sat["requests_per_s"]
    log(f"served at saturation: {sat_rps:.0f} requests/s, p50 {sat['p50_us']:.0f} us")
    # the latency-throughput curve: Poisson arrivals at fractions of the served saturation rate,
    # and at the rates plain per-request lookups could sustain
    of_served, of_plain = {}, {}
    for f in (0.25, 0.5, 0.8, 0.95):
        of_served[str(f)] = run(f * sat_rps)
        log(f"load {f} of served: p50 {of_served[str(f)]['p50_us']:.0f} us p99 {of_served[str(f)]['p99_us']:.0f} us")
    for f in (0.5, 0.8, 0.95):
        of_plain[str(f)] = run(f * plain_rps)
        log(f"load {f} of plain: p50 {of_plain[str(f)]['p50_us']:.0f} us p99 {of_plain[str(f)]['p99_us']:.0f} us")
    st = server.stats()
    server.close()
    for o in qs + outs:
        o.close()
    for h in fns:
        h.close()
    pcie = pcie_rate()
    log(f"host exchange over PCIe: {pcie['bytes_per_s'] / 1e9:.1f} GB/s; served moves "
        f"{16 * sat['keys_per_s'] / 1e9:.1f} GB/s")
    return {
        "value": sat["keys_per_s"], "unit": "keys/s", "ms_per_step": 1e3 * total_keys / sat["keys_per_s"],
        "config": {"workload": f"serving: {nfn} resident functions, sizes floor(1e6*1000^u*{args.serve_scale}) "
                               f"(seed 6), gamma=2; {R} requests of floor(1e6^u) keys (seed 8), 90% present, "
                               f"10% absent, from pinned host memory",
                   "functions": nfn, "function_keys": sum(sizes), "structure_bytes": struct_bytes,
                   "requests": R, "request_keys": total_keys, "hbm_budget": int(args.hbm_budget),
                   "max_inflight": int(args.inflight)},
        "plain": {"requests_per_s": plain_rps, "keys_per_s": total_keys / plain_s,
                  "what": "per request: copy in, lookup, copy out, wait"},
        "served_saturation": sat, "served_over_plain": sat["keys_per_s"] / (total_keys / plain_s),
        "pcie": {"exchange_bytes_per_s": pcie["bytes_per_s"], "served_bytes_per_s": 16 * sat["keys_per_s"],
                 "frac": 16 * sat["keys_per_s"] / pcie["bytes_per_s"],
                 "what": "each served key is read from pinned host memory and its label written back (8 B each "
                         "way) against a kernel exchanging pinned host memory over PCIe, measured in this run"},
        "poisson_loads_of_served_capacity": of_served,
        "poisson_loads_of_plain_capacity": of_plain,
        "server_stats": st,
    }


def bench_serve(args):
    r = run_serve(args)
    res = {"metric": METRIC, "value": r["value"], "unit": "keys/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64", "data": "synthetic", "config": r["config"]}
    res.update({k: v for k, v in r.items() if k not in res})
    print(json.dumps(res))


def bench_kmer(args):
    """k-mer keys: canonical 31-mers of a seeded random DNA sequence, first occurrences up to the
    target; plain build + lookup, and the batched path over hash sets, on the same keys."""
    import math

    import torch

    from paper_1702_03154_amd import inputs, mphf

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nb, target, k = int(args.kmer_bases), int(args.kmer_keys), 31
    t0 = time.perf_counter()
    seq = inputs.dna_sequence(nb, seed=5, device=dev)
    km = mphf.kmers(seq, nb, k)
    del seq
    keys = mphf.first_occurrences(km, target)
    del km
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    n = keys.numel()
    print(f"# {n} distinct canonical {k}-mers from {nb} bases in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    s = torch.cuda.current_stream()
    out = torch.empty_like(keys)

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        r = fn()
        e1.record(s)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    def bijective(lab, base=None):
        seen = torch.zeros(n, dtype=torch.int8, device=dev)
        idx = lab - 1 if base is None else base + lab - 1
        ok = bool(((idx >= 0) & (idx < n)).all())
        seen[idx.clamp(0, n - 1)] = 1
        return ok and bool(seen.all())

    # plain path
    build_ms, lookup_ms = [], []
    stats = None
    for it in range(args.warmup + args.steps):
        h, tb = timed(lambda: mphf.build(keys, args.gamma, 0))
        _, tl = timed(lambda: h.lookup(keys, out=out))
        if it >= args.warmup:
            build_ms.append(tb)
            lookup_ms.append(tl)
        if stats is None:
            stats = h.stats()
        h.close()
        print(f"# plain step {it}: build {tb:.1f} ms lookup {tl:.1f} ms", file=sys.stderr, flush=True)
    plain_ok = bijective(out)
    # per-level placed keys against the exact occupancy mean (structured keys, hashed)
    worst = 0.0
    for d in range(stats["num_levels"]):
        nd, md, wd = stats["level_n"][d], stats["level_m"][d], stats["level_weight"][d]
        if nd < 100:
            break
        # exact occupancy moments: E[X] = n (1-1/m)^(n-1), E[X(X-1)] = n (n-1) (1-1/m) (1-2/m)^(n-2)
        mu = nd * math.exp((nd - 1) * math.log1p(-1.0 / md))
        e2 = (md - 1) / md * nd * (nd - 1) * math.exp((nd - 2) * math.log1p(-2.0 / md))
        var = e2 + mu - mu * mu
        worst = max(worst, abs(wd - mu) / math.sqrt(max(var, 1e-9)))

    # batched path: hash sets of about n / 2^bits keys (the plain build's cached workspace is
    # released first: both paths together would not fit)
    mphf.trim()
    bits = int(args.kmer_set_bits)
    # the first call also maps the partition's temporary device memory (about 2 n words)
    (grouped, off), tpart_first = timed(lambda: mphf.partition_sets(keys, bits, seed=0x5E7))
    del grouped, off
    (grouped, off), tpart = timed(lambda: mphf.partition_sets(keys, bits, seed=0x5E7))
    print(f"# partition: first call {tpart_first:.1f} ms, then {tpart:.1f} ms", file=sys.stderr, flush=True)
    ids, tids = timed(lambda: mphf.set_ids(keys, bits, seed=0x5E7))
    bb_ms, bl_ms = [], []
    for it in range(args.warmup + args.steps):
        b, tb = timed(lambda: mphf.build_batch(grouped, off, args.gamma, 0))
        _, tl = timed(lambda: b.lookup(ids, keys, out=out))
        if it >= args.warmup:
            bb_ms.append(tb)
            bl_ms.append(tl)
        tot = b.totals()
        b.close()
        print(f"# batched step {it}: build {tb:.1f} ms lookup {tl:.1f} ms", file=sys.stderr, flush=True)
    batch_ok = bijective(out, off[ids])
    import statistics
    tb, tl = statistics.median(build_ms), statistics.median(lookup_ms)
    bb, bl = statistics.median(bb_ms), statistics.median(bl_ms)
    res = {
        "metric": METRIC,
        "value": n / ((tb + tl) / 1e3), "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": tb + tl,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"canonical {k}-mers of a {nb}-base SplitMix64 (seed 5) DNA sequence, first "
                               f"{target} distinct in sequence order, gamma={args.gamma}",
                   "keys": n, "bases": nb, "k": k, "gamma": args.gamma, "key_bytes": 8 * n},
        "plain": {"build_keys_per_s": n / (tb / 1e3), "lookup_queries_per_s": n / (tl / 1e3),
                  "build_ms": tb, "lookup_ms": tl, "labels_bijective": plain_ok,
                  "levels": stats["num_levels"], "bits_per_key": stats["bits_per_key"],
                  "level_n": stats["level_n"][:stats["num_levels"]],
                  "worst_level_sigma": worst, "peak_bytes": stats["peak_bytes"]},
        "batched": {"sets": 1 << bits, "partition_ms": tpart, "partition_first_call_ms": tpart_first,
                    "set_ids_ms": tids,
                    "build_keys_per_s": n / (bb / 1e3), "lookup_queries_per_s": n / (bl / 1e3),
                    "build_ms": bb, "lookup_ms": bl, "labels_bijective": batch_ok,
                    "bits_per_key": tot["bits_per_key"]},
    }
    print(json.dumps(res))


def bench_stream(args):
    """Streaming build over n generated keys (never stored), or with --stream-host over the same keys
    stored in pinned host memory; then the lookup of every key, regenerated chunk by chunk; bijection
    checked with one byte per label."""
    import statistics

    import numpy as np
    import torch

    from paper_1702_03154_amd import mphf

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = int(args.n)
    resident = int(args.resident_keys)
    s = torch.cuda.current_stream()
    host = None
    if args.stream_host:
        # the same keys stored in pinned host memory, filled from the device in chunks
        t0 = time.perf_counter()
        host = mphf.HostArray(n)
        step = 1 << 28
        for c0 in range(0, n, step):
            c = min(step, n - c0)
            host.a[c0:c0 + c] = mphf.stream_keys(1, c0, c).cpu().numpy().view(np.uint64)
        log(f"{n} keys in pinned host memory ({8 * n / 2**30:.1f} GiB) in {time.perf_counter() - t0:.1f} s")
    build_ms, builds = [], []
    h = None
    for it in range(args.warmup + args.steps):
        if h is not None:
            h.close()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        if host is not None:
            h = mphf.build_host(host, args.gamma, 0, resident_keys=resident)
        else:
            h = mphf.build_stream(n, 1, args.gamma, 0, resident_keys=resident)
        e1.record(s)
        torch.cuda.synchronize()
        paths = h.stats()["level_path"]
        builds.append({"ms": e0.elapsed_time(e1), "streamed": sum(p.startswith("streamed") for p in paths),
                       "paths": sorted(set(paths))})
        if it >= args.warmup:
            build_ms.append(e0.elapsed_time(e1))
        log(f"stream build {it}: {e0.elapsed_time(e1):.1f} ms, level paths {sorted(set(paths))}")
    st = h.stats()
    chunk = 1 << 28
    seen = torch.zeros(n, dtype=torch.int8, device=dev)
    q = torch.empty(min(chunk, n), dtype=torch.int64, device=dev)
    lab = torch.empty_like(q)
    lookup_ms, in_range = 0.0, True
    for c0 in range(0, n, chunk):
        c = min(chunk, n - c0)
        q[:c] = mphf.stream_keys(1, c0, c)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        h.lookup(q[:c], out=lab[:c])
        e1.record(s)
        torch.cuda.synchronize()
        lookup_ms += e0.elapsed_time(e1)
        v = lab[:c]
        in_range = in_range and bool(((v >= 1) & (v <= n)).all())
        seen[(v - 1).clamp(0, n - 1)] = 1
    ok = in_range and bool(seen.all())
    del seen
    streamed = sum(1 for x in st["level_n"][:st["num_levels"]] if x > resident)
    tb = statistics.median(build_ms)
    res = {
        "metric": METRIC,
        "value": n / ((tb + lookup_ms) / 1e3), "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": tb + lookup_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"streaming build over {n} SplitMix64 keys (seed 1) "
                               f"{'stored in pinned host memory' if host is not None else 'generated on the fly'}, "
                               f"re-scanned while more than {resident} survive, gamma={args.gamma}; "
                               f"lookup of every key regenerated in chunks",
                   "n": n, "gamma": args.gamma, "resident_keys": resident,
                   "key_source": "host" if host is not None else "generated"},
        "builds": builds,
        "build_keys_per_s": n / (tb / 1e3), "lookup_queries_per_s": n / (lookup_ms / 1e3),
        "build_ms": tb, "lookup_ms": lookup_ms, "labels_bijective": ok,
        "levels": st["num_levels"], "streamed_levels": streamed, "bits_per_key": st["bits_per_key"],
        "n_fallback": st["n_fallback"], "structure_bytes": st["structure_bytes"],
        "level_n": st["level_n"][:st["num_levels"]],
    }
    h.close()
    if host is not None:
        host.close()
    print(json.dumps(res))


def bench_gamma(args):
    """The influence of gamma (build time, query time, bits/key, probes per query) and the 1024-bit
    rank sampling ('minirank'), each beside the space analysis."""
    import math
    import statistics

    import torch

    from paper_1702_03154_amd import inputs, mphf

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = int(args.n)
    keys = inputs.keys(n, seed=1, device=dev)
    queries = inputs.shuffled_queries(keys, seed=2)
    out = torch.empty_like(keys)
    s = torch.cuda.current_stream()
    rows = []
    runs = [(g, 512) for g in (1.0, 1.5, 2.0, 3.0, 5.0, 7.0, 10.0)] + [(1.0, 1024), (2.0, 1024)]
    for gamma, rs in runs:
        bms, lms = [], []
        st = None
        for it in range(args.warmup + args.steps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            torch.cuda.synchronize()
            e0.record(s)
            h = mphf.build(keys, gamma, 0, rank_sample=rs)
            e1.record(s)
            h.lookup(queries, out=out)
            e2.record(s)
            torch.cuda.synchronize()
            if it >= args.warmup:
                bms.append(e0.elapsed_time(e1))
                lms.append(e1.elapsed_time(e2))
            st = h.stats()
            h.close()
        tb, tl = statistics.median(bms), statistics.median(lms)
        row = {"gamma": gamma, "rank_sample": rs, "build_keys_per_s": n / (tb / 1e3),
               "lookup_queries_per_s": n / (tl / 1e3), "build_ms": tb, "lookup_ms": tl,
               "bits_per_key": st["bits_per_key"],
               "bits_per_key_analysis": (1 + 64 / rs) * gamma * math.exp(1 / gamma),
               "mean_probes": mean_probes(st), "mean_probes_analysis": math.exp(1 / gamma),
               "levels": st["num_levels"], "n_fallback": st["n_fallback"]}
        rows.append(row)
        print(f"# gamma {gamma} rank {rs}: build {tb:.1f} ms lookup {tl:.1f} ms, {row['bits_per_key']:.3f} bits/key",
              file=sys.stderr, flush=True)
    base = next(r for r in rows if r["gamma"] == 2.0 and r["rank_sample"] == 512)
    res = {
        "metric": METRIC,
        "value": n / ((base["build_ms"] + base["lookup_ms"]) / 1e3), "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": base["build_ms"] + base["lookup_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"gamma sweep: plain build + shuffled lookup of N={n} SplitMix64 keys (seed 1) "
                               f"for gamma in 1..10 and 1024-bit rank sampling", "n": n},
        "rows": rows,
    }
    print(json.dumps(res))




def plain_steps(mphf, keys, queries, out, gamma, steps, warmup, tag="", **build_opts):
    """`warmup` + `steps` build + lookup steps; per-step event times on the current stream."""
    import torch
    s = torch.cuda.current_stream()
    build_ms, lookup_ms, step_ms = [], [], []
    stats = None
    for it in range(warmup + steps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(s)
        h = mphf.build(keys, gamma, 0, **build_opts)
        e1.record(s)
        h.lookup(queries, out=out)
        e2.record(s)
        torch.cuda.synchronize()
        if it >= warmup:
            build_ms.append(e0.elapsed_time(e1))
            lookup_ms.append(e1.elapsed_time(e2))
            step_ms.append(e0.elapsed_time(e2))
        if stats is None:
            stats = h.stats()
        h.close()
        log(f"{tag}step {it}: build {e0.elapsed_time(e1):.3f} ms lookup {e1.elapsed_time(e2):.3f} ms")
    return build_ms, lookup_ms, step_ms, stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["plain", "batch", "serve", "kmer", "stream", "gamma", "roofline"],
                    default="plain")
    ap.add_argument("--resident-keys", type=float, default=2 ** 31, help="stream: survivors kept in memory")
    ap.add_argument("--stream-host", action="store_true", help="stream: keys stored in pinned host memory")
    ap.add_argument("--kmer-bases", type=float, default=4.2e9, help="kmer: sequence length")
    ap.add_argument("--kmer-keys", type=float, default=4e9, help="kmer: distinct k-mers kept")
    ap.add_argument("--kmer-set-bits", type=float, default=15, help="kmer: log2 of the batched sets")
    ap.add_argument("--functions", type=float, default=64, help="serve: resident functions")
    ap.add_argument("--serve-scale", type=float, default=1.0, help="serve: function size scale")
    ap.add_argument("--requests", type=float, default=2000, help="serve: requests per run")
    ap.add_argument("--hbm-budget", type=float, default=2 << 30, help="serve: admission budget (bytes)")
    ap.add_argument("--inflight", type=float, default=2, help="serve: batches in flight")
    ap.add_argument("--sets", type=float, default=65536)
    ap.add_argument("--plain-sample", type=float, default=2048)
    ap.add_argument("--tune", action="store_true", help="batch: autotune the build launch first")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=float, default=1e9)
    ap.add_argument("--gamma", type=float, default=2.0)
    ap.add_argument("--cpu-sample", type=float, default=1e8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain: only the timed steps and the roofline (no gamma1, batched, served parts)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (a known-size kernel for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path is built "
              "and timed on a single GPU; no multi-GPU sharding is implemented)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
    workloads = {"batch": bench_batch, "serve": bench_serve, "kmer": bench_kmer, "gamma": bench_gamma,
                 "roofline": bench_roofline}
    if args.workload in workloads:
        workloads[args.workload](args)
        return
    if args.workload == "stream":
        if args.n == 1e9:
            args.n = 1e10
        bench_stream(args)
        return

    import statistics

    import torch

    from paper_1702_03154_amd import inputs, mphf

    n = int(args.n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    keys = inputs.keys(n, seed=1, device=dev)
    queries = inputs.shuffled_queries(keys, seed=2)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"inputs ready: {n} keys")

    build_ms, lookup_ms, step_ms, stats = plain_steps(mphf, keys, queries, out, args.gamma, args.steps,
                                                      args.warmup)
    ok = bool(torch.equal(torch.sort(out).values, torch.arange(1, n + 1, device=dev)))
    tb, tl = (statistics.median(x) for x in (build_ms, lookup_ms))
    total_ms = sum(step_ms)

    # ---- roofline of the lookup (the dominant kernel: one launch, timed with events on its stream)
    probes = mean_probes(stats)
    foot = int(stats["lookup_bytes"])
    sec_rate = probe_rate("random_sector64", foot, ops=1 << 29)
    line_rate = probe_rate("random_read8", foot, ops=1 << 29)
    copy_rate = probe_rate("stream_copy", 4 << 30)
    lk_bytes = n * LOOKUP_BYTES_PER_QUERY
    lk_ops = n * probes
    t_stream = lk_bytes / (HBM_PEAK_GBS * 1e9)
    t_rand = lk_ops / sec_rate["ops_per_s"]
    t_lb = max(t_stream, t_rand)
    achieved = lk_bytes / (tl / 1e3) / 1e9
    roofline = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(n), "kernel": "k_lookup",
        "algorithmic_bytes_per_query": LOOKUP_BYTES_PER_QUERY,
        "random": {"ops_per_query": probes, "ops_per_s": lk_ops / (tl / 1e3),
                   "peak_ops_per_s": sec_rate["ops_per_s"], "frac": lk_ops / (tl / 1e3) / sec_rate["ops_per_s"],
                   "footprint_bytes": foot,
                   "what": "level probes (one 64-byte sector each, e^(1/gamma) per member query) against "
                           "random 64-byte sector reads over the same footprint, measured in this run"},
        "line_traffic_bytes_per_query": LOOKUP_BYTES_PER_QUERY + LINE_BYTES * probes,
        "random_read8_ops_per_s": line_rate["ops_per_s"],
        "stream_copy_gbs": copy_rate["bytes_per_s"] / 1e9,
        "t_lb_ms": t_lb * 1e3, "t_meas_ms": tl, "t_lb_over_t_meas": t_lb / (tl / 1e3),
    }
    log(f"lookup: {achieved:.0f} GB/s algorithmic, probes {lk_ops / (tl / 1e3):.3e}/s of "
        f"{sec_rate['ops_per_s']:.3e}/s at {foot / 2**20:.0f} MiB; T_lb/T = {t_lb / (tl / 1e3):.3f}")

    # ---- roofline of the build: its streaming bytes, and its random test-and-sets and bit reads,
    # which the partitioned levels make in LDS (a global test-and-set model is given for context)
    bb = build_algorithmic_bytes(stats)
    bops = build_random_ops(stats)
    lds_rate = probe_rate("lds_atomic_or", 8192, ops=1 << 32)
    m0 = stats["level_m"][0] if stats["num_levels"] else 1
    glob_rate = probe_rate("random_atomic_or", 2 * ((m0 + 63) // 64) * 8, ops=1 << 28)
    tb_stream = bb / (HBM_PEAK_GBS * 1e9)
    tb_lb = max(tb_stream, bops / lds_rate["ops_per_s"])
    build_roofline = {
        "bound": "hbm", "achieved": bb / (tb / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": bb / (tb / 1e3) / 1e9 / HBM_PEAK_GBS, "traffic": measured_build_traffic(n),
        "algorithmic_bytes_per_key": bb / n,
        "random": {"ops_per_key": bops / n, "lds_peak_ops_per_s": lds_rate["ops_per_s"],
                   "global_atomic_peak_ops_per_s": glob_rate["ops_per_s"],
                   "global_atomic_model_ms": 1e3 * bops / glob_rate["ops_per_s"],
                   "what": "a test-and-set and a filter read per key and level; here made in LDS by the "
                           "position-partitioned levels; the global-atomic model is the same ops at the "
                           "measured random atomicOr rate over level 0's A and C"},
        "t_lb_ms": tb_lb * 1e3, "t_meas_ms": tb, "t_lb_over_t_meas": tb_lb / (tb / 1e3),
        "stream_copy_frac": bb / (tb / 1e3) / copy_rate["bytes_per_s"],
    }

    res = {
        "metric": METRIC,
        "value": n * args.steps / (total_ms / 1e3),
        "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"plain build + shuffled lookup of N={n} distinct SplitMix64 keys "
                               f"(seed 1), gamma={args.gamma}", "n": n, "gamma": args.gamma},
        "build_keys_per_s": n / (tb / 1e3),
        "lookup_queries_per_s": n / (tl / 1e3),
        "build_ms": tb, "lookup_ms": tl,
        "labels_bijective": ok,
        "levels": stats["num_levels"], "bits_per_key": stats["bits_per_key"],
        "n_fallback": stats["n_fallback"], "mean_probes": probes,
        "roofline": roofline,
        "build_roofline": build_roofline,
    }

    if not args.no_extras:
        # gamma = 1 on the same keys and queries (the second gamma of the large plain workload)
        b1, l1, _, st1 = plain_steps(mphf, keys, queries, out, 1.0, 3, 1, tag="gamma 1 ")
        ok1 = bool(torch.equal(torch.sort(out).values, torch.arange(1, n + 1, device=dev)))
        t1b, t1l = statistics.median(b1), statistics.median(l1)
        res["gamma1"] = {"build_keys_per_s": n / (t1b / 1e3), "lookup_queries_per_s": n / (t1l / 1e3),
                         "build_ms": t1b, "lookup_ms": t1l, "labels_bijective": ok1,
                         "levels": st1["num_levels"], "bits_per_key": st1["bits_per_key"],
                         "n_fallback": st1["n_fallback"], "mean_probes": mean_probes(st1), "steps": 3}
        # the same build with every level filled by global atomicOr test-and-set (the old bit
        # deciding the collision mark): the design the partitioned levels replace, measured
        ba, _, _, sta = plain_steps(mphf, keys, queries, out, args.gamma, 2, 1, tag="atomic levels ",
                                    atomic_levels=True)
        oka = bool(torch.equal(torch.sort(out).values, torch.arange(1, n + 1, device=dev)))
        tba = statistics.median(ba)
        res["atomic_levels"] = {
            "build_ms": tba, "build_keys_per_s": n / (tba / 1e3), "over_partitioned": tba / tb,
            "labels_bijective": oka, "same_total_bits": sta["total_bits"] == stats["total_bits"], "steps": 2,
            "what": "every level built by global atomicOr test-and-set on interleaved A/C words "
                    "(MPHF_FLAG_ATOMIC_LEVELS) instead of the position-partitioned LDS passes"}
    keys_host = queries_host = None
    if not args.no_cpu_baseline:
        import numpy as np
        keys_host = keys.cpu().numpy().view(np.uint64)
        queries_host = queries.cpu().numpy().view(np.uint64)
    del keys, queries, out
    torch.cuda.empty_cache()
    mphf.trim()

    if not args.no_extras:
        rb = run_batch(args, 3, 1, graph=True)
        res["batched"] = {k: rb[k] for k in ("value", "unit", "config", "build_keys_per_s", "lookup_queries_per_s",
                                            "build_ms", "lookup_ms", "labels_bijective_per_set", "bits_per_key",
                                            "graph_replay", "plain_loop", "batched_over_plain")}
        res["batched_over_plain"] = rb["batched_over_plain"]
        mphf.trim()
        torch.cuda.empty_cache()
        rs = run_serve(args)
        res["served"] = {k: rs[k] for k in ("value", "unit", "config", "plain", "served_saturation",
                                            "served_over_plain", "pcie", "poisson_loads_of_served_capacity",
                                            "poisson_loads_of_plain_capacity")}
        res["served_over_plain"] = rs["served_over_plain"]

    if not args.no_cpu_baseline:
        cb = cpu_baseline(int(args.cpu_sample), args.gamma)
        log(f"cpu oracle: {cb['value']:.3e} keys/s")
        cb["threaded"] = threaded_baseline(keys_host, queries_host, args.gamma)
        log(f"cpu threaded: {cb['threaded']['value']:.3e} keys/s on {cb['threaded']['cores']} threads")
        cb["host"] = host_info()
        res["cpu_baseline"] = cb
    print(json.dumps(res))


if __name__ == "__main__":
    main()
