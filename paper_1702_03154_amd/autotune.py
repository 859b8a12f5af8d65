"""Autotuner for the batched build's launch configuration.

The batched build kernel has five knobs: threads per workgroup (128, 256, 512), keys each
thread keeps in flight in the level passes (4, 8, 16), workgroups per CU (bounded by the LDS
the largest set needs), and the size-class split of its work queue: the class below which a
set counts as small, and which share of the workgroups takes small sets first (one queue,
largest sets first; or every 2nd or 4th workgroup on the sets below 4096 keys).  Which is
fastest depends on the device and on the batch's size distribution, not on the key values, so
the tuner times every candidate on seeded synthetic keys of the caller's set sizes with a
planned batch (build kernels only, HIP events on the build stream, median of a few
repetitions) and keeps the winner in a JSON cache on disk.

The cache key is the device (name, architecture, CU count), gamma, the level limit and the
histogram of set sizes by power of two (sets of sizes in [2^k, 2^(k+1)) behave alike), so a
new batch with the same shape reuses the tuned choice without timing anything.

    launch = autotune.batch_launch(offsets, gamma)         # cached or tuned now
    b = mphf.build_batch(keys, offsets, gamma, launch=launch)
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
import threading

import torch

from . import inputs, mphf

THREADS = (128, 256, 512)
ITEMS = (4, 8, 16)
WGS_PER_CU = (0, 2, 4)          # 0: as many as the LDS allows (at most 8)
# (small class, small every): (1, 2) has no small sets, so one queue, largest first
QUEUES = ((1, 2), (13, 2), (13, 4))
DEFAULT = (256, 4, 0, 13, 2)    # the library's default launch

_lock = threading.Lock()


def cache_path() -> str:
    p = os.environ.get("MPHF_TUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "mphf_amd", "batch_launch.json")


def device_key(device=None) -> str:
    d = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    p = torch.cuda.get_device_properties(d)
    arch = getattr(p, "gcnArchName", "")
    return f"{p.name}|{arch}|{p.multi_processor_count}"


def workload_key(offsets: torch.Tensor, gamma: float, max_levels: int) -> str:
    sizes = (offsets[1:] - offsets[:-1]).cpu()
    cls = torch.where(sizes > 0, torch.floor(torch.log2(sizes.clamp(min=1).double())).long() + 1,
                      torch.zeros_like(sizes))
    hist = torch.bincount(cls, minlength=65).tolist()
    sig = json.dumps({"gamma": float(gamma), "D": int(max_levels), "hist": hist}, sort_keys=True)
    return hashlib.sha256(sig.encode()).hexdigest()[:24]


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def candidates():
    for t in THREADS:
        for i in ITEMS:
            for w in WGS_PER_CU:
                for c, e in QUEUES:
                    yield (t, i, w, c, e)


def time_launch(offsets: torch.Tensor, keys: torch.Tensor, gamma: float, max_levels: int, launch,
                reps: int = 3) -> float:
    """Median milliseconds of one rebuild of a planned batch with this launch configuration."""
    b = mphf.Batch.plan(offsets, gamma, 0, max_levels=max_levels, launch=launch)
    try:
        s = torch.cuda.current_stream()
        b.rebuild(keys)
        b.status()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            b.rebuild(keys)
            e1.record(s)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        b.status()
        return statistics.median(ms)
    finally:
        b.close()


def tune(offsets: torch.Tensor, gamma: float = 2.0, max_levels: int = 25, reps: int = 3,
         keys: torch.Tensor | None = None, verbose: bool = False) -> dict:
    """Time every candidate on synthetic keys of these set sizes; returns the result record."""
    offsets = offsets.cuda() if not offsets.is_cuda else offsets
    if keys is None:
        sizes = (offsets[1:] - offsets[:-1]).cpu()
        keys = inputs.set_keys(sizes, seed=0x7E57, device=offsets.device)
    results = []
    for c in candidates():
        t = time_launch(offsets, keys, gamma, max_levels, c, reps)
        results.append((t, c))
        if verbose:
            print(f"# tune {c}: {t:.3f} ms", flush=True)
    results.sort()
    best_t, best = results[0]
    default_t = next(t for t, c in results if c == DEFAULT)
    return {"launch": list(best), "ms": best_t, "default_ms": default_t,
            "candidates": [[list(c), t] for t, c in results]}


def batch_launch(offsets: torch.Tensor, gamma: float = 2.0, max_levels: int = 25, retune: bool = False,
                 verbose: bool = False):
    """The tuned (threads, items, workgroups per CU, small class, small every) for this device and
    batch shape: from the cache, or tuned now and stored."""
    dk, wk = device_key(offsets.device if offsets.is_cuda else None), workload_key(offsets, gamma, max_levels)
    with _lock:
        cache = _load()
        rec = cache.get(dk, {}).get(wk)
        if rec is not None and not retune:
            return tuple(rec["launch"])
        rec = tune(offsets, gamma, max_levels, verbose=verbose)
        cache = _load()
        cache.setdefault(dk, {})[wk] = rec
        _store(cache)
        return tuple(rec["launch"])
