"""Python binding of ``libmphf.so`` (ctypes): argument marshalling only.

Every step of the build and of the lookup runs in the library's HIP kernels.
PyTorch supplies device memory and the current stream, nothing else.  If the
library is missing, every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmphf.so")
MAX_LEVELS = 64

OK, E_INVALID, E_NOMEM, E_DUPLICATE_KEYS, E_DEVICE = range(5)


class MphfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mphf status {status}: {msg}")
        self.status = status


class DuplicateKeysError(MphfError):
    pass


class Opts(C.Structure):
    _fields_ = [("max_levels", C.c_uint32), ("rank_sample", C.c_uint32),
                ("mem_budget", C.c_uint64), ("keep_collisions", C.c_uint32),
                ("flags", C.c_uint32), ("batch_threads", C.c_uint32), ("batch_items", C.c_uint32),
                ("batch_wgs_per_cu", C.c_uint32), ("bucket_bits", C.c_uint32),
                ("batch_small_class", C.c_uint32), ("batch_small_every", C.c_uint32)]


_U64L = C.c_uint64 * MAX_LEVELS


class Stats(C.Structure):
    _fields_ = [("n", C.c_uint64), ("gamma", C.c_double), ("seed", C.c_uint64),
                ("num_levels", C.c_uint32), ("rank_sample", C.c_uint32),
                ("level_n", _U64L), ("level_m", _U64L), ("level_weight", _U64L),
                ("level_offset", _U64L), ("level_seed", _U64L),
                ("n_fallback", C.c_uint64), ("total_bits", C.c_uint64),
                ("rank_entries", C.c_uint64), ("structure_bytes", C.c_uint64),
                ("bits_per_key", C.c_double), ("peak_bytes", C.c_uint64), ("lookup_bytes", C.c_uint64),
                ("level_path", C.c_uint32 * MAX_LEVELS), ("bucket_bits", C.c_uint32), ("reserved", C.c_uint32)]

# values of Stats.level_path (how a level was built)
PATH_NAMES = {1: "tail", 2: "one_pass", 3: "two_pass", 4: "two_pass_wide", 5: "atomic", 6: "streamed",
              7: "streamed_atomic"}


class SetInfo(C.Structure):
    _fields_ = [("n", C.c_uint64), ("num_levels", C.c_uint32), ("n_fallback", C.c_uint32),
                ("level_n", _U64L), ("level_m", _U64L), ("level_offset", _U64L),
                ("total_bits", C.c_uint64)]


class KeyStream(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("start", C.c_uint64)]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_inflight", C.c_uint32),
                ("max_batch_requests", C.c_uint32)]


class RequestInfo(C.Structure):
    _fields_ = [("done", C.c_uint32), ("batch_requests", C.c_uint32), ("batch", C.c_uint64),
                ("submit_us", C.c_double), ("start_us", C.c_double), ("done_us", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("requests", C.c_uint64), ("keys", C.c_uint64), ("batches", C.c_uint64),
                ("max_batch_requests_seen", C.c_uint64), ("peak_bytes_in_flight", C.c_uint64)]


class View(C.Structure):
    _fields_ = [("words", C.c_void_p), ("rank", C.c_void_p), ("fallback_keys", C.c_void_p),
                ("collisions", C.c_void_p), ("total_words", C.c_uint64), ("rank_entries", C.c_uint64),
                ("n_fallback", C.c_uint64)]


_lib = None


def lib() -> C.CDLL:
    """Load libmphf.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32, st = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
        sig = {
            "mphf_default_opts": (st, [C.POINTER(Opts)]),
            "mphf_build": (vp, [vp, u64, C.c_double, u64]),
            "mphf_lookup": (C.c_int, [vp, vp, u64, vp]),
            "mphf_build_ex": (st, [vp, u64, C.c_double, u64, C.POINTER(Opts), vp, C.POINTER(vp)]),
            "mphf_lookup_ex": (st, [vp, vp, u64, vp, vp]),
            "mphf_destroy": (None, [vp]),
            "mphf_stats": (st, [vp, C.POINTER(Stats)]),
            "mphf_view": (st, [vp, C.POINTER(View)]),
            "mphf_export": (st, [vp, vp, u64, vp, u64, vp, u64]),
            "mphf_export_collisions": (st, [vp, u32, vp, u64]),
            "mphf_positions": (st, [vp, u64, u64, u64, vp, vp]),
            "mphf_trim": (st, []),
            "mphf_build_batch": (st, [vp, vp, u64, C.c_double, u64, C.POINTER(Opts), vp, C.POINTER(vp)]),
            "mphf_batch_lookup": (st, [vp, vp, vp, u64, vp, vp]),
            "mphf_batch_set_info": (st, [vp, u64, C.POINTER(SetInfo)]),
            "mphf_batch_export_set": (st, [vp, u64, vp, u64, vp, u64]),
            "mphf_batch_totals": (st, [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                       C.POINTER(C.c_uint64), C.POINTER(C.c_double)]),
            "mphf_batch_destroy": (None, [vp]),
            "mphf_batch_plan": (st, [vp, u64, C.c_double, u64, C.POINTER(Opts), vp, C.POINTER(vp)]),
            "mphf_batch_rebuild": (st, [vp, vp, vp]),
            "mphf_batch_status": (st, [vp, vp]),
            "mphf_batch_export_sectors": (st, [vp, u64, vp, u64]),
            "mphf_last_error": (C.c_char_p, []),
            "mphf_build_stream": (st, [C.POINTER(KeyStream), u64, C.c_double, u64, C.POINTER(Opts), u64, vp,
                                       C.POINTER(vp)]),
            "mphf_stream_keys": (st, [C.POINTER(KeyStream), u64, u64, vp, vp]),
            "mphf_build_host": (st, [vp, u64, C.c_double, u64, C.POINTER(Opts), u64, vp, C.POINTER(vp)]),
            "mphf_kmers": (st, [vp, u64, u32, vp, vp]),
            "mphf_first_occurrences": (st, [vp, u64, u64, vp, C.POINTER(C.c_uint64), vp]),
            "mphf_partition_sets": (st, [vp, u64, u32, u64, vp, vp, vp]),
            "mphf_set_ids": (st, [vp, u64, u32, u64, vp, vp]),
            "mphf_partition_sets_noalloc": (st, [vp, u64, u32, u64, vp, vp, vp]),
            "mphf_probe": (st, [u32, vp, u64, vp, u64, u64, vp]),
            "mphf_probe_ops": (u64, [u64]),
            "mphf_server_default_opts": (st, [C.POINTER(ServerOpts)]),
            "mphf_server_create": (st, [C.POINTER(ServerOpts), C.POINTER(vp)]),
            "mphf_server_register": (st, [vp, vp, C.POINTER(C.c_uint32)]),
            "mphf_server_submit": (st, [vp, u32, vp, u64, vp, C.POINTER(C.c_uint64)]),
            "mphf_server_poll": (st, [vp, u64, C.c_int, C.POINTER(RequestInfo)]),
            "mphf_server_get_stats": (st, [vp, C.POINTER(ServerStats)]),
            "mphf_server_destroy": (None, [vp]),
            "mphf_host_alloc": (st, [u64, C.POINTER(vp)]),
            "mphf_host_free": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        msg = lib().mphf_last_error().decode(errors="replace")
        cls = DuplicateKeysError if status == E_DUPLICATE_KEYS else MphfError
        raise cls(status, msg)


def _dev(t: torch.Tensor, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a tensor in GPU memory")
    if t.dtype not in (torch.int64, torch.uint64) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 64-bit integer tensor")
    return t.data_ptr()


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class _DeviceArray:
    """A device buffer owned by the library, seen by torch without a copy."""

    def __init__(self, ptr: int, n: int):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<i8", "data": (ptr, False),
                                         "version": 2, "strides": None}


class MPHF:
    """A built function; owns its device memory until close()."""

    def __init__(self, handle: int, keys_device: torch.device):
        self._h = handle
        self.device = keys_device

    @classmethod
    def build(cls, keys: torch.Tensor, gamma: float = 2.0, seed: int = 0, max_levels: int = 25,
              rank_sample: int = 512, mem_budget: int = 0, keep_collisions: bool = False,
              bucket_bits: int = 0, atomic_levels: bool = False, stream=None) -> "MPHF":
        L = lib()
        ptr = _dev(keys, "keys") if keys.numel() else (keys.data_ptr() if keys.is_cuda else 0)
        if not keys.is_cuda:
            raise ValueError("keys must be a tensor in GPU memory")
        o = Opts(max_levels, rank_sample, mem_budget, 1 if keep_collisions else 0, 1 if atomic_levels else 0)
        o.bucket_bits = bucket_bits
        h = C.c_void_p()
        with torch.cuda.device(keys.device):
            _check(L.mphf_build_ex(ptr, keys.numel(), float(gamma), seed & (2**64 - 1), C.byref(o),
                                   _stream(stream), C.byref(h)))
        return cls(h.value, keys.device)

    def lookup(self, queries: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(queries.numel(), dtype=torch.int64, device=queries.device)
        if queries.numel():
            _check(lib().mphf_lookup_ex(self._h, _dev(queries, "queries"), queries.numel(),
                                        _dev(out, "out"), _stream(stream)))
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(lib().mphf_stats(self._h, C.byref(s)))
        L = s.num_levels
        return {
            "n": s.n, "gamma": s.gamma, "seed": s.seed, "num_levels": L,
            "rank_sample": s.rank_sample,
            "level_n": list(s.level_n[:L]), "level_m": list(s.level_m[:L]),
            "level_weight": list(s.level_weight[:L]), "level_offset": list(s.level_offset[:L]),
            "level_seed": list(s.level_seed[:L]), "n_fallback": s.n_fallback,
            "total_bits": s.total_bits, "rank_entries": s.rank_entries,
            "structure_bytes": s.structure_bytes, "bits_per_key": s.bits_per_key,
            "peak_bytes": s.peak_bytes, "lookup_bytes": s.lookup_bytes,
            "level_path": [PATH_NAMES.get(v, str(v)) for v in s.level_path[:L]], "bucket_bits": s.bucket_bits,
        }

    def export(self) -> dict:
        """Host copies (numpy uint64) of the concatenated A, the rank table and H's keys."""
        st = self.stats()
        w = np.zeros(st["total_bits"] // 64, dtype=np.uint64)
        r = np.zeros(st["rank_entries"], dtype=np.uint64)
        f = np.zeros(st["n_fallback"], dtype=np.uint64)
        _check(lib().mphf_export(self._h, w.ctypes.data, len(w), r.ctypes.data, len(r),
                                 f.ctypes.data, len(f)))
        return {"words": w, "rank": r, "fallback_keys": f}

    def export_collisions(self, level: int) -> np.ndarray:
        m = self.stats()["level_m"][level]
        out = np.zeros((m + 63) // 64, dtype=np.uint64)
        _check(lib().mphf_export_collisions(self._h, level, out.ctypes.data, len(out)))
        return out

    def device_views(self) -> dict:
        """int64 torch views (no copy) of the device words, rank table and fallback keys."""
        v = View()
        _check(lib().mphf_view(self._h, C.byref(v)))
        res = {}
        for name, ptr, n in (("words", v.words, v.total_words), ("rank", v.rank, v.rank_entries),
                             ("fallback_keys", v.fallback_keys, v.n_fallback),
                             ("collisions", v.collisions, v.total_words if v.collisions else 0)):
            res[name] = (torch.as_tensor(_DeviceArray(ptr, n), device=self.device) if n
                         else torch.zeros(0, dtype=torch.int64, device=self.device))
        return res

    def close(self):
        if self._h:
            lib().mphf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent functions built in one launch (mphf_build_batch); owns its device memory."""

    def __init__(self, handle: int, device: torch.device):
        self._h = handle
        self.device = device

    @staticmethod
    def _opts(max_levels: int, launch) -> Opts:
        o = Opts(max_levels, 512, 0, 0, 0)
        if launch is not None:
            v = [int(x) for x in launch]
            if len(v) not in (3, 5):
                raise ValueError("launch: (threads, items, workgroups per CU[, small class, small every])")
            o.batch_threads, o.batch_items, o.batch_wgs_per_cu = v[:3]
            if len(v) == 5:
                o.batch_small_class, o.batch_small_every = v[3:]
        return o

    @classmethod
    def build(cls, keys: torch.Tensor, offsets: torch.Tensor, gamma: float = 2.0, seed: int = 0,
              max_levels: int = 25, stream=None, launch=None) -> "Batch":
        """One-shot batched build.  ``launch``: (threads, items, workgroups per CU[, small class,
        small every]), e.g. from :func:`paper_1702_03154_amd.autotune.batch_launch`; None = the
        library's default."""
        L = lib()
        o = cls._opts(max_levels, launch)
        h = C.c_void_p()
        kp = _dev(keys, "keys") if keys.numel() else keys.data_ptr()
        with torch.cuda.device(keys.device):
            _check(L.mphf_build_batch(kp, _dev(offsets, "offsets"), offsets.numel() - 1, float(gamma),
                                      seed & (2**64 - 1), C.byref(o), _stream(stream), C.byref(h)))
        return cls(h.value, keys.device)

    @classmethod
    def plan(cls, offsets: torch.Tensor, gamma: float = 2.0, seed: int = 0, max_levels: int = 25,
             stream=None, launch=None) -> "Batch":
        """A planned batch for these set sizes; fill it with :meth:`rebuild`."""
        L = lib()
        o = cls._opts(max_levels, launch)
        h = C.c_void_p()
        with torch.cuda.device(offsets.device):
            _check(L.mphf_batch_plan(_dev(offsets, "offsets"), offsets.numel() - 1, float(gamma),
                                     seed & (2**64 - 1), C.byref(o), _stream(stream), C.byref(h)))
        return cls(h.value, offsets.device)

    def rebuild(self, keys: torch.Tensor, stream=None) -> "Batch":
        """Enqueue the build of a planned batch (launches only; capturable in a graph)."""
        kp = _dev(keys, "keys") if keys.numel() else 0
        _check(lib().mphf_batch_rebuild(self._h, kp, _stream(stream)))
        return self

    def status(self, stream=None) -> "Batch":
        """Wait for the stream and raise if the last build of a planned batch failed."""
        _check(lib().mphf_batch_status(self._h, _stream(stream)))
        return self

    def export_sectors(self, s: int) -> np.ndarray:
        info = self.set_info(s)
        ns = (info["total_bits"] + 479) // 480
        out = np.zeros(ns * 16, dtype=np.uint32)
        _check(lib().mphf_batch_export_sectors(self._h, s, out.ctypes.data, ns))
        return out.reshape(ns, 16)

    def lookup(self, set_ids: torch.Tensor, queries: torch.Tensor, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(queries.numel(), dtype=torch.int64, device=queries.device)
        if queries.numel():
            _check(lib().mphf_batch_lookup(self._h, _dev(set_ids, "set_ids"), _dev(queries, "queries"),
                                           queries.numel(), _dev(out, "out"), _stream(stream)))
        return out

    def set_info(self, s: int) -> dict:
        i = SetInfo()
        _check(lib().mphf_batch_set_info(self._h, s, C.byref(i)))
        L = i.num_levels
        return {"n": i.n, "num_levels": L, "n_fallback": i.n_fallback,
                "level_n": list(i.level_n[:L]), "level_m": list(i.level_m[:L]),
                "level_offset": list(i.level_offset[:L]), "total_bits": i.total_bits}

    def export_set(self, s: int) -> dict:
        info = self.set_info(s)
        w = np.zeros(info["total_bits"] // 64, dtype=np.uint64)
        f = np.zeros(info["n_fallback"], dtype=np.uint64)
        _check(lib().mphf_batch_export_set(self._h, s, w.ctypes.data, len(w), f.ctypes.data, len(f)))
        return {"words": w, "fallback_keys": f}

    def totals(self) -> dict:
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        d = C.c_double()
        _check(lib().mphf_batch_totals(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return {"nsets": a.value, "nkeys": b.value, "total_bits": c.value, "bits_per_key": d.value}

    def close(self):
        if self._h:
            lib().mphf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_batch(keys: torch.Tensor, offsets: torch.Tensor, gamma: float = 2.0, seed: int = 0, **kw) -> Batch:
    return Batch.build(keys, offsets, gamma, seed, **kw)


def build(keys: torch.Tensor, gamma: float = 2.0, seed: int = 0, **kw) -> MPHF:
    return MPHF.build(keys, gamma, seed, **kw)


def positions(keys: torch.Tensor, level_seed: int, m: int, stream=None) -> torch.Tensor:
    """The device level-hash position of each key (the kernels' hash and exact mod)."""
    out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
    if keys.numel():
        _check(lib().mphf_positions(_dev(keys, "keys"), keys.numel(), level_seed & (2**64 - 1), m,
                                    _dev(out, "out"), _stream(stream)))
    return out


def build_stream(n: int, key_seed: int, gamma: float = 2.0, seed: int = 0, resident_keys: int = 1 << 31,
                 start: int = 0, max_levels: int = 25, rank_sample: int = 512, atomic_levels: bool = False,
                 device=None, stream=None) -> "MPHF":
    """Streaming build over keys generated on the fly (mphf_build_stream): key i is output start+i of
    the SplitMix64 stream of key_seed; no more than resident_keys survivors are ever stored."""
    L = lib()
    o = Opts(max_levels, rank_sample, 0, 0, 1 if atomic_levels else 0)
    src = KeyStream(key_seed & (2**64 - 1), start)
    h = C.c_void_p()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        _check(L.mphf_build_stream(C.byref(src), n, float(gamma), seed & (2**64 - 1), C.byref(o), resident_keys,
                                   _stream(stream), C.byref(h)))
    return MPHF(h.value, dev)


def build_host(keys, gamma: float = 2.0, seed: int = 0, resident_keys: int = 1 << 31, max_levels: int = 25,
               rank_sample: int = 512, atomic_levels: bool = False, device=None, stream=None) -> "MPHF":
    """Streaming build over keys stored in host memory (mphf_build_host): a numpy uint64/int64 array or
    a HostArray; every streamed level copies the keys to the device in chunks."""
    a = keys.a if isinstance(keys, HostArray) else keys
    if not isinstance(a, np.ndarray) or a.dtype.itemsize != 8 or not a.flags.c_contiguous:
        raise ValueError("keys must be a contiguous 64-bit host array")
    L = lib()
    o = Opts(max_levels, rank_sample, 0, 0, 1 if atomic_levels else 0)
    h = C.c_void_p()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        _check(L.mphf_build_host(a.ctypes.data if len(a) else 0, len(a), float(gamma), seed & (2**64 - 1),
                                 C.byref(o), resident_keys, _stream(stream), C.byref(h)))
    return MPHF(h.value, dev)


def stream_keys(key_seed: int, first: int, count: int, start: int = 0, device="cuda", stream=None) -> torch.Tensor:
    """Keys first .. first+count-1 of a streamed key set (mphf_stream_keys)."""
    out = torch.empty(count, dtype=torch.int64, device=device)
    src = KeyStream(key_seed & (2**64 - 1), start)
    if count:
        _check(lib().mphf_stream_keys(C.byref(src), first, count, _dev(out, "out"), _stream(stream)))
    return out


def trim() -> None:
    """Release the build workspaces the library caches per device (mphf_trim)."""
    _check(lib().mphf_trim())


# ---------------------------------------------------------------- k-mer keys

def kmers(seq: torch.Tensor, nbases: int, k: int = 31, stream=None) -> torch.Tensor:
    """Canonical k-mers at every position of a 2-bit packed sequence (mphf_kmers)."""
    n = max(0, nbases - k + 1)
    out = torch.empty(max(n, 1), dtype=torch.int64, device=seq.device)
    _check(lib().mphf_kmers(_dev(seq, "seq"), nbases, k, _dev(out, "out"), _stream(stream)))
    return out[:n]


def first_occurrences(keys: torch.Tensor, target: int, stream=None) -> torch.Tensor:
    """The first `target` distinct keys in order of first occurrence (mphf_first_occurrences)."""
    out = torch.empty(max(1, min(target, keys.numel())), dtype=torch.int64, device=keys.device)
    n = C.c_uint64()
    if keys.numel() and target:
        _check(lib().mphf_first_occurrences(_dev(keys, "keys"), keys.numel(), target, _dev(out, "out"),
                                            C.byref(n), _stream(stream)))
    return out[:n.value]


def partition_sets(keys: torch.Tensor, bits: int, seed: int = 0, stream=None):
    """Keys grouped into 2^bits hash sets and the set offsets (mphf_partition_sets)."""
    out = torch.empty_like(keys)
    off = torch.empty((1 << bits) + 1, dtype=torch.int64, device=keys.device)
    kp = _dev(keys, "keys") if keys.numel() else 0
    op = _dev(out, "out") if keys.numel() else 0
    _check(lib().mphf_partition_sets(kp, keys.numel(), bits, seed & (2**64 - 1), op, _dev(off, "offsets"),
                                     _stream(stream)))
    return out, off


def partition_sets_noalloc(keys: torch.Tensor, bits: int, seed: int = 0, out: torch.Tensor | None = None,
                           offsets: torch.Tensor | None = None, stream=None):
    """mphf_partition_sets_noalloc: the library allocates nothing (its scratch is a fixed device
    array); the caller's out and offsets tensors receive the result, asynchronously on the stream."""
    if out is None:
        out = torch.empty_like(keys)
    if offsets is None:
        offsets = torch.empty((1 << bits) + 1, dtype=torch.int64, device=keys.device)
    kp = _dev(keys, "keys") if keys.numel() else 0
    op = _dev(out, "out") if keys.numel() else 0
    _check(lib().mphf_partition_sets_noalloc(kp, keys.numel(), bits, seed & (2**64 - 1), op,
                                             _dev(offsets, "offsets"), _stream(stream)))
    return out, offsets


def set_ids(keys: torch.Tensor, bits: int, seed: int = 0, stream=None) -> torch.Tensor:
    out = torch.empty_like(keys)
    if keys.numel():
        _check(lib().mphf_set_ids(_dev(keys, "keys"), keys.numel(), bits, seed & (2**64 - 1), _dev(out, "out"),
                                  _stream(stream)))
    return out


# ---------------------------------------------------------------- roofline probes

PROBE_KINDS = {"stream_read": 0, "stream_copy": 1, "random_read8": 2, "random_sector64": 3,
               "random_atomic_or": 4, "lds_atomic_or": 5, "host_exchange": 6}


def probe(kind: str, buf: torch.Tensor | None = None, nbytes: int = 0, dst: torch.Tensor | None = None,
          ops: int = 0, seed: int = 1, stream=None) -> int:
    """Enqueue one roofline microbenchmark (mphf_probe) on the stream; returns the number of random
    operations it performs (0 for the streaming kinds)."""
    k = PROBE_KINDS[kind]
    bp = buf.data_ptr() if buf is not None else 0
    if buf is not None and (not buf.is_cuda or nbytes > buf.numel() * buf.element_size()):
        raise ValueError("buf must be a GPU tensor of at least nbytes")
    dp = dst.data_ptr() if dst is not None else 0
    if dst is not None and (not dst.is_cuda or nbytes > dst.numel() * dst.element_size()):
        raise ValueError("dst must be a GPU tensor of at least nbytes")
    _check(lib().mphf_probe(k, bp, nbytes, dp, ops, seed, _stream(stream)))
    return int(lib().mphf_probe_ops(ops)) if 2 <= k <= 5 else 0


def probe_host_exchange(src: "HostArray", dst: "HostArray", nbytes: int, stream=None) -> None:
    """Enqueue the PCIe probe (mphf_probe, MPHF_PROBE_HOST_EXCHANGE): a kernel reads nbytes of the
    pinned array src and writes them to the pinned array dst."""
    if nbytes > 8 * min(len(src.a), len(dst.a)):
        raise ValueError("src and dst must hold nbytes")
    _check(lib().mphf_probe(PROBE_KINDS["host_exchange"], src._p.value, nbytes, dst._p.value, 0, 0,
                            _stream(stream)))


# ---------------------------------------------------------------- serving

class HostArray:
    """Pinned host memory from mphf_host_alloc, seen as a numpy uint64 array (``.a``)."""

    def __init__(self, n: int):
        self._p = C.c_void_p()
        _check(lib().mphf_host_alloc(max(1, n) * 8, C.byref(self._p)))
        buf = (C.c_uint64 * max(1, n)).from_address(self._p.value)
        self.a = np.ctypeslib.as_array(buf)[:n]

    def close(self):
        if self._p:
            lib().mphf_host_free(self._p)
            self._p = None
            self.a = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Resident functions answering lookup requests from host memory, batched as they arrive
    (mphf_server_*).  Registered functions must stay alive while the server runs."""

    def __init__(self, hbm_budget: int = 1 << 30, max_inflight: int = 2, max_batch_requests: int = 1024):
        o = ServerOpts(int(hbm_budget), int(max_inflight), int(max_batch_requests))
        h = C.c_void_p()
        _check(lib().mphf_server_create(C.byref(o), C.byref(h)))
        self._h = h.value
        self._keep = {}      # ticket -> (keys, out): the arrays must outlive the request
        self._fns = []

    def register(self, f: "MPHF") -> int:
        i = C.c_uint32()
        _check(lib().mphf_server_register(self._h, f._h, C.byref(i)))
        self._fns.append(f)
        return i.value

    def submit(self, fn: int, keys: np.ndarray, out: np.ndarray) -> int:
        """Queue the labelling of ``keys`` (uint64/int64 host array) into ``out`` (same length)."""
        if keys.dtype.itemsize != 8 or out.dtype.itemsize != 8 or not keys.flags.c_contiguous \
                or not out.flags.c_contiguous or not out.flags.writeable or len(out) < len(keys):
            raise ValueError("keys and out must be contiguous 64-bit host arrays, out writable and as long")
        t = C.c_uint64()
        _check(lib().mphf_server_submit(self._h, fn, keys.ctypes.data, len(keys), out.ctypes.data,
                                        C.byref(t)))
        self._keep[t.value] = (keys, out)
        return t.value

    def poll(self, ticket: int, wait: bool = True) -> dict:
        info = RequestInfo()
        try:
            _check(lib().mphf_server_poll(self._h, ticket, 1 if wait else 0, C.byref(info)))
        finally:
            if info.done:
                self._keep.pop(ticket, None)
        return {"done": bool(info.done), "batch": info.batch, "batch_requests": info.batch_requests,
                "submit_us": info.submit_us, "start_us": info.start_us, "done_us": info.done_us}

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().mphf_server_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().mphf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
