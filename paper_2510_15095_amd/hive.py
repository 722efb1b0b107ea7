"""Python binding of the C ABI in include/hive.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
work of its own beyond checking tensors and passing pointers: all table work
runs in the HIP kernels of libhive.so.  Device buffers are torch tensors on
the GPU; streams are torch streams (the current stream by default).

The library must have been built (`python -m paper_2510_15095_amd.build`);
importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhive.so")

HIVE_OK = 0
HIVE_ERR_ARG = -1
HIVE_ERR_OOM = -2
HIVE_ERR_HIP = -3
HIVE_ERR_BUDGET = -4
HIVE_ERR_LOST = -5
HIVE_WARN_INVALID_KEYS = 1
HIVE_WARN_PENDING = 2

HIVE_FIXED = 0
HIVE_LINEAR = 1
HIVE_UNIQUE = 1
HIVE_OP_INSERT, HIVE_OP_DELETE, HIVE_OP_LOOKUP, HIVE_OP_MIXED = 0, 1, 2, 3


class hive_config(ctypes.Structure):
    _fields_ = [
        ("slots_per_bucket", ctypes.c_uint32),
        ("max_evictions", ctypes.c_uint32),
        ("stash_capacity", ctypes.c_uint64),
        ("pending_capacity", ctypes.c_uint64),
        ("addressing", ctypes.c_uint32),
        ("resize_k", ctypes.c_uint32),
        ("lf_expand_pct", ctypes.c_uint32),
        ("lf_contract_pct", ctypes.c_uint32),
        ("pre_expand", ctypes.c_uint32),
        ("post_policy", ctypes.c_uint32),
        ("max_buckets", ctypes.c_uint64),
        ("max_batch", ctypes.c_uint64),
        ("probe_both", ctypes.c_uint32),
        ("hash_pair", ctypes.c_uint32),
        ("entry_bits", ctypes.c_uint32),
        ("probe_tuning", ctypes.c_uint32),
        ("probe_grid", ctypes.c_uint32),
    ]


class hive_stats_t(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "live", "n_buckets", "index_mask", "split_ptr", "stash_count", "pending_count", "evictions",
        "stash_inserts", "pending_inserts", "full_chains", "invalid_keys", "evict_items", "bytes_reserved",
        "slots_per_bucket", "max_buckets", "error_bits")]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class hive_batch_desc(ctypes.Structure):
    _fields_ = [
        ("op_mode", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("d_ops", ctypes.c_void_p),
        ("d_keys", ctypes.c_void_p),
        ("d_vals", ctypes.c_void_p),
        ("d_vals_out", ctypes.c_void_p),
        ("d_flags_out", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
    ]


class HiveError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.hive_status_string(status).decode() if _lib else str(status)
        super().__init__(f"{where}: {msg} ({status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_15095_amd.build`")
    # torch ships its own HIP and HSA runtimes.  Loaded first, they also
    # satisfy libhive.so's dependencies, so the process has one runtime;
    # loaded after libhive.so (which links the system ROCm copies), the
    # process holds two, and the one initialised second finds no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    p, u64, u32, i64, st = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int
    sig = {
        "hive_config_default": ([ctypes.POINTER(hive_config)], st),
        "hive_create": ([ctypes.POINTER(hive_config), u64, p, ctypes.POINTER(p)], st),
        "hive_destroy": ([p], st),
        "hive_insert_batch": ([p, p, p, u64, u32, p], st),
        "hive_lookup_batch": ([p, p, u64, p, p, p], st),
        "hive_delete_batch": ([p, p, u64, u32, p, p], st),
        "hive_mixed_batch": ([p, p, p, p, u64, u32, p, p, p], st),
        "hive_mixed_batch_noalloc": ([p, p, p, p, u64, u32, p, p, p], st),
        "hive_resize": ([p, i64, p], st),
        "hive_stats": ([p, ctypes.POINTER(hive_stats_t), p], st),
        "hive_dump": ([p, p, p, u64, ctypes.POINTER(u64), p], st),
        "hive_clear": ([p, p], st),
        "hive_placement": ([p, ctypes.POINTER(u64), p], st),
        "hive_live_async": ([p, p, p], st),
        "hive_status_string": ([st], ctypes.c_char_p),
        "hive_bithash1": ([u32], u32),
        "hive_bithash2": ([u32], u32),
        "hive_bucket_of": ([p, u32, ctypes.POINTER(u64)], st),
        "hive_fastmod_magic": ([u32], u64),
        "hive_fastmod": ([u32, u64, u32], u32),
        "hive_drain_create": ([u32, u32, u64, u32, u64, ctypes.POINTER(p)], st),
        "hive_drain_submit": ([p, p, ctypes.POINTER(hive_batch_desc), ctypes.POINTER(u64)], st),
        "hive_drain_launch": ([p, st, p], st),
        "hive_drain_poll": ([p, u64, ctypes.POINTER(st)], st),
        "hive_drain_result": ([p, u64, ctypes.POINTER(st), ctypes.POINTER(u64)], st),
        "hive_drain_results": ([p, p, u64, p, p], st),
        "hive_phase_timing": ([p, st], st),
        "hive_hash_buckets": ([u32, p, u64, u64, p, p], st),
        "hive_gather_lines": ([p, u64, p, u64, p, p], st),
        "hive_hash_collisions": ([u32, p, u64, u64, p, p, p], st),
        "hive_phase_times": ([p, p], st),
        "hive_drain_stop": ([p, p], st),
        "hive_drain_destroy": ([p], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib = _load()
lib = _lib


# ---------------------------------------------------------------- marshalling
def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name, n=None, optional=False):
    import torch
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {n}")
    return ctypes.c_void_p(t.data_ptr())


def _check(status: int, where: str, warn_ok: bool = False) -> int:
    if status < 0 or (status > 0 and not warn_ok):
        raise HiveError(status, where)
    return status


# probe-kernel variants (hive_config.probe_tuning): (waves per SIMD, loads in
# flight) per variant index; inserts take the ones in PROBE_INSERT_VARIANTS
PROBE_VARIANTS = ((4, 16), (6, 16), (8, 8), (6, 8), (8, 4))
PROBE_INSERT_VARIANTS = (0, 3, 4)
PROBE_KINDS = ("insert", "delete", "lookup", "mixed")


def probe_tuning(insert: int = 0, delete: int = 0, lookup: int = 0, mixed: int = 0) -> int:
    """Pack one probe-kernel variant per operation kind into the
    hive_config.probe_tuning word."""
    return insert | delete << 4 | lookup << 8 | mixed << 12


# ----------------------------------------------------------- C ABI mirrors
def hive_config_default(**overrides) -> hive_config:
    cfg = hive_config()
    _check(_lib.hive_config_default(ctypes.byref(cfg)), "hive_config_default")
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise AttributeError(f"hive_config has no field {k!r}")
        setattr(cfg, k, v)
    return cfg


def hive_create(cfg: hive_config, initial_buckets: int, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(_lib.hive_create(ctypes.byref(cfg), initial_buckets, _stream_ptr(stream), ctypes.byref(h)),
           "hive_create")
    return h


def hive_destroy(h) -> None:
    _check(_lib.hive_destroy(h), "hive_destroy")


def hive_insert_batch(h, keys, vals, flags: int = 0, stream=None) -> None:
    import torch
    n = keys.numel()
    _check(_lib.hive_insert_batch(h, _dev(keys, torch.uint32, "keys"),
                                  _dev(vals, torch.uint32, "vals", n, optional=True), n, flags,
                                  _stream_ptr(stream)), "hive_insert_batch")


def hive_lookup_batch(h, keys, vals_out=None, found_out=None, stream=None) -> None:
    import torch
    n = keys.numel()
    _check(_lib.hive_lookup_batch(h, _dev(keys, torch.uint32, "keys"), n,
                                  _dev(vals_out, torch.uint32, "vals_out", n, optional=True),
                                  _dev(found_out, torch.uint8, "found_out", n, optional=True),
                                  _stream_ptr(stream)), "hive_lookup_batch")


def hive_delete_batch(h, keys, deleted_out=None, flags: int = 0, stream=None) -> None:
    import torch
    n = keys.numel()
    _check(_lib.hive_delete_batch(h, _dev(keys, torch.uint32, "keys"), n, flags,
                                  _dev(deleted_out, torch.uint8, "deleted_out", n, optional=True),
                                  _stream_ptr(stream)), "hive_delete_batch")


def hive_mixed_batch(h, ops, keys, vals, vals_out=None, flags_out=None, flags: int = 0, stream=None) -> None:
    import torch
    n = keys.numel()
    _check(_lib.hive_mixed_batch(h, _dev(ops, torch.uint8, "ops", n), _dev(keys, torch.uint32, "keys"),
                                 _dev(vals, torch.uint32, "vals", n, optional=True), n, flags,
                                 _dev(vals_out, torch.uint32, "vals_out", n, optional=True),
                                 _dev(flags_out, torch.uint8, "flags_out", n, optional=True),
                                 _stream_ptr(stream)), "hive_mixed_batch")


def hive_mixed_batch_noalloc(h, ops, keys, vals, vals_out=None, flags_out=None, flags: int = 0,
                             stream=None) -> None:
    import torch
    n = keys.numel()
    _check(_lib.hive_mixed_batch_noalloc(h, _dev(ops, torch.uint8, "ops", n), _dev(keys, torch.uint32, "keys"),
                                         _dev(vals, torch.uint32, "vals", n), n, flags,
                                         _dev(vals_out, torch.uint32, "vals_out", n, optional=True),
                                         _dev(flags_out, torch.uint8, "flags_out", n, optional=True),
                                         _stream_ptr(stream)), "hive_mixed_batch_noalloc")


def hive_resize(h, delta: int, stream=None) -> None:
    _check(_lib.hive_resize(h, delta, _stream_ptr(stream)), "hive_resize")


def hive_stats(h, stream=None) -> tuple[int, dict]:
    out = hive_stats_t()
    status = _check(_lib.hive_stats(h, ctypes.byref(out), _stream_ptr(stream)), "hive_stats", warn_ok=True)
    return status, out.as_dict()


def hive_dump(h, words_out, where_out=None, stream=None) -> int:
    import torch
    n = ctypes.c_uint64()
    _check(_lib.hive_dump(h, _dev(words_out, torch.uint64, "words_out"),
                          _dev(where_out, torch.int64, "where_out", words_out.numel(), optional=True),
                          words_out.numel(), ctypes.byref(n), _stream_ptr(stream)), "hive_dump")
    return int(n.value)


def hive_placement(h, stream=None) -> tuple[int, int, int]:
    out = (ctypes.c_uint64 * 3)()
    _check(_lib.hive_placement(h, out, _stream_ptr(stream)), "hive_placement")
    return int(out[0]), int(out[1]), int(out[2])


def hive_live_async(h, host_dst_ptr: int, stream=None) -> None:
    """host_dst_ptr: address of 8 bytes of pinned host memory."""
    _check(_lib.hive_live_async(h, ctypes.c_void_p(host_dst_ptr), _stream_ptr(stream)), "hive_live_async")


def hive_clear(h, stream=None) -> None:
    _check(_lib.hive_clear(h, _stream_ptr(stream)), "hive_clear")


def hive_status_string(status: int) -> str:
    return _lib.hive_status_string(status).decode()


def hive_bithash1(key: int) -> int:
    return int(_lib.hive_bithash1(key))


def hive_bithash2(key: int) -> int:
    return int(_lib.hive_bithash2(key))


def hive_bucket_of(h, mixed_hash: int) -> int:
    b = ctypes.c_uint64()
    _check(_lib.hive_bucket_of(h, mixed_hash, ctypes.byref(b)), "hive_bucket_of")
    return int(b.value)


def hive_fastmod_magic(d: int) -> int:
    return int(_lib.hive_fastmod_magic(d))


def hive_fastmod(a: int, magic: int, d: int) -> int:
    return int(_lib.hive_fastmod(a, magic, d))


def hive_drain_create(slots_per_bucket: int = 16, blocks_per_cu: int = 0, ring_capacity: int = 1024,
                      max_tables: int = 64, idle_timeout_us: int = 0) -> ctypes.c_void_p:
    d = ctypes.c_void_p()
    _check(_lib.hive_drain_create(slots_per_bucket, blocks_per_cu, ring_capacity, max_tables, idle_timeout_us,
                                  ctypes.byref(d)), "hive_drain_create")
    return d


def hive_drain_submit(d, h, op_mode, keys, vals=None, ops=None, vals_out=None, flags_out=None,
                      flags: int = 0) -> int | None:
    """Queue one batch; returns its ticket, or None when the ring is full."""
    import torch
    n = keys.numel()
    b = hive_batch_desc()
    b.op_mode = op_mode
    b.flags = flags
    b.d_ops = _dev(ops, torch.uint8, "ops", n, optional=True)
    b.d_keys = _dev(keys, torch.uint32, "keys")
    b.d_vals = _dev(vals, torch.uint32, "vals", n, optional=True)
    b.d_vals_out = _dev(vals_out, torch.uint32, "vals_out", n, optional=True)
    b.d_flags_out = _dev(flags_out, torch.uint8, "flags_out", n, optional=True)
    b.n = n
    t = ctypes.c_uint64()
    status = _lib.hive_drain_submit(d, h, ctypes.byref(b), ctypes.byref(t))
    if status == HIVE_ERR_BUDGET:
        return None
    _check(status, "hive_drain_submit")
    return int(t.value)


def hive_drain_launch(d, resident: int = 0, stream=None) -> None:
    _check(_lib.hive_drain_launch(d, resident, _stream_ptr(stream)), "hive_drain_launch")


def hive_drain_poll(d, ticket: int) -> bool:
    done = ctypes.c_int()
    _check(_lib.hive_drain_poll(d, ticket, ctypes.byref(done)), "hive_drain_poll")
    return bool(done.value)


def hive_drain_result(d, ticket: int) -> tuple[bool, int]:
    done, live = ctypes.c_int(), ctypes.c_uint64()
    _check(_lib.hive_drain_result(d, ticket, ctypes.byref(done), ctypes.byref(live)), "hive_drain_result")
    return bool(done.value), int(live.value)


def hive_drain_results(d, tickets):
    """(done, live_after) numpy arrays for an array of tickets, in one call."""
    import numpy as np
    t = np.ascontiguousarray(tickets, dtype=np.uint64)
    done = np.zeros(t.size, dtype=np.uint8)
    live = np.zeros(t.size, dtype=np.uint64)
    _check(_lib.hive_drain_results(d, t.ctypes.data, t.size, done.ctypes.data, live.ctypes.data),
           "hive_drain_results")
    return done.astype(bool), live


HIVE_PAIR_BITHASH, HIVE_PAIR_CRC, HIVE_PAIR_MURMUR, HIVE_PAIR_TRIPLE = 0, 1, 2, 3
HASH_KINDS = ("bithash1", "bithash2", "crc32", "crc64", "murmur3", "city32")
HIVE_HASH_KINDS = len(HASH_KINDS)


def hive_hash_buckets(kind: str, keys, m: int, out, stream=None) -> None:
    """out[i] = bucket of keys[i] under hash `kind` (uint32 GPU tensors)."""
    import torch
    n = keys.numel()
    _check(_lib.hive_hash_buckets(HASH_KINDS.index(kind), _dev(keys, torch.uint32, "keys"), n, m,
                                  _dev(out, torch.uint32, "out", n), _stream_ptr(stream)), "hive_hash_buckets")


def hive_hash_collisions(kind: str, keys, m: int, scratch, stream=None) -> int:
    """Collision count Y of `keys` over m buckets; scratch: uint32 GPU tensor
    of at least 2 + ceil(m / 32) words."""
    import torch
    y = ctypes.c_uint64()
    _check(_lib.hive_hash_collisions(HASH_KINDS.index(kind), _dev(keys, torch.uint32, "keys"), keys.numel(), m,
                                     _dev(scratch, torch.uint32, "scratch", 2 + (m + 31) // 32),
                                     ctypes.byref(y), _stream_ptr(stream)), "hive_hash_collisions")
    return int(y.value)


def hive_gather_lines(table, idx, out, stream=None) -> None:
    """out[i] = XOR of the 16 words of line idx[i] of table (uint64 GPU tensor
    of n_lines x 16 words; idx uint32, out uint64 GPU tensors)."""
    import torch
    n = idx.numel()
    _check(_lib.hive_gather_lines(_dev(table, torch.uint64, "table"), table.numel() // 16,
                                  _dev(idx, torch.uint32, "idx"), n, _dev(out, torch.uint64, "out", n),
                                  _stream_ptr(stream)), "hive_gather_lines")


PHASE_KINDS = ("dedupe", "probe", "evict", "resize", "drain", "finish", "stash")


def hive_phase_timing(h, enable: bool) -> None:
    _check(_lib.hive_phase_timing(h, int(bool(enable))), "hive_phase_timing")


def hive_phase_times(h) -> dict:
    """Milliseconds per phase group since the previous call (then reset)."""
    out = (ctypes.c_double * len(PHASE_KINDS))()
    _check(_lib.hive_phase_times(h, out), "hive_phase_times")
    return {k: float(out[i]) for i, k in enumerate(PHASE_KINDS)}


def hive_drain_stop(d, stream=None) -> None:
    _check(_lib.hive_drain_stop(d, _stream_ptr(stream)), "hive_drain_stop")


def hive_drain_destroy(d) -> None:
    _check(_lib.hive_drain_destroy(d), "hive_drain_destroy")


# ------------------------------------------------------------ convenience
class Table:
    """Owning handle around hive_create/hive_destroy with the batch calls."""

    def __init__(self, initial_buckets: int, stream=None, **cfg):
        self.cfg = hive_config_default(**cfg)
        self.h = hive_create(self.cfg, initial_buckets, stream)
        self.stream = stream

    def close(self):
        if getattr(self, "h", None):
            hive_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, keys, vals, flags=0):
        hive_insert_batch(self.h, keys, vals, flags, self.stream)

    def lookup(self, keys):
        import torch
        v = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
        f = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        hive_lookup_batch(self.h, keys, v, f, self.stream)
        return v, f

    def delete(self, keys, flags=0):
        import torch
        d = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        hive_delete_batch(self.h, keys, d, flags, self.stream)
        return d

    def mixed(self, ops, keys, vals, flags=0):
        import torch
        v = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
        f = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        hive_mixed_batch(self.h, ops, keys, vals, v, f, flags, self.stream)
        return v, f

    def resize(self, delta: int):
        hive_resize(self.h, delta, self.stream)

    def stats(self) -> dict:
        status, d = hive_stats(self.h, self.stream)
        d["status"] = status
        return d

    def dump(self, with_where=False):
        """All live words, sorted by key, as host numpy arrays."""
        import numpy as np
        import torch
        st = self.stats()
        cap = st["live"] + st["stash_count"] + st["pending_count"] + 1
        words = torch.empty(cap, dtype=torch.uint64, device="cuda")
        where = torch.empty(cap, dtype=torch.int64, device="cuda") if with_where else None
        n = hive_dump(self.h, words, where, self.stream)
        if n > cap:
            raise RuntimeError("dump capacity too small")
        w = words[:n].cpu().numpy()
        order = np.argsort(w & np.uint64(0xFFFFFFFF), kind="stable")
        if with_where:
            return w[order], where[:n].cpu().numpy()[order]
        return w[order]

    def clear(self):
        hive_clear(self.h, self.stream)

    def placement(self) -> tuple[int, int, int]:
        return hive_placement(self.h, self.stream)
