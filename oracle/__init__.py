"""CPU oracle for the Hive hash table -- TEST INFRASTRUCTURE.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The library under paper_2510_15095_amd/ never does.

`O1` is the dictionary definition of the operations (Section III-D); `O2` is
the sequential model of the Hive table (Sections III and IV).  Both live in
hive_oracle.c, built by `python -m oracle.build` into libhive_oracle.so.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhive_oracle.so")

ADDR_FIXED = 0
ADDR_LINEAR = 1
EMPTY_WORD = 0xFFFFFFFFFFFFFFFF

_lib = None


def lib():
    """The built oracle library (compiled on first use if missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        _lib = bind(LIB_PATH)
    return _lib


def bind(path: str):
    """Load an oracle library from `path` and declare its signatures."""
    L = ctypes.CDLL(path)
    p, u64, i64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
    L.o1_create.argtypes = [u64]
    L.o1_create.restype = p
    L.o1_destroy.argtypes = [p]
    L.o1_apply.argtypes = [p, p, p, p, u64, p, p]
    L.o1_apply.restype = i32
    L.o1_size.argtypes = [p]
    L.o1_size.restype = u64
    L.o1_dump.argtypes = [p, p, u64]
    L.o1_dump.restype = u64
    L.o2_create.argtypes = [u32, u32, u64, i32, u64, u64, u64, u32, u32]
    L.o2_create.restype = p
    L.o2_destroy.argtypes = [p]
    L.o2_apply.argtypes = [p, p, p, p, u64, p, p]
    L.o2_apply.restype = i32
    L.o2_split.argtypes = [p, u64]
    L.o2_split.restype = i64
    L.o2_merge.argtypes = [p, u64]
    L.o2_merge.restype = i64
    L.o2_policy_pre.argtypes = [p, u64]
    L.o2_policy_pre.restype = i64
    L.o2_policy_post.argtypes = [p]
    L.o2_policy_post.restype = i64
    L.o2_stats.argtypes = [p, p]
    L.o2_kick_hist.argtypes = [p, p]
    L.o2_dump.argtypes = [p, p, p, u64]
    L.o2_dump.restype = u64
    L.o2_check.argtypes = [p, ctypes.c_char_p, i32]
    L.o2_check.restype = i32
    L.o2_bithash1.argtypes = [u32]
    L.o2_bithash1.restype = u32
    L.o2_bithash2.argtypes = [u32]
    L.o2_bithash2.restype = u32
    L.o2_bucket_of.argtypes = [p, u32]
    L.o2_bucket_of.restype = u64
    L.hs_crc32.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.hs_crc32.restype = u32
    L.hs_crc64.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.hs_crc64.restype = u64
    L.hs_murmur3.argtypes = [ctypes.c_char_p, ctypes.c_size_t, u32]
    L.hs_murmur3.restype = u32
    L.hs_city32_short.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.hs_city32_short.restype = u32
    L.hs_buckets.argtypes = [i32, p, u64, u64, p]
    L.hs_buckets.restype = i32
    return L


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _batch_args(ops, keys, vals):
    ops = np.ascontiguousarray(ops, dtype=np.uint8)
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    if vals is None:
        vals = np.zeros(keys.shape, np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    if not (ops.shape == keys.shape == vals.shape) or ops.ndim != 1:
        raise ValueError("ops, keys and vals must be 1-D arrays of one length")
    return ops, keys, vals


class _Model:
    _apply_name = ""
    _L = None

    @property
    def L(self):
        return self._L if self._L is not None else lib()

    def apply(self, ops, keys, vals=None):
        """Apply a batch in index order.  Returns (vals_out, flags_out):
        lookup -> value (0xFFFFFFFF if absent) and found; delete -> flag =
        was present (vals_out 0xFFFFFFFF); insert -> both untouched (value
        0xFFFFFFFF, flag 0)."""
        ops, keys, vals = _batch_args(ops, keys, vals)
        vout = np.full(keys.shape, 0xFFFFFFFF, np.uint32)
        fout = np.zeros(keys.shape, np.uint8)
        rc = getattr(self.L, self._apply_name)(self._h, _ptr(ops), _ptr(keys), _ptr(vals), keys.size,
                                              _ptr(vout), _ptr(fout))
        if rc != 0:
            raise RuntimeError(f"oracle apply failed ({rc})")
        return vout, fout

    def insert(self, keys, vals):
        self.apply(np.zeros(len(keys), np.uint8), keys, vals)

    def delete(self, keys):
        return self.apply(np.ones(len(keys), np.uint8), keys)[1]

    def lookup(self, keys):
        return self.apply(np.full(len(keys), 2, np.uint8), keys)


class O1(_Model):
    """Dictionary definition (Section III-D)."""
    _apply_name = "o1_apply"

    def __init__(self, expected: int = 1024, lib_handle=None):
        self._L = lib_handle
        self._h = self.L.o1_create(max(64, int(expected)))
        if not self._h:
            raise MemoryError("o1_create failed")

    def __del__(self):
        if getattr(self, "_h", None):
            self.L.o1_destroy(self._h)
            self._h = None

    def __len__(self):
        return int(self.L.o1_size(self._h))

    def dump(self) -> np.ndarray:
        """All entries as packed words (value << 32 | key), sorted by key."""
        n = len(self)
        out = np.empty(max(n, 1), np.uint64)
        self.L.o1_dump(self._h, _ptr(out), n)
        out = out[:n]
        return out[np.argsort(out & np.uint64(0xFFFFFFFF), kind="stable")]


STAT_NAMES = ("live", "n_buckets", "index_mask", "split_ptr", "stash_count", "pending_count",
              "evictions", "stash_inserts", "pending_inserts", "full_chains", "invalid_keys")


class O2(_Model):
    """Sequential model of the Hive table (Sections III and IV)."""
    _apply_name = "o2_apply"

    def __init__(self, slots_per_bucket=16, max_evictions=8, stash_capacity=1024, addressing=ADDR_FIXED,
                 n_buckets=1024, max_buckets=None, resize_k=64, lf_expand_pct=90, lf_contract_pct=25,
                 lib_handle=None):
        mb = n_buckets if max_buckets is None else max_buckets
        self.S = slots_per_bucket
        self._L = lib_handle
        self._h = self.L.o2_create(slots_per_bucket, max_evictions, stash_capacity, addressing, n_buckets, mb,
                                  resize_k, lf_expand_pct, lf_contract_pct)
        if not self._h:
            raise ValueError("o2_create rejected the configuration")

    def __del__(self):
        if getattr(self, "_h", None):
            self.L.o2_destroy(self._h)
            self._h = None

    def split(self, k: int) -> int:
        return int(self.L.o2_split(self._h, k))

    def merge(self, k: int) -> int:
        return int(self.L.o2_merge(self._h, k))

    def policy_pre(self, n_ins: int) -> int:
        return int(self.L.o2_policy_pre(self._h, n_ins))

    def policy_post(self) -> int:
        return int(self.L.o2_policy_post(self._h))

    def stats(self) -> dict:
        out = np.zeros(16, np.uint64)
        self.L.o2_stats(self._h, _ptr(out))
        return {k: int(out[i]) for i, k in enumerate(STAT_NAMES)}

    def kick_hist(self) -> np.ndarray:
        out = np.zeros(65, np.uint64)
        self.L.o2_kick_hist(self._h, _ptr(out))
        return out

    def dump(self, with_where: bool = False):
        n = int(self.L.o2_dump(self._h, None, None, 0))
        words = np.empty(max(n, 1), np.uint64)
        where = np.empty(max(n, 1), np.int64)
        self.L.o2_dump(self._h, _ptr(words), _ptr(where), n)
        words, where = words[:n], where[:n]
        order = np.argsort(words & np.uint64(0xFFFFFFFF), kind="stable")
        return (words[order], where[order]) if with_where else words[order]

    def check(self) -> None:
        buf = ctypes.create_string_buffer(256)
        rc = self.L.o2_check(self._h, buf, 256)
        if rc != 0:
            raise AssertionError(f"oracle invariant {rc}: {buf.value.decode()}")

    def bucket_of(self, mixed_hash: int) -> int:
        return int(self.L.o2_bucket_of(self._h, mixed_hash))

    def candidates(self, keys) -> tuple[np.ndarray, np.ndarray]:
        k = np.asarray(keys, dtype=np.uint32)
        c1 = np.array([self.bucket_of(int(self.L.o2_bithash1(int(x)))) for x in k], np.int64)
        c2 = np.array([self.bucket_of(int(self.L.o2_bithash2(int(x)))) for x in k], np.int64)
        return c1, c2


def bithash1(key: int) -> int:
    """Full 32-bit BitHash1 mix (Section III-C), before the bucket reduction."""
    return int(lib().o2_bithash1(key))


def bithash2(key: int) -> int:
    return int(lib().o2_bithash2(key))


# ---- hash-function study (Section III-C; plain transcriptions in hash_study.c)
HASH_KINDS = ("bithash1", "bithash2", "crc32", "crc64", "murmur3", "city32")


def crc32_bytes(data: bytes) -> int:
    return int(lib().hs_crc32(data, len(data)))


def crc64_bytes(data: bytes) -> int:
    return int(lib().hs_crc64(data, len(data)))


def murmur3_bytes(data: bytes, seed: int = 0) -> int:
    return int(lib().hs_murmur3(data, len(data), seed))


def city32_bytes(data: bytes) -> int:
    """CityHash32 of at most four bytes."""
    assert len(data) <= 4
    return int(lib().hs_city32_short(data, len(data)))


def hash_buckets(kind: str, keys, m: int) -> np.ndarray:
    """Bucket of every key: the hash of its four little-endian bytes mod m."""
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    out = np.empty(k.size, np.uint32)
    rc = lib().hs_buckets(HASH_KINDS.index(kind), _ptr(k), k.size, m, _ptr(out))
    if rc != 0:
        raise ValueError(f"bad hash kind or m: {kind}, {m}")
    return out


def collisions(buckets, m: int) -> int:
    """Y = sum over the m buckets of (load - 1)+, loads counted directly."""
    loads = np.bincount(np.asarray(buckets, dtype=np.int64), minlength=m)
    return int(np.maximum(loads - 1, 0).sum())


def expected_collisions(n: int, m: int) -> float:
    """E[Y] for n keys thrown independently and uniformly into m buckets
    (the uniform-hashing theorem of Section III-C): n - m (1 - (1 - 1/m)^n)."""
    if m == 1:
        return float(max(n - 1, 0))
    return float(n - m * -np.expm1(n * np.log1p(-1.0 / m)))

