"""Seeded synthetic workloads for the Hive hash table (arXiv 2510.15095).

This module is the ONLY code shared by the CPU oracle's tests and the HIP
path's tests and benchmark, and it holds none of the hash table's arithmetic:
no bucket hashing, no placement, no eviction.  It only produces operation
streams (keys, values, op codes) from seeds.

The paper evaluates on synthetic, uniformly distributed 32-bit key/value pairs
(Section V, first paragraph and V-C), up to about 32 M pairs.  The generator
here reproduces that shape and adds the Zipf(0.99) streams of the mixed and
served workloads.

Key streams
    key_s(i) = P_s(r(i)), where P_s is a seeded 4-round Feistel permutation of
    the 32-bit integers and r skips the two indices whose image would be a
    reserved key (0 or 0xFFFFFFFF).  key_s is a bijection from
    [0, 2^32 - 2) onto the valid keys, so distinct indices give distinct keys
    and a key's index is recovered in O(1) (`KeyStream.index_of`).

Values
    value(k) = low 32 bits of the first output of a SplitMix64 generator
    seeded with k (Steele, Lea and Flood, "Fast splittable pseudorandom number
    generators", OOPSLA 2014).

Zipf
    Ranks 1..N with P(k) proportional to k^-s, drawn by rejection-inversion
    (Hoermann and Derflinger, "Rejection-inversion to generate variates from
    monotone discrete distributions", ACM TOMACS 1996).  rank r -> key_s(r-1).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

M32 = 0xFFFFFFFF
M64 = 0xFFFFFFFFFFFFFFFF
EMPTY_KEY = 0xFFFFFFFF      # reserved key values: never generated
ZERO_KEY = 0

OP_INSERT = 0
OP_DELETE = 1
OP_LOOKUP = 2

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libworkload_gen.so")
_lib = None


def _native():
    """The compiled generator (csrc/workload_gen.c), or None if not built."""
    global _lib
    if _lib is None and os.path.exists(_LIB_PATH):
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.wl_keys.argtypes = [p, i64, i64, p, i64, p]
        lib.wl_keys_range.argtypes = [p, i64, i64, i64, i64, p]
        lib.wl_index_of.argtypes = [p, i64, i64, p, i64, p]
        lib.wl_values.argtypes = [p, i64, p]
        lib.wl_mixed_many.argtypes = [i64] + [p] * 14
        lib.wl_mixed_many.restype = ctypes.c_int
        lib.wl_domain_perm.argtypes = [p, i64, p, i64, p]
        lib.wl_domain_perm.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_SM_M1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_first(x) -> np.ndarray:
    """First output of SplitMix64 seeded with x (vectorised, uint64 wrap)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _SM_M1
        z = (z ^ (z >> np.uint64(27))) * _SM_M2
        return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed: int, n: int) -> np.ndarray:
    """n successive outputs of a SplitMix64 generator with state `seed`."""
    with np.errstate(over="ignore"):
        states = np.uint64(seed & M64) + _GOLDEN * np.arange(n, dtype=np.uint64)
    # output i mixes state_i + golden; splitmix64_first adds the golden ratio once
    return splitmix64_first(states)


def batch_seed(seed: int, batch: int) -> int:
    """Per-batch seed derived from a config seed and a batch number."""
    return int(splitmix64_first(np.uint64(((seed & M32) << 32) ^ (batch & M32))))


def values_for(keys, native: bool = True) -> np.ndarray:
    """value(k) = lo32(splitmix64(k))."""
    lib = _native() if native else None
    if lib is not None:
        k = np.ascontiguousarray(keys, dtype=np.uint32)
        out = np.empty(k.shape, np.uint32)
        lib.wl_values(_ptr(k), k.size, _ptr(out))
        return out
    return (splitmix64_first(np.asarray(keys, dtype=np.uint64)) & np.uint64(M32)).astype(np.uint32)


def _feistel_f(half: np.ndarray, rk: int) -> np.ndarray:
    with np.errstate(over="ignore"):
        x = (half.astype(np.uint64) * np.uint64(0x9E3779B1) + np.uint64(rk)) & np.uint64(M32)
        x ^= x >> np.uint64(15)
        x = (x * np.uint64(0x2C1B3C6D)) & np.uint64(M32)
        x ^= x >> np.uint64(12)
        return (x & np.uint64(0xFFFF)).astype(np.uint32)


class KeyStream:
    """Seeded bijection index -> valid 32-bit key (see module docstring)."""

    N_VALID = (1 << 32) - 2

    def __init__(self, seed: int, native: bool = True):
        self.seed = int(seed)
        rk = splitmix64_stream(self.seed, 4)
        self._rk = [int(r) & M32 for r in rk]
        self._rk_arr = np.array(self._rk, dtype=np.uint32)
        bad = self._perm_inv(np.array([0, M32], dtype=np.uint32)).astype(np.int64)
        self._a, self._b = int(bad.min()), int(bad.max())
        self._lib = _native() if native else None

    def _perm(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.uint32)
        left, right = x >> np.uint32(16), x & np.uint32(0xFFFF)
        for rk in self._rk:
            left, right = right, left ^ _feistel_f(right, rk)
        return (left << np.uint32(16)) | right

    def _perm_inv(self, y: np.ndarray) -> np.ndarray:
        y = np.asarray(y, dtype=np.uint32)
        left, right = y >> np.uint32(16), y & np.uint32(0xFFFF)
        for rk in reversed(self._rk):
            left, right = right ^ _feistel_f(left, rk), left
        return (left << np.uint32(16)) | right

    def keys(self, idx) -> np.ndarray:
        """key_s(i) for an array of indices in [0, 2^32 - 2)."""
        i = np.ascontiguousarray(idx, dtype=np.int64)
        if i.size and (i.min() < 0 or i.max() >= self.N_VALID):
            raise ValueError("key index out of range")
        if self._lib is not None:
            out = np.empty(i.shape, np.uint32)
            self._lib.wl_keys(_ptr(self._rk_arr), self._a, self._b, _ptr(i), i.size, _ptr(out))
            return out
        j = i + (i >= self._a) + (i >= self._b - 1)
        return self._perm(j.astype(np.uint32))

    def range(self, start: int, stop: int) -> np.ndarray:
        if start < 0 or stop > self.N_VALID or stop < start:
            raise ValueError("key index range out of bounds")
        if self._lib is not None:
            out = np.empty(stop - start, np.uint32)
            self._lib.wl_keys_range(_ptr(self._rk_arr), self._a, self._b, start, stop - start, _ptr(out))
            return out
        return self.keys(np.arange(start, stop, dtype=np.int64))

    def index_of(self, keys) -> np.ndarray:
        """Inverse of `keys`: the generator index of each (valid) key."""
        k = np.ascontiguousarray(keys, dtype=np.uint32)
        if self._lib is not None:
            out = np.empty(k.shape, np.int64)
            self._lib.wl_index_of(_ptr(self._rk_arr), self._a, self._b, _ptr(k), k.size, _ptr(out))
            if np.any(out < 0):
                raise ValueError("reserved key has no index")
            return out
        j = self._perm_inv(k).astype(np.int64)
        if np.any((j == self._a) | (j == self._b)):
            raise ValueError("reserved key has no index")
        return j - (j > self._a) - (j > self._b)


class Zipf:
    """Zipf(s) over ranks 1..N by rejection-inversion (Hoermann-Derflinger 1996).

    H(x) = (x^(1-s) - 1)/(1-s) is an antiderivative of h(x) = x^-s.  A uniform
    u on [H(1.5) - h(1), H(N + 0.5)] is inverted to x = H^-1(u); k = round(x)
    is accepted when u >= H(k + 0.5) - h(k).  Because h is convex, every
    accepted region has length exactly h(k), so P(k) is proportional to k^-s.
    """

    def __init__(self, n: int, s: float = 0.99):
        if n < 1 or not (0.0 < s) or s == 1.0:
            raise ValueError("need N >= 1 and s > 0, s != 1")
        self.n, self.s = int(n), float(s)
        self._q = 1.0 - self.s
        self._lo = self._H(1.5) - 1.0
        self._hi = self._H(self.n + 0.5)

    def _H(self, x):
        return np.expm1(self._q * np.log(x)) / self._q

    def _Hinv(self, y):
        return np.exp(np.log1p(self._q * y) / self._q)

    def pmf(self, k) -> np.ndarray:
        norm = np.sum(np.arange(1, self.n + 1, dtype=np.float64) ** -self.s)
        return np.asarray(k, dtype=np.float64) ** -self.s / norm

    def sample(self, rng: np.random.Generator, count: int) -> np.ndarray:
        out = np.empty(count, dtype=np.int64)
        todo = np.arange(count)
        while todo.size:
            u = self._lo + rng.random(todo.size) * (self._hi - self._lo)
            x = self._Hinv(u)
            k = np.clip(np.floor(x + 0.5), 1, self.n)
            ok = u >= self._H(k + 0.5) - k ** -self.s
            out[todo[ok]] = k[ok].astype(np.int64)
            todo = todo[~ok]
        return out


class DomainPerm:
    """Seeded permutation of [0, n): a 4-round Feistel network on 2h bits,
    2^(2h) >= n, restricted to [0, n) by cycle walking.  Used for sampling
    without replacement (the first m images) and for shuffles."""

    def __init__(self, seed: int, n: int):
        if n <= 0:
            raise ValueError("empty domain")
        self.n = int(n)
        self._rk = np.array([int(r) & M32 for r in splitmix64_stream(seed ^ 0x5EED, 4)], np.uint32)
        self._hb = 1
        while (1 << (2 * self._hb)) < self.n:
            self._hb += 1

    def _perm_np(self, x: np.ndarray) -> np.ndarray:
        mask = np.uint64((1 << self._hb) - 1)
        hb = np.uint64(self._hb)
        left, right = x >> hb, x & mask
        with np.errstate(over="ignore"):
            for rk in self._rk:
                f = (right * np.uint64(0x9E3779B97F4A7C15)) ^ np.uint64(rk)
                f ^= f >> np.uint64(29)
                f *= np.uint64(0xBF58476D1CE4E5B9)
                f ^= f >> np.uint64(32)
                left, right = right, left ^ (f & mask)
        return (left << hb) | right

    def __call__(self, pos, native: bool = True) -> np.ndarray:
        p = np.ascontiguousarray(pos, dtype=np.int64)
        if p.size and (p.min() < 0 or p.max() >= self.n):
            raise ValueError("position outside the permutation's domain")
        lib = _native() if native else None
        if lib is not None:
            out = np.empty(p.shape, np.int64)
            if lib.wl_domain_perm(_ptr(self._rk), self.n, _ptr(p), p.size, _ptr(out)) != 0:
                raise ValueError("domain permutation failed")
            return out
        x = p.astype(np.uint64)
        todo = np.ones(x.shape, bool)
        while todo.any():
            x[todo] = self._perm_np(x[todo])
            todo = x >= np.uint64(self.n)
        return x.astype(np.int64)

    def sample(self, m: int) -> np.ndarray:
        """m distinct values of [0, n) in pseudorandom order."""
        if m > self.n:
            raise ValueError("sample larger than the domain")
        return self(np.arange(m, dtype=np.int64))

    def shuffle(self, a: np.ndarray) -> np.ndarray:
        if len(a) != self.n:
            raise ValueError("shuffle length must equal the domain size")
        return a[self(np.arange(self.n, dtype=np.int64))]


# ---------------------------------------------------------------------------
# Workload recipes.  Each returns plain numpy arrays; nothing here touches a
# hash table.
# ---------------------------------------------------------------------------

def bulk_workload(seed: int, n_keys: int, n_queries: int | None = None,
                  n_deletes: int | None = None) -> dict:
    """Unique uniform inserts, 50%-hit queries, then deletes of a random half.

    * inserts: key_s(0..n_keys-1), value(k);
    * queries: n_queries/2 present keys (random inserted indices, without
      replacement) and n_queries/2 absent keys (indices >= n_keys, so they are
      guaranteed absent), shuffled;
    * deletes: n_deletes distinct inserted keys, random order.
    The re-query phase reuses the query array.
    """
    n_queries = n_keys if n_queries is None else n_queries
    n_deletes = n_keys // 2 if n_deletes is None else n_deletes
    if n_deletes > n_keys or n_queries // 2 > n_keys:
        raise ValueError("more present queries/deletes than keys")
    ks = KeyStream(seed)
    ins_keys = ks.range(0, n_keys)
    ins_vals = values_for(ins_keys)
    n_present = n_queries // 2
    n_absent = n_queries - n_present
    sub = batch_seed(seed, 0xC0FFEE)
    present_idx = DomainPerm(sub + 1, n_keys).sample(n_present) if n_present else np.empty(0, np.int64)
    # indices past the inserted range are never inserted: guaranteed misses
    absent_idx = n_keys + np.arange(n_absent, dtype=np.int64)
    q_idx = np.concatenate([present_idx, absent_idx]).astype(np.int64)
    if q_idx.size:
        q_idx = DomainPerm(sub + 2, q_idx.size).shuffle(q_idx)
    del_idx = DomainPerm(sub + 3, n_keys).sample(n_deletes) if n_deletes else np.empty(0, np.int64)
    return {
        "ins_keys": ins_keys,
        "ins_vals": ins_vals,
        "query_keys": ks.keys(q_idx),
        "query_idx": q_idx,
        "del_keys": ks.keys(del_idx),
        "del_idx": del_idx.astype(np.int64),
        "stream": ks,
    }


def tiny_workload(seed: int = 1) -> dict:
    """2^16 unique keys, 2^16 queries (50% present), delete a random half."""
    return bulk_workload(seed, 1 << 16)


def _mixed_counts(n_ops: int, frac_insert: float, frac_delete: float) -> tuple[int, int]:
    n_ins = int(round(n_ops * frac_insert))
    n_del = int(round(n_ops * frac_delete))
    if n_ins + n_del > n_ops:
        raise ValueError("op fractions exceed 1")
    return n_ins, n_del


def mixed_batches(jobs) -> list[dict]:
    """Many mixed batches at once (csrc/workload_gen.c, one thread per batch).

    `jobs` holds dicts of `mixed_batch`'s arguments.  Each batch's random
    numbers come from one SplitMix64 stream seeded with batch_seed(seed,
    batch), consumed in this order: a Fisher-Yates shuffle of the op codes
    (exact counts), one rank per op (Zipf(s) by rejection-inversion, or
    uniform over 1..universe when zipf_s is None), then the ranks that the
    per-type disjointness rule redraws (see `mixed_batch_reference`).  The
    results are views into shared arrays, one dict per job."""
    lib = _native()
    if lib is None:
        raise RuntimeError("the native generator (libworkload_gen.so) is not built")
    jobs = [dict(j) for j in jobs]
    count = len(jobs)
    n = np.array([int(j["n_ops"]) for j in jobs], np.int64)
    off = np.zeros(count, np.int64)
    if count:
        off[1:] = np.cumsum(n)[:-1]
    total = int(n.sum())
    seeds = np.empty(count, np.uint64)
    n_ins = np.empty(count, np.int64)
    n_del = np.empty(count, np.int64)
    uni = np.empty(count, np.int64)
    zs = np.empty(count, np.float64)
    rk = np.empty(4 * count, np.uint32)
    ab = np.empty(2 * count, np.int64)
    salt = np.empty(count, np.uint32)
    for c, j in enumerate(jobs):
        stream = j.get("stream") or KeyStream(j["seed"])
        seeds[c] = batch_seed(j["seed"], j["batch"])
        n_ins[c], n_del[c] = _mixed_counts(int(n[c]), j.get("frac_insert", 0.4), j.get("frac_delete", 0.4))
        uni[c] = int(j["universe"])
        if n_del[c] > uni[c] or uni[c] < 1 or uni[c] > KeyStream.N_VALID:
            raise ValueError("the universe must hold the batch's distinct delete keys and fit the key stream")
        z = j.get("zipf_s", 0.99)
        if z is not None and (z <= 0 or z == 1.0):
            raise ValueError("need zipf_s > 0, != 1 (or None for uniform)")
        zs[c] = -1.0 if z is None else float(z)
        rk[4 * c:4 * c + 4] = stream._rk_arr
        ab[2 * c], ab[2 * c + 1] = stream._a, stream._b
        salt[c] = int(j.get("value_salt", 0)) & M32
    ops = np.empty(total, np.uint8)
    keys = np.empty(total, np.uint32)
    vals = np.empty(total, np.uint32)
    ranks = np.empty(total, np.int64)
    if count:
        rc = lib.wl_mixed_many(count, _ptr(seeds), _ptr(n), _ptr(off), _ptr(n_ins), _ptr(n_del), _ptr(uni),
                               _ptr(zs), _ptr(rk), _ptr(ab), _ptr(salt), _ptr(ops), _ptr(keys), _ptr(vals),
                               _ptr(ranks))
        if rc == -1:
            raise RuntimeError("mixed batch: key universe too small for per-type disjoint keys")
        if rc != 0:
            raise MemoryError("mixed batch generator could not allocate")
    out = []
    for c in range(count):
        sl = slice(int(off[c]), int(off[c] + n[c]))
        out.append({"ops": ops[sl], "keys": keys[sl], "vals": vals[sl], "ranks": ranks[sl]})
    return out


def mixed_batch(seed: int, batch: int, n_ops: int, universe: int,
                frac_insert: float = 0.4, frac_delete: float = 0.4,
                zipf_s: float | None = 0.99, stream: KeyStream | None = None,
                value_salt: int = 0) -> dict:
    """One mixed batch with exact op counts and per-type disjoint key sets.

    Op types are laid out with exact counts and shuffled; each op then draws a
    rank (Zipf(s) over `universe`, or uniform when zipf_s is None).  A key is
    owned by the type of its first occurrence in index order; an op whose key
    is owned by another type, or a repeated delete of one key, redraws.
    Inserts may repeat a key (last occurrence wins); lookups may repeat.
    value_salt != 0 makes insert values differ from value(k) (replace tests).
    """
    return mixed_batches([dict(seed=seed, batch=batch, n_ops=n_ops, universe=universe, frac_insert=frac_insert,
                               frac_delete=frac_delete, zipf_s=zipf_s, stream=stream, value_salt=value_salt)])[0]


def mixed_batch_reference(seed: int, batch: int, n_ops: int, universe: int,
                          frac_insert: float = 0.4, frac_delete: float = 0.4,
                          zipf_s: float | None = 0.99, stream: KeyStream | None = None,
                          value_salt: int = 0) -> dict:
    """Pure-Python statement of `mixed_batch` (small batches only): the same
    SplitMix64 stream, shuffle, rank draws and disjointness rule, written
    with Python integers and the math module."""
    import math
    stream = stream or KeyStream(seed, native=False)
    state = [batch_seed(seed, batch)]

    def nxt() -> int:
        state[0] = (state[0] + 0x9E3779B97F4A7C15) & M64
        z = state[0]
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)

    def below(m: int) -> int:
        return (nxt() * m) >> 64

    if zipf_s is not None:
        q = 1.0 - zipf_s
        H = lambda x: math.expm1(q * math.log(x)) / q  # noqa: E731
        Hinv = lambda y: math.exp(math.log1p(q * y) / q)  # noqa: E731
        lo, hi = H(1.5) - 1.0, H(universe + 0.5)

    def rank() -> int:
        if zipf_s is None:
            return 1 + below(universe)
        while True:
            u = lo + ((nxt() >> 11) * 2.0 ** -53) * (hi - lo)
            k = min(max(math.floor(Hinv(u) + 0.5), 1), universe)
            if u >= H(k + 0.5) - math.pow(k, -zipf_s):
                return k

    n_ins, n_del = _mixed_counts(n_ops, frac_insert, frac_delete)
    ops = [OP_INSERT] * n_ins + [OP_DELETE] * n_del + [OP_LOOKUP] * (n_ops - n_ins - n_del)
    for i in range(n_ops - 1, 0, -1):
        j = below(i + 1)
        ops[i], ops[j] = ops[j], ops[i]
    ranks = [rank() for _ in range(n_ops)]
    owner: dict[int, int] = {}
    for i, t in enumerate(ops):
        r = ranks[i]
        while True:
            o = owner.get(r)
            if o is None:
                owner[r] = t
                break
            if o == t and t != OP_DELETE:
                break
            r = rank()
        ranks[i] = r
    ranks = np.array(ranks, np.int64)
    keys = stream.keys(ranks - 1)
    vals = values_for(keys, native=False) ^ np.uint32(value_salt & M32)
    return {"ops": np.array(ops, np.uint8), "keys": keys, "vals": vals.astype(np.uint32), "ranks": ranks}
