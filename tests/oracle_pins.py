"""Pins for the CPU oracle, written as functions of an oracle library handle.

Each pin checks the oracle against something other than itself: Python's own
dict (the definition of a dictionary), inverses of the hash maps derived from
their algebra, hand-traced scenarios of the paper's algorithms, closed forms,
invariants, and special cases that reduce to plain modulo addressing.
`tests/test_oracle.py` runs them on the built oracle; `tests/test_oracle_mutants.py`
runs them on copies of the oracle with planted mistakes and requires that
some pin fails for every mistake.
"""
from __future__ import annotations

import random

import numpy as np

import oracle
from oracle import ADDR_FIXED, ADDR_LINEAR, O1, O2

M32 = 0xFFFFFFFF


# ---------------------------------------------------------------- O1 vs dict
def pin_o1_matches_python_dict(L, seed=0, n_ops=6000):
    rng = random.Random(seed)
    d = O1(64, lib_handle=L)
    ref: dict[int, int] = {}
    universe = [rng.randrange(1, M32) for _ in range(300)] + [0, M32]
    ops, keys, vals = [], [], []
    for _ in range(n_ops):
        ops.append(rng.choice([0, 0, 1, 2, 2]))
        keys.append(rng.choice(universe))
        vals.append(rng.getrandbits(32))
    vout, fout = d.apply(np.array(ops, np.uint8), np.array(keys, np.uint32), np.array(vals, np.uint32))
    for i, (o, k, v) in enumerate(zip(ops, keys, vals)):
        valid = k not in (0, M32)
        if o == 0:
            if valid:
                ref[k] = v
        elif o == 1:
            exp = valid and k in ref
            assert fout[i] == exp, f"delete flag at op {i}"
            if exp:
                del ref[k]
        else:
            exp = ref.get(k) if valid else None
            assert fout[i] == (exp is not None), f"lookup found at op {i}"
            assert vout[i] == (M32 if exp is None else exp), f"lookup value at op {i}"
    assert len(d) == len(ref)
    dump = d.dump()
    assert [int(w) & M32 for w in dump] == sorted(ref)
    assert all(int(w) >> 32 == ref[int(w) & M32] for w in dump)


# ------------------------------------------------------------ hash inverses
def _mul_inverse(a):
    inv = a  # correct to 3 bits for odd a; Newton doubles the precision
    for _ in range(5):
        inv = (inv * (2 - a * inv)) & M32
    assert (a * inv) & M32 == 1
    return inv


def _inv_affine(y, a, c):
    return (_mul_inverse(a) * ((y - c) & M32)) & M32


def _inv_xorshr(y, s, c):
    z = y ^ c
    x, sh = z, s
    while sh < 32:
        x ^= z >> sh
        sh += s
    return x


def _inv_tfunction(y, f):
    """Invert a map whose output bit i depends only on input bits 0..i."""
    x = 0
    for i in range(32):
        if (f(x) ^ y) >> i & 1:
            x |= 1 << i
    return x


def bithash1_inverse(y):
    # BitHash1 (Section III-C) as maps: (2^15-1)x - 1; x^(x>>12); 5x;
    # x^(x>>4); 2057x; x^(x>>16).  Undo them in reverse order.
    x = _inv_xorshr(y, 16, 0)
    x = _inv_affine(x, 2057, 0)
    x = _inv_xorshr(x, 4, 0)
    x = _inv_affine(x, 5, 0)
    x = _inv_xorshr(x, 12, 0)
    return _inv_affine(x, (1 << 15) - 1, M32)


def bithash2_inverse(y):
    # BitHash2 (Section III-C): (x + c1) + (x << 12); (x ^ c2) ^ (x >> 19);
    # (x + c3) + (x << 5); (x + c4) ^ (x << 9); (x + c5) + (x << 3);
    # (x ^ c6) ^ (x >> 16).
    x = _inv_xorshr(y, 16, 0xB55A4F09)
    x = _inv_affine(x, 1 + (1 << 3), 0xFD7046C5)
    x = _inv_tfunction(x, lambda t: ((t + 0xD3A2646C) ^ (t << 9)) & M32)
    x = _inv_affine(x, 1 + (1 << 5), 0x165667B1)
    x = _inv_xorshr(x, 19, 0xC761C23C)
    return _inv_affine(x, 1 + (1 << 12), 0x7ED55D16)


def pin_hash_inverses(L, n=3000, seed=1):
    rng = random.Random(seed)
    xs = [0, 1, 2, M32, 0x80000000] + [rng.getrandbits(32) for _ in range(n)]
    for x in xs:
        assert bithash1_inverse(int(L.o2_bithash1(x))) == x, f"BitHash1 inverse at {x:#x}"
        assert bithash2_inverse(int(L.o2_bithash2(x))) == x, f"BitHash2 inverse at {x:#x}"
    for y in xs[:500]:  # and the other way round: every output is reached
        assert int(L.o2_bithash1(bithash1_inverse(y))) == y
        assert int(L.o2_bithash2(bithash2_inverse(y))) == y


# -------------------------------------------- hashes as the listing prints them
def listing_bithash1(key: int) -> int:
    """BitHash1 of the Section III-C listing, one statement per line as it is
    printed, on a 32-bit unsigned key (every statement wraps mod 2^32); the
    listing's final "% nBuckets" is left to the addressing."""
    key = (~key + (key << 15)) & M32
    key ^= key >> 12
    key = (key + (key << 2)) & M32
    key ^= key >> 4
    key = (key * 2057) & M32
    key ^= key >> 16
    return key


def listing_bithash2(key: int) -> int:
    """BitHash2 of the Section III-C listing, statement by statement."""
    key = ((key + 0x7ED55D16) + (key << 12)) & M32
    key = ((key ^ 0xC761C23C) ^ (key >> 19)) & M32
    key = ((key + 0x165667B1) + (key << 5)) & M32
    key = ((key + 0xD3A2646C) ^ (key << 9)) & M32
    key = ((key + 0xFD7046C5) + (key << 3)) & M32
    key = ((key ^ 0xB55A4F09) ^ (key >> 16)) & M32
    return key


LISTING_EDGE_KEYS = [0, 1, 2, 3, 0x7FFF, 0x8000, 0xFFFF, 0x10000, 0x7FFFFFFF, 0x80000000, 0x80000001,
                     0xFFFFFFFE, M32] + [1 << b for b in range(32)] + [M32 ^ (1 << b) for b in range(32)]


def pin_bithash_as_printed(L, n=100_000, seed=9):
    """The oracle's hashes equal the listing's statements evaluated as
    printed (not the oracle's own restatement as affine and xor-shift maps),
    on edge keys and n random keys."""
    rng = random.Random(seed)
    keys = LISTING_EDGE_KEYS + [rng.getrandbits(32) for _ in range(n)]
    for k in keys:
        assert int(L.o2_bithash1(k)) == listing_bithash1(k), f"BitHash1 differs from the listing at {k:#x}"
        assert int(L.o2_bithash2(k)) == listing_bithash2(k), f"BitHash2 differs from the listing at {k:#x}"


# ------------------------------------------------------ addressing pins
def pin_fixed_addressing_is_modulo(L, seed=2):
    rng = random.Random(seed)
    for n in (1, 3, 7, 1000, 8192, 4415057):
        t = O2(4, 8, 16, ADDR_FIXED, n, lib_handle=L)
        for _ in range(200):
            h = rng.getrandbits(32)
            assert t.bucket_of(h) == h % n


def pin_linear_addressing_textbook(L, seed=3):
    """Linear hashing (Litwin 1980): with 2^m + sp buckets, an address is
    H mod 2^(m+1) when H mod 2^m < sp, else H mod 2^m."""
    rng = random.Random(seed)
    t = O2(4, 8, 16, ADDR_LINEAR, 8, max_buckets=64, lib_handle=L)
    for steps in range(0, 40):
        st = t.stats()
        n = st["n_buckets"]
        m = n.bit_length() - 1
        sp = n - (1 << m)
        assert st["split_ptr"] == sp and st["index_mask"] == (1 << m) - 1
        for _ in range(50):
            h = rng.getrandbits(32)
            exp = h % (1 << (m + 1)) if h % (1 << m) < sp else h % (1 << m)
            assert t.bucket_of(h) == exp
            assert exp < n
        t.split(1)


# ------------------------------------------------ O2 vs O1, brute force
def _run_sequence(L, rng, S, n_buckets, addressing, max_buckets, E, stash_cap, n_ops, universe, resize_every=0,
                  K=1, check_every=1):
    t = O2(S, E, stash_cap, addressing, n_buckets, max_buckets=max_buckets, resize_k=K, lib_handle=L)
    d = O1(64, lib_handle=L)
    keys_u = [rng.randrange(1, M32) for _ in range(universe)]
    for i in range(n_ops):
        o = rng.choice([0, 0, 0, 1, 2])
        k = rng.choice(keys_u) if rng.random() > 0.01 else rng.choice([0, M32])
        v = rng.getrandbits(32)
        args = (np.array([o], np.uint8), np.array([k], np.uint32), np.array([v], np.uint32))
        a = t.apply(*args)
        b = d.apply(*args)
        assert a[0][0] == b[0][0] and a[1][0] == b[1][0], f"op {i} ({o}, {k}) differs from the dictionary"
        if resize_every and i % resize_every == resize_every - 1:
            r = rng.random()
            if r < 0.4:
                t.split(K)
            elif r < 0.8:
                t.merge(K)
            else:
                t.policy_post()
        if i % check_every == 0:
            t.check()
    t.check()
    assert np.array_equal(t.dump(), d.dump())
    assert t.stats()["live"] == len(d)
    return t


def pin_o2_matches_o1_fixed(L, seed=4):
    rng = random.Random(seed)
    for S, nb in ((1, 1), (1, 5), (2, 3), (4, 8), (16, 2), (16, 7)):
        cap = S * nb
        _run_sequence(L, rng, S, nb, ADDR_FIXED, nb, E=rng.choice([1, 2, 8]), stash_cap=rng.choice([1, 4, 64]),
                      n_ops=400, universe=max(2, int(cap * 1.3)))


def pin_o2_matches_o1_linear_with_resizes(L, seed=5):
    rng = random.Random(seed)
    for S, nb, mb in ((1, 1, 16), (2, 2, 32), (4, 3, 64), (16, 4, 64)):
        _run_sequence(L, rng, S, nb, ADDR_LINEAR, mb, E=rng.choice([2, 8]), stash_cap=rng.choice([2, 16]),
                      n_ops=600, universe=max(4, S * mb // 2), resize_every=7, K=rng.choice([1, 2, 5]))


def pin_linear_power_of_two_equals_fixed(L, seed=6):
    """I9: LINEAR with 2^m buckets and split pointer 0 addresses exactly like
    FIXED, so one op sequence builds the same layout in both."""
    for S, nb in ((2, 4), (4, 16), (16, 64)):
        rng = random.Random(seed)
        keys = np.array([rng.randrange(1, M32) for _ in range(int(S * nb * 0.97))], np.uint32)
        vals = np.array([rng.getrandbits(32) for _ in keys], np.uint32)
        a = O2(S, 8, 64, ADDR_FIXED, nb, lib_handle=L)
        b = O2(S, 8, 64, ADDR_LINEAR, nb, max_buckets=nb, lib_handle=L)
        a.insert(keys, vals)
        b.insert(keys, vals)
        wa, pa = a.dump(with_where=True)
        wb, pb = b.dump(with_where=True)
        assert np.array_equal(wa, wb) and np.array_equal(pa, pb)
        dl = keys[::3]
        assert np.array_equal(a.delete(dl), b.delete(dl))
        wa, pa = a.dump(with_where=True)
        wb, pb = b.dump(with_where=True)
        assert np.array_equal(wa, wb) and np.array_equal(pa, pb)


# ------------------------------------------------ hand-traced scenarios
def pin_eviction_chain_single_bucket(L):
    """S = 1, one bucket: every key's two candidates coincide.  Inserting k2
    into a full table runs Algorithm 3: each round evicts the occupant and
    the displaced key returns to the same bucket.  After E rounds the item in
    hand goes to the stash: k2 when E is even, k1 when E is odd."""
    k1, k2 = 1111, 2222
    for E in (1, 2, 7, 8):
        t = O2(1, E, 4, ADDR_FIXED, 1, lib_handle=L)
        t.insert(np.array([k1, k2], np.uint32), np.array([10, 20], np.uint32))
        words, where = t.dump(with_where=True)
        place = {int(w) & M32: int(p) for w, p in zip(words, where)}
        in_stash = k2 if E % 2 == 0 else k1
        in_bucket = k1 if E % 2 == 0 else k2
        assert place == {in_bucket: 0, in_stash: -1}, (E, place)
        st = t.stats()
        assert st["evictions"] == E and st["stash_count"] == 1 and st["full_chains"] == 1
        v, f = t.lookup(np.array([k1, k2], np.uint32))
        assert f.tolist() == [1, 1] and v.tolist() == [10, 20]
        t.check()


def pin_stash_full_goes_pending(L):
    """Stash capacity 1, one single-slot bucket, E = 2: k1 is placed, k2 ends
    in the stash, k3 finds the ring full and is held as pending."""
    t = O2(1, 2, 1, ADDR_FIXED, 1, lib_handle=L)
    t.insert(np.array([5, 6, 7], np.uint32), np.array([50, 60, 70], np.uint32))
    words, where = t.dump(with_where=True)
    place = {int(w) & M32: int(p) for w, p in zip(words, where)}
    assert place == {5: 0, 6: -1, 7: -2}
    st = t.stats()
    assert st["stash_count"] == 1 and st["pending_count"] == 1 and st["live"] == 3
    v, f = t.lookup(np.array([5, 6, 7, 8], np.uint32))
    assert f.tolist() == [1, 1, 1, 0] and v.tolist() == [50, 60, 70, M32]
    # replace and delete reach the stash and pending entries
    t.insert(np.array([6, 7], np.uint32), np.array([61, 71], np.uint32))
    assert t.lookup(np.array([6, 7], np.uint32))[0].tolist() == [61, 71]
    assert t.delete(np.array([6, 7, 6], np.uint32)).tolist() == [1, 1, 0]
    assert t.stats()["live"] == 1
    t.check()


def _find_keys(t, pred, count, start=1):
    out, k = [], start
    while len(out) < count:
        c1, c2 = t.candidates([k])
        if pred(int(c1[0]), int(c2[0])):
            out.append(k)
        k += 1
    return out


def pin_two_choice_placement(L):
    """Step 2 claims in the candidate with more free slots; a tie goes to the
    first hash; the claimed slot is the lowest free one (Algorithm 2)."""
    t = O2(2, 8, 4, ADDR_FIXED, 5, lib_handle=L)
    (ka,) = _find_keys(t, lambda a, b: a != b, 1)
    a1, a2 = (int(x[0]) for x in t.candidates([ka]))
    t.insert(np.array([ka], np.uint32), np.array([1], np.uint32))
    _, where = t.dump(with_where=True)
    assert int(where[0]) == a1  # tie: first hash
    # a key whose first candidate is a1 (one free slot left) and second is
    # another, empty bucket goes to the second
    (kb,) = _find_keys(t, lambda a, b: a == a1 and b not in (a1, a2), 1, start=ka + 1)
    b2 = int(t.candidates([kb])[1][0])
    t.insert(np.array([kb], np.uint32), np.array([2], np.uint32))
    words, where = t.dump(with_where=True)
    place = {int(w) & M32: int(p) for w, p in zip(words, where)}
    assert place[kb] == b2
    t.check()


def pin_eviction_reroutes_to_alternate(L):
    """Algorithm 3 moves a victim to its alternate bucket (AltBucket): the
    other candidate of the bucket it was evicted from.

    Single-slot buckets.  k0 (both candidates c) fills c, so k1 (first
    candidate c, second b) lands in b; k0 is deleted, freeing c.  k2 (both
    candidates b) then evicts k1 from b, and k1's alternate from b is c,
    which is free: one eviction, nothing stashed."""
    t = O2(1, 8, 4, ADDR_FIXED, 3, lib_handle=L)
    (k1,) = _find_keys(t, lambda a, b: a != b, 1)
    c1, c2 = (int(x[0]) for x in t.candidates([k1]))
    (k0,) = _find_keys(t, lambda a, b: a == c1 and b == c1, 1)
    (k2,) = _find_keys(t, lambda a, b: a == c2 and b == c2, 1)
    t.insert(np.array([k0, k1], np.uint32), np.array([1, 2], np.uint32))
    assert t.delete(np.array([k0], np.uint32)).tolist() == [1]
    t.insert(np.array([k2], np.uint32), np.array([3], np.uint32))
    words, where = t.dump(with_where=True)
    place = {int(w) & M32: int(p) for w, p in zip(words, where)}
    assert place == {k1: c1, k2: c2}, place
    st = t.stats()
    assert st["evictions"] == 1 and st["stash_count"] == 0
    t.check()


def pin_replace_on_reinsert(L):
    """I7: re-inserting (k, v2) keeps one copy of k, with value v2."""
    t = O2(4, 8, 8, ADDR_FIXED, 4, lib_handle=L)
    ks = np.arange(1000, 1012, dtype=np.uint32)
    t.insert(ks, ks * 3)
    t.insert(ks[::2], ks[::2] * 7)
    v, f = t.lookup(ks)
    exp = ks * 3
    exp[::2] = ks[::2] * 7
    assert f.all() and np.array_equal(v, exp)
    assert t.stats()["live"] == 12
    t.check()


def pin_split_and_merge_geometry(L):
    """Section IV-C: a split advances the split pointer and the round doubles
    the index mask when the pointer wraps; a merge walks back from the top and
    regresses the round when the pointer is 0."""
    t = O2(4, 8, 8, ADDR_LINEAR, 4, max_buckets=32, lib_handle=L)
    g = lambda: (t.stats()["n_buckets"], t.stats()["index_mask"], t.stats()["split_ptr"])  # noqa: E731
    assert g() == (4, 3, 0)
    assert t.split(1) == 1 and g() == (5, 3, 1)
    assert t.split(3) == 3 and g() == (8, 7, 0)
    assert t.split(2) == 2 and g() == (10, 7, 2)
    assert t.merge(3) == 3 and g() == (7, 3, 3)
    assert t.merge(10) == 3 and g() == (4, 3, 0)  # never below the initial size
    t.check()


def pin_split_keeps_every_key_reachable(L, seed=7):
    rng = random.Random(seed)
    t = O2(4, 8, 16, ADDR_LINEAR, 2, max_buckets=128, lib_handle=L)
    keys = np.array(rng.sample(range(1, 1 << 31), 7), np.uint32)
    vals = np.arange(7, dtype=np.uint32)
    t.insert(keys, vals)
    for _ in range(60):
        t.split(1)
        t.check()  # I3: every entry sits in one of its candidates
        v, f = t.lookup(keys)
        assert f.all() and np.array_equal(v, vals)
    for _ in range(60):
        t.merge(1)
        t.check()
        v, f = t.lookup(keys)
        assert f.all() and np.array_equal(v, vals)


def pin_merge_aborts_when_low_bucket_lacks_room(L):
    """A merge of (lo, hi) needs hi's live entries to fit lo's free slots
    (Section IV-C-2); otherwise the batch stops there."""
    t = O2(2, 8, 8, ADDR_LINEAR, 2, max_buckets=8, lib_handle=L)
    t.split(1)  # 3 buckets: pair (0, 2) is split
    both_lo = _find_keys(t, lambda a, b: a == 0 and b == 0, 2)
    both_hi = _find_keys(t, lambda a, b: a == 2 and b == 2, 1)
    t.insert(np.array(both_lo + both_hi, np.uint32), np.array([1, 2, 3], np.uint32))
    assert t.merge(1) == 0 and t.stats()["n_buckets"] == 3
    t.delete(np.array(both_lo[:1], np.uint32))
    assert t.merge(1) == 1 and t.stats()["n_buckets"] == 2
    words, where = t.dump(with_where=True)
    place = {int(w) & M32: int(p) for w, p in zip(words, where)}
    assert place == {both_lo[1]: 0, both_hi[0]: 0}
    t.check()


def pin_policy_pre_expand(L):
    """Pre-batch growth stops at the smallest bucket count that holds the
    batch under the expand threshold: 100 keys, 4-slot buckets, 90% -> 28
    buckets with K=1; with K=5 the steps go 4, 9, ..., 29."""
    for K, exp in ((1, 28), (5, 29)):
        t = O2(4, 8, 16, ADDR_LINEAR, 4, max_buckets=256, resize_k=K, lf_expand_pct=90, lib_handle=L)
        t.policy_pre(100)
        assert t.stats()["n_buckets"] == exp
        keys = np.arange(1, 101, dtype=np.uint32)
        t.insert(keys, keys)
        t.check()
        assert t.lookup(keys)[1].all()


def pin_policy_post_contract(L):
    """Contraction merges while the load factor is under 25% and the table is
    above its initial size; it never removes a key."""
    t = O2(4, 8, 16, ADDR_LINEAR, 4, max_buckets=256, resize_k=2, lib_handle=L)
    keys = np.arange(1, 301, dtype=np.uint32)
    t.policy_pre(300)
    t.insert(keys, keys)
    t.policy_post()
    big = t.stats()["n_buckets"]
    assert 300 * 100 <= 90 * big * 4
    t.delete(keys[:280])
    t.policy_post()
    st = t.stats()
    assert st["n_buckets"] < big
    assert st["n_buckets"] == 4 or st["live"] * 100 >= 25 * st["n_buckets"] * 4 or t.merge(1) == 0
    v, f = t.lookup(keys[280:])
    assert f.all() and np.array_equal(v, keys[280:])
    t.check()


ALL_PINS = [
    pin_o1_matches_python_dict,
    pin_hash_inverses,
    pin_bithash_as_printed,
    pin_fixed_addressing_is_modulo,
    pin_linear_addressing_textbook,
    pin_o2_matches_o1_fixed,
    pin_o2_matches_o1_linear_with_resizes,
    pin_linear_power_of_two_equals_fixed,
    pin_eviction_chain_single_bucket,
    pin_stash_full_goes_pending,
    pin_two_choice_placement,
    pin_eviction_reroutes_to_alternate,
    pin_replace_on_reinsert,
    pin_split_and_merge_geometry,
    pin_split_keeps_every_key_reachable,
    pin_merge_aborts_when_low_bucket_lacks_room,
    pin_policy_pre_expand,
    pin_policy_post_contract,
]


def default_lib():
    return oracle.lib()
