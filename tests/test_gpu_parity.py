"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every integer output is compared bit-exactly: lookup values and found flags,
delete flags, and the final key->value set.  Physical placement is not part
of the contract, but every stored entry must sit in one of its two candidate
buckets as the oracle computes them, and every key must be stored once.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2510_15095_amd import workload as wl

pytestmark = pytest.mark.gpu

M32 = 0xFFFFFFFF


def case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_15095_amd import hive
    return hive


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.cpu().numpy()


def check_placement(table_dump, where, S, n_buckets, addressing=oracle.ADDR_FIXED, max_buckets=None, geo=None):
    """Every bucket entry sits in a candidate bucket (oracle addressing) and
    every key appears once."""
    keys = (table_dump & np.uint64(M32)).astype(np.uint32)
    assert np.unique(keys).size == keys.size, "a key is stored twice"
    o2 = oracle.O2(S, 8, 16, addressing, n_buckets, max_buckets=max_buckets)
    if geo is not None:  # LINEAR: advance the oracle geometry to the same point
        while o2.stats()["n_buckets"] < geo:
            o2.split(1)
    in_bucket = where >= 0
    c1, c2 = o2.candidates(keys[in_bucket])
    w = where[in_bucket]
    bad = (w != c1) & (w != c2)
    assert not bad.any(), f"{bad.sum()} entries outside their candidate buckets"


def run_tiny(H, S, seed=1, n_keys=1 << 16, n_buckets=None, probe_both=0):
    """The tiny configuration: insert all, look up (50% present), delete a
    random half, look up again; compared with the oracle step by step."""
    w = wl.bulk_workload(seed, n_keys)
    n_buckets = n_buckets or (2 * n_keys) // S  # 50% load
    case(f"tiny S={S} keys={n_keys} buckets={n_buckets} probe_both={probe_both}")
    t = H.Table(n_buckets, slots_per_bucket=S, max_evictions=8, stash_capacity=1024, probe_both=probe_both)
    o = oracle.O2(S, 8, 1024, oracle.ADDR_FIXED, n_buckets)
    t.insert(dev(w["ins_keys"]), dev(w["ins_vals"]), flags=H.HIVE_UNIQUE)
    o.insert(w["ins_keys"], w["ins_vals"])
    qk = dev(w["query_keys"])
    v, f = t.lookup(qk)
    ov, of = o.lookup(w["query_keys"])
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    d = t.delete(dev(w["del_keys"]), flags=H.HIVE_UNIQUE)
    assert np.array_equal(host(d), o.delete(w["del_keys"]))
    v, f = t.lookup(qk)
    ov, of = o.lookup(w["query_keys"])
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    st = t.stats()
    assert st["status"] == H.HIVE_OK and st["live"] == o.stats()["live"]
    words, where = t.dump(with_where=True)
    assert np.array_equal(words, o.dump())
    check_placement(words, where, S, n_buckets)
    t.close()


@pytest.mark.parametrize("probe_both", [0, 1])
def test_tiny_config_s16(H, probe_both):
    run_tiny(H, 16, probe_both=probe_both)


@pytest.mark.parametrize("S", [32, 64])
def test_tiny_config_other_widths(H, S):
    run_tiny(H, S, seed=11, n_keys=1 << 14)


def test_ragged_sizes_and_tiny_batches(H):
    for n in (1, 2, 63, 64, 65, 255, 257, 1000, 4097):
        case(f"ragged n={n}")
        t = H.Table(max(1, (2 * n) // 16 + 1))
        w = wl.bulk_workload(7 + n, n, n_queries=n + 1, n_deletes=n // 2)
        t.insert(dev(w["ins_keys"]), dev(w["ins_vals"]))
        v, f = t.lookup(dev(w["query_keys"]))
        present = w["query_idx"] < n
        assert np.array_equal(host(f).astype(bool), present)
        exp = np.where(present, wl.values_for(w["query_keys"]), np.uint32(M32))
        assert np.array_equal(host(v), exp)
        d = t.delete(dev(w["del_keys"]))
        assert host(d).all()
        assert t.stats()["live"] == n - n // 2
        t.close()


def test_empty_batch_and_empty_table(H):
    import torch
    case("empty")
    t = H.Table(64)
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    t.insert(e, e)
    v, f = t.lookup(e)
    assert v.numel() == 0
    keys = dev(np.array([1, 2, 3, 0xFFFFFFFE], np.uint32))
    v, f = t.lookup(keys)
    assert host(f).tolist() == [0, 0, 0, 0] and host(v).tolist() == [M32] * 4
    assert host(t.delete(keys)).tolist() == [0, 0, 0, 0]
    assert t.stats()["live"] == 0
    t.close()


def test_reserved_keys_are_noops(H):
    case("reserved keys")
    t = H.Table(64)
    keys = np.array([0, 5, M32, 6], np.uint32)
    t.insert(dev(keys), dev(np.array([1, 2, 3, 4], np.uint32)))
    v, f = t.lookup(dev(keys))
    assert host(f).tolist() == [0, 1, 0, 1] and host(v).tolist() == [M32, 2, M32, 4]
    assert host(t.delete(dev(keys))).tolist() == [0, 1, 0, 1]
    st = t.stats()
    assert st["invalid_keys"] == 6 and st["status"] == H.HIVE_WARN_INVALID_KEYS and st["live"] == 0
    t.close()


def test_replace_on_reinsert(H):
    case("replace")
    n = 5000
    t = H.Table(n // 8)
    o = oracle.O1()
    keys = wl.KeyStream(21).range(0, n)
    v1 = wl.values_for(keys)
    t.insert(dev(keys), dev(v1), flags=H.HIVE_UNIQUE)
    o.insert(keys, v1)
    v2 = (v1 ^ np.uint32(0x5A5A5A5A)).astype(np.uint32)
    t.insert(dev(keys[::3]), dev(v2[::3]), flags=H.HIVE_UNIQUE)
    o.insert(keys[::3], v2[::3])
    v, f = t.lookup(dev(keys))
    ov, of = o.lookup(keys)
    assert np.array_equal(host(v), ov) and host(f).all()
    assert t.stats()["live"] == n
    assert np.array_equal(t.dump(), o.dump())
    t.close()


def test_dedupe_last_insert_wins_first_delete_reports(H):
    case("dedupe")
    rng = np.random.default_rng(3)
    base = wl.KeyStream(31).range(0, 3000)
    keys = base[rng.integers(0, base.size, 20000)]
    vals = rng.integers(1, 1 << 32, keys.size, dtype=np.uint64).astype(np.uint32)
    t = H.Table(512)
    o = oracle.O1()
    t.insert(dev(keys), dev(vals))
    o.insert(keys, vals)
    v, f = t.lookup(dev(base))
    ov, of = o.lookup(base)
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    dkeys = base[rng.integers(0, base.size, 5000)]
    d = t.delete(dev(dkeys))
    assert np.array_equal(host(d), o.delete(dkeys))
    assert t.stats()["live"] == len(o)
    assert np.array_equal(t.dump(), o.dump())
    t.close()


def _lowbias32(x):
    """The library's mix for its dedupe partitions ("lowbias32", C. Wellons),
    restated here only to build keys that all land in one partition."""
    x = x.astype(np.uint64)
    m = np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7FEB352D)) & m
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846CA68B)) & m
    return (x ^ (x >> np.uint64(16))).astype(np.uint32)


def _one_partition_keys(n, top, seed):
    """n distinct valid keys whose mix has the same top nine bits (one dedupe
    partition of the plain path)."""
    rng = np.random.default_rng(seed)
    out = np.empty(0, np.uint32)
    while out.size < n:
        x = rng.integers(1, 0xFFFFFFFF, 1 << 24, dtype=np.uint64).astype(np.uint32)
        out = np.unique(np.concatenate([out, x[(_lowbias32(x) >> np.uint32(23)) == top]]))
    return rng.permutation(out)[:n]


@pytest.mark.parametrize("kind", ["insert", "mixed", "set32"])
def test_dedupe_partition_beyond_its_lds_table(H, kind):
    """The plain path deduplicates per hash partition in an LDS table that
    takes 6,144 distinct keys; a batch that puts about 9,000 distinct keys
    of one type (with repeats) in one partition takes the partition's HBM
    fallback table.  Outputs, key count and contents equal the
    dictionary's."""
    keys = _one_partition_keys(12000, 77, 41)
    rng = np.random.default_rng(42)
    reps = keys[rng.integers(0, keys.size, 30000)]
    case(f"dedupe partition overflow, {kind}")
    set32 = kind == "set32"
    t = H.Table(4096, slots_per_bucket=32, entry_bits=32) if set32 else H.Table(4096)
    o = oracle.O1()
    if kind in ("insert", "set32"):
        ins = np.concatenate([keys, reps])
        vals = np.zeros(ins.size, np.uint32) if set32 else rng.integers(1, 1 << 32, ins.size, dtype=np.uint64).astype(np.uint32)
        t.insert(dev(ins), None if set32 else dev(vals))
        o.insert(ins, vals)
        dk = np.concatenate([keys[rng.integers(0, keys.size, 20000)], wl.KeyStream(43).range(0, 500)])
        assert np.array_equal(host(t.delete(dev(dk))), o.delete(dk))
    else:
        pre = keys[:3000]
        t.insert(dev(pre), dev(wl.values_for(pre)), flags=H.HIVE_UNIQUE)
        o.insert(pre, wl.values_for(pre))
        # inserts of keys[3000:] with repeats, deletes of keys[:2000] with
        # repeats, lookups of others: disjoint key sets per type
        ins = keys[3000:][rng.integers(0, 9000, 30000)]
        dels = keys[:2000][rng.integers(0, 2000, 8000)]
        looks = keys[2000:3000][rng.integers(0, 1000, 4000)]
        ks = np.concatenate([ins, dels, looks])
        ops = np.concatenate([np.full(ins.size, wl.OP_INSERT), np.full(dels.size, wl.OP_DELETE),
                              np.full(looks.size, wl.OP_LOOKUP)]).astype(np.uint8)
        perm = rng.permutation(ks.size)
        ks, ops = ks[perm], ops[perm]
        vals = rng.integers(1, 1 << 32, ks.size, dtype=np.uint64).astype(np.uint32)
        v, f = t.mixed(dev(ops), dev(ks), dev(vals))
        ov, of = o.apply(ops, ks, vals)
        assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    st = t.stats()
    assert st["status"] >= 0 and st["live"] == len(o), st
    assert np.array_equal(t.dump(), o.dump())
    t.close()


def test_dedupe_every_partition_falls_back(H):
    """An insert batch of 2^22 distinct keys plus 2^20 repeats (no
    HIVE_UNIQUE): about 8,200 distinct keys per dedupe partition, more than
    the LDS table takes, so every partition resolves in its own HBM table at
    once.  The last occurrence of each key wins, as in the dictionary."""
    n_keys, n_rep = 1 << 22, 1 << 20
    case(f"dedupe with every partition in its fallback table: {n_keys} keys + {n_rep} repeats")
    rng = np.random.default_rng(47)
    keys = wl.KeyStream(47).range(0, n_keys)
    ins = np.concatenate([keys, keys[rng.integers(0, n_keys, n_rep)]])
    perm = rng.permutation(ins.size)
    ins = ins[perm]
    vals = rng.integers(1, 1 << 32, ins.size, dtype=np.uint64).astype(np.uint32)
    nb = int(np.ceil(n_keys / (0.6 * 16)))
    t = H.Table(nb, max_batch=ins.size)
    o = oracle.O1(n_keys)
    t.insert(dev(ins), dev(vals))
    o.insert(ins, vals)
    st = t.stats()
    assert st["status"] == H.HIVE_OK and st["live"] == n_keys == len(o), st
    assert np.array_equal(t.dump(), o.dump())
    t.close()


@pytest.mark.parametrize("path", ["plain", "persistent"])
def test_dedupe_delete_batch_sized_from_the_batch(H, path):
    """A delete batch with repeats (no HIVE_UNIQUE) on a table whose scratch
    was never grown by a deduped insert (max_batch = 0, inserts with
    HIVE_UNIQUE): the dedupe set must be sized from the whole batch, which
    sends nothing to the eviction worklist."""
    import torch
    rng = np.random.default_rng(19)
    keys = wl.KeyStream(19).range(0, 12000)
    t = H.Table(2048)
    o = oracle.O1()
    t.insert(dev(keys), dev(wl.values_for(keys)), flags=H.HIVE_UNIQUE)
    o.insert(keys, wl.values_for(keys))
    dkeys = np.concatenate([keys[rng.integers(0, keys.size, 15000)], wl.KeyStream(20).range(0, 3000)])
    case(f"dedupe-sized delete batch of {dkeys.size}, {path}")
    if path == "plain":
        d = host(t.delete(dev(dkeys)))
    else:
        dr = H.hive_drain_create(16, 1, 16, 2, 10_000_000)
        k_ = dev(dkeys)
        fo = torch.full((dkeys.size,), 9, dtype=torch.uint8, device="cuda")
        vo = torch.empty(dkeys.size, dtype=torch.uint32, device="cuda")
        tk = H.hive_drain_submit(dr, t.h, H.HIVE_OP_DELETE, k_, None, None, vo, fo)
        H.hive_drain_launch(dr, 0)
        torch.cuda.synchronize()
        assert H.hive_drain_poll(dr, tk)
        d = host(fo)
        H.hive_drain_destroy(dr)
    assert np.array_equal(d, o.delete(dkeys))
    st = t.stats()
    assert st["status"] == H.HIVE_OK and st["live"] == len(o)
    assert np.array_equal(t.dump(), o.dump())
    t.close()


@pytest.mark.parametrize("timed", [False, True])
@pytest.mark.parametrize("E,stash,lf", [(8, 1024, 0.97), (2, 64, 0.99), (1, 8, 0.995), (0, 4, 0.99)])
def test_eviction_stash_pending_heavy(H, E, stash, lf, timed):
    """Small tables near capacity: eviction chains, the stash and the pending
    list all carry entries, and every operation still matches the oracle.
    With phase timing on, step 4 runs as a launch of its own (the eviction
    launch leaves the entries still in hand in the worklist)."""
    S, nb = 16, 97
    n = int(S * nb * lf)
    case(f"evict-heavy E={E} stash={stash} lf={lf} timed={timed}")
    ks = wl.KeyStream(40 + E)
    keys = ks.range(0, n)
    vals = wl.values_for(keys)
    t = H.Table(nb, max_evictions=E, stash_capacity=stash, pending_capacity=4096)
    H.hive_phase_timing(t.h, timed)
    o = oracle.O1()
    t.insert(dev(keys), dev(vals), flags=H.HIVE_UNIQUE)
    o.insert(keys, vals)
    st = t.stats()
    assert st["status"] in (H.HIVE_OK, H.HIVE_WARN_PENDING), st
    assert st["live"] == n and st["stash_count"] <= stash
    # every chain that ran out of kicks placed its entry in the stash or the
    # pending list, and the counters (summed per wave) say which
    _, where0 = t.dump(with_where=True)
    assert st["full_chains"] == st["stash_inserts"] + st["pending_inserts"]
    assert st["stash_inserts"] == int((where0 == -1).sum()) and st["pending_inserts"] == int((where0 == -2).sum())
    q = ks.range(0, n + 500)
    v, f = t.lookup(dev(q))
    ov, of = o.lookup(q)
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    words, where = t.dump(with_where=True)
    assert np.array_equal(words, o.dump())
    check_placement(words, where, S, nb)
    # replace and delete reach entries wherever they sit, stash included
    v2 = (vals ^ np.uint32(0xABCDEF)).astype(np.uint32)
    t.insert(dev(keys[::2]), dev(v2[::2]), flags=H.HIVE_UNIQUE)
    o.insert(keys[::2], v2[::2])
    dk = keys[1::3]
    assert np.array_equal(host(t.delete(dev(dk), flags=H.HIVE_UNIQUE)), o.delete(dk))
    v, f = t.lookup(dev(q))
    ov, of = o.lookup(q)
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    assert np.array_equal(t.dump(), o.dump())
    t.close()


def test_stash_churn_reuses_deleted_words(H):
    """Insert/delete churn on a FIXED table at 97% load: deleted stash
    entries leave TOMB words, which later placements reuse, so the stash's
    used words (TOMB included) stay below the number of entries it has
    taken; every round matches the dictionary.  No eviction (bound 0): every
    insert whose two buckets are full goes to the stash, so the stash sees
    heavy traffic (with chains, look-ahead displacement leaves it nearly
    empty)."""
    S, nb, cap = 16, 512, 4096
    n = int(S * nb * 0.97)
    ks = wl.KeyStream(44)
    t = H.Table(nb, max_evictions=0, stash_capacity=cap, pending_capacity=cap)
    o = oracle.O1()
    keys = ks.range(0, n)
    t.insert(dev(keys), dev(wl.values_for(keys)), flags=H.HIVE_UNIQUE)
    o.insert(keys, wl.values_for(keys))
    rng = np.random.default_rng(44)
    present = list(keys)
    nxt = n
    for r in range(40):
        case(f"stash churn round {r}")
        pick = rng.choice(len(present), 200, replace=False)
        dk = np.array([present[i] for i in pick], np.uint32)
        for i in sorted(pick.tolist(), reverse=True):
            present[i] = present[-1]
            present.pop()
        assert np.array_equal(host(t.delete(dev(dk), flags=H.HIVE_UNIQUE)), o.delete(dk))
        ik = ks.range(nxt, nxt + 200)
        nxt += 200
        present += list(ik)
        t.insert(dev(ik), dev(wl.values_for(ik)), flags=H.HIVE_UNIQUE)
        o.insert(ik, wl.values_for(ik))
        st = t.stats()
        assert st["status"] in (H.HIVE_OK, H.HIVE_WARN_PENDING), st
        assert st["live"] == len(o) and st["stash_count"] <= cap
    assert st["stash_count"] < st["stash_inserts"], st
    q = ks.range(0, nxt + 100)
    v, f = t.lookup(dev(q))
    ov, of = o.lookup(q)
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    assert np.array_equal(t.dump(), o.dump())
    t.close()


def test_phase_timing_groups_reset_and_results(H):
    """Phase timing: an insert call times its dedupe, probe, eviction and
    finish groups, a lookup only its probe launch, a LINEAR insert also its
    resize and drain groups; reading resets, many calls between reads are
    summed, turning it off stops it, and results are unchanged."""
    S, nb = 16, 97
    n = int(S * nb * 0.97)
    ks = wl.KeyStream(90)
    keys = ks.range(0, n)
    vals = wl.values_for(keys)
    t = H.Table(nb, stash_capacity=1024, pending_capacity=4096)
    o = oracle.O1()
    H.hive_phase_timing(t.h, True)
    t.insert(dev(keys), dev(vals))  # not flagged unique: the dedupe set runs
    o.insert(keys, vals)
    ms = H.hive_phase_times(t.h)
    assert ms["dedupe"] > 0 and ms["probe"] > 0 and ms["evict"] > 0 and ms["finish"] > 0, ms
    assert ms["stash"] > 0, ms  # 97% load: some chains run out, step 4 is timed apart
    assert ms["resize"] == 0 and ms["drain"] == 0, ms
    st = t.stats()
    assert st["full_chains"] > 0 and st["full_chains"] == st["stash_inserts"] + st["pending_inserts"], st
    assert all(x == 0 for x in H.hive_phase_times(t.h).values())
    q = ks.range(0, n + 100)
    v, f = t.lookup(dev(q))
    ms = H.hive_phase_times(t.h)
    assert ms["probe"] > 0 and ms["evict"] == ms["dedupe"] == ms["finish"] == 0, ms
    ov, of = o.lookup(q)
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    for _ in range(40):
        t.lookup(dev(q[:64]))
    assert H.hive_phase_times(t.h)["probe"] > 0
    H.hive_phase_timing(t.h, False)
    t.lookup(dev(q))
    assert all(x == 0 for x in H.hive_phase_times(t.h).values())
    assert np.array_equal(t.dump(), o.dump())
    t.close()
    lt = linear_table(H, 8, 4096, 64)
    H.hive_phase_timing(lt.h, True)
    lk = ks.range(10_000, 13_000)
    lt.insert(dev(lk), dev(wl.values_for(lk)), flags=H.HIVE_UNIQUE)
    ms = H.hive_phase_times(lt.h)
    assert ms["resize"] > 0 and ms["drain"] > 0 and ms["probe"] > 0, ms
    assert lt.stats()["live"] == lk.size
    lt.close()


def test_large_stash_probe_runs(H):
    """Thousands of entries in the stash (no cuckoo chains, buckets far over
    capacity): searches, replaces, deletes (tombstones) and re-inserts all go
    through the stash's linear-probe runs and match the dictionary."""
    S, nb = 16, 64
    n = 4000  # 1,024 bucket slots: about 3,000 entries end in the stash
    case(f"large stash n={n} buckets={nb}")
    ks = wl.KeyStream(47)
    keys = ks.range(0, n)
    vals = wl.values_for(keys)
    t = H.Table(nb, max_evictions=0, stash_capacity=8192, pending_capacity=1024)
    o = oracle.O1()
    t.insert(dev(keys), dev(vals), flags=H.HIVE_UNIQUE)
    o.insert(keys, vals)
    st = t.stats()
    assert st["status"] == H.HIVE_OK and st["live"] == n
    assert 2500 < st["stash_count"] <= 8192 and st["pending_count"] == 0
    q = ks.range(0, n + 3000)
    for step in range(3):
        v, f = t.lookup(dev(q))
        ov, of = o.lookup(q)
        assert np.array_equal(host(f), of) and np.array_equal(host(v), ov), step
        assert np.array_equal(t.dump(), o.dump()), step
        if step == 0:  # replace every third key, wherever it sits
            v2 = (vals[::3] ^ np.uint32(0x5A5A5A)).astype(np.uint32)
            t.insert(dev(keys[::3]), dev(v2), flags=H.HIVE_UNIQUE)
            o.insert(keys[::3], v2)
        elif step == 1:  # delete half, then put a quarter back
            dk = keys[1::2]
            assert np.array_equal(host(t.delete(dev(dk), flags=H.HIVE_UNIQUE)), o.delete(dk))
            rk = dk[::2]
            rv = (wl.values_for(rk) + np.uint32(1)).astype(np.uint32)
            t.insert(dev(rk), dev(rv), flags=H.HIVE_UNIQUE)
            o.insert(rk, rv)
    assert t.stats()["live"] == len(o)
    t.close()


@pytest.mark.parametrize("probe_both", [0, 1])
def test_mixed_batches_zipf(H, probe_both):
    """Prefill, then mixed batches (40% insert with repeats, 40% delete, 20%
    lookup, Zipf keys, per-type disjoint): per-batch outputs and the final
    set equal the dictionary's."""
    S, nb = 16, 4096
    universe = 1 << 16
    ks = wl.KeyStream(3)
    pre = ks.keys(wl.DomainPerm(33, universe).sample(int(0.8 * S * nb * 0.9)))
    t = H.Table(nb, stash_capacity=2048, probe_both=probe_both)
    o = oracle.O1()
    t.insert(dev(pre), dev(wl.values_for(pre)), flags=H.HIVE_UNIQUE)
    o.insert(pre, wl.values_for(pre))
    for b in range(6):
        case(f"mixed batch {b}")
        mb = wl.mixed_batch(3, b, 1 << 14, universe, stream=ks, value_salt=b + 1)
        v, f = t.mixed(dev(mb["ops"]), dev(mb["keys"]), dev(mb["vals"]))
        ov, of = o.apply(mb["ops"], mb["keys"], mb["vals"])
        assert np.array_equal(host(f), of), f"flags differ in batch {b}"
        assert np.array_equal(host(v), ov), f"values differ in batch {b}"
        assert t.stats()["live"] == len(o)
    assert np.array_equal(t.dump(), o.dump())
    t.close()


@pytest.mark.parametrize("probe_both", [0, 1])
def test_bulk_95pct_reduced(H, probe_both):
    """The bulk configuration at 2^20 keys: FIXED table at 95% load, 50%-hit
    queries, delete half, re-query; exact expected outputs come from the
    generator (present iff inserted and not deleted, value = value(key))."""
    run_bulk(H, 1 << 20, seed=2, probe_both=probe_both)


def run_bulk(H, n_keys, seed, probe_both=0, **cfg):
    S = 16
    nb = int(np.ceil(n_keys / (0.95 * S)))
    case(f"bulk n={n_keys} buckets={nb} probe_both={probe_both} {cfg}")
    w = wl.bulk_workload(seed, n_keys)
    t = H.Table(nb, probe_both=probe_both, **cfg)
    t.insert(dev(w["ins_keys"]), dev(w["ins_vals"]), flags=H.HIVE_UNIQUE)
    st = t.stats()
    assert st["live"] == n_keys and st["status"] == H.HIVE_OK, st
    qk = dev(w["query_keys"])
    present = w["query_idx"] < n_keys
    exp_v = np.where(present, wl.values_for(w["query_keys"]), np.uint32(M32))
    v, f = t.lookup(qk)
    assert np.array_equal(host(f).astype(bool), present)
    assert np.array_equal(host(v), exp_v)
    d = t.delete(dev(w["del_keys"]), flags=H.HIVE_UNIQUE)
    assert host(d).all()
    deleted = np.zeros(n_keys, bool)
    deleted[w["del_idx"]] = True
    still = present.copy()
    still[present] = ~deleted[w["query_idx"][present]]
    v, f = t.lookup(qk)
    assert np.array_equal(host(f).astype(bool), still)
    assert np.array_equal(host(v), np.where(still, exp_v, np.uint32(M32)))
    st = t.stats()
    assert st["live"] == n_keys - w["del_keys"].size
    words = t.dump()
    idx = w["stream"].index_of((words & np.uint64(M32)).astype(np.uint32))
    assert idx.size == st["live"] and np.unique(idx).size == idx.size
    assert not deleted[idx].any() and (idx < n_keys).all()
    assert np.array_equal((words >> np.uint64(32)).astype(np.uint32), w["ins_vals"][idx])
    t.close()
    return st


def test_bulk_95pct_full_size(H):
    """2^26 keys into 4,415,057 16-slot buckets (95% load): every output is
    checked against the generator's closed-form expectation."""
    st = run_bulk(H, 1 << 26, seed=2)
    print("bulk 2^26 stats:", st)


def tuned_probe_cfg():
    """The probe-kernel variant word and grid cap the benchmark launches
    with (the autotuner's picks for this GPU), or a non-default variant of
    every kind when none are recorded."""
    from paper_2510_15095_amd import autotune
    from paper_2510_15095_amd import hive
    pk = autotune.load("probe_kernel") or {}
    tuning = pk.get("probe_tuning", 0) or hive.probe_tuning(4, 2, 2, 2)
    return dict(probe_tuning=tuning, probe_grid=pk.get("probe_grid", 0))


def test_bulk_95pct_full_size_tuned_probe(H):
    """The same full-size sequence with the probe-kernel variants and grid
    cap the benchmark runs."""
    st = run_bulk(H, 1 << 26, seed=2, **tuned_probe_cfg())
    print("bulk 2^26 tuned stats:", st)


def test_bulk_launches_striding_over_tiles_with_ragged_tails(H):
    """Batches beyond the probe launch's block cap: each block strides over
    two or more tiles of 256 operations and the last tile is partial (insert
    and lookup 2 x 32,768 x 256 + 1,000 operations, delete half of that)."""
    st = run_bulk(H, 2 * 32768 * 256 + 1000, seed=4)
    print("bulk ragged stats:", st)


def linear_table(H, nb, max_buckets, K, pre=1, post=1, lf_e=90, lf_c=25, stash=256):
    return H.Table(nb, addressing=H.HIVE_LINEAR, max_buckets=max_buckets, resize_k=K, pre_expand=pre,
                   post_policy=post, lf_expand_pct=lf_e, lf_contract_pct=lf_c, stash_capacity=stash,
                   pending_capacity=1024)


def geometry(st):
    return st["n_buckets"], st["index_mask"], st["split_ptr"]


def same_geometry(gpu_st, o2):
    """Equal bucket counts give equal addressing; (im, sp) agree up to the
    equivalent form sp == im + 1 that a merge regress leaves."""
    ost = o2.stats()
    g, o = geometry(gpu_st), (ost["n_buckets"], ost["index_mask"], ost["split_ptr"])
    norm = lambda t: (t[0], 2 * t[1] + 1, 0) if t[2] == t[1] + 1 else t  # noqa: E731
    return norm(g) == norm(o)


def next_merge_blocked(S, geo, where):
    """The next merge pair (from the top) of a LINEAR table with geometry
    (n_buckets, index_mask, split_ptr) does not fit: its high bucket holds
    more entries than its low bucket has free slots (Section IV-C-2)."""
    nb, im, sp = geo
    if sp == 0:
        im, sp = im >> 1, (im >> 1) + 1
    lo, hi = sp - 1, sp + im
    counts = np.bincount(where[where >= 0], minlength=nb)
    return counts[hi] > S - counts[lo]


def check_post_policy(t, S, lf_e=90, lf_c=25, initial=None):
    """After a post-batch policy call the table is not over the expand
    threshold, and it is under the contract threshold only when it is at its
    initial size or its next merge pair does not fit."""
    st = t.stats()
    nb, live = st["n_buckets"], st["live"]
    assert live * 100 <= lf_e * nb * S
    if live * 100 < lf_c * nb * S and nb != initial:
        _, where = t.dump(with_where=True)
        assert next_merge_blocked(S, geometry(st), where), f"next merge of {geometry(st)} fits but the policy stopped"


def check_divergence(S, geo_a, where_a, geo_b, where_b):
    """Two tables that ran the same batches part only where a merge step
    stopped early on one side (the pair did not fit its layout); the side
    with more buckets is blocked at its next pair."""
    if geo_a == geo_b:
        return
    geo, where = (geo_a, where_a) if geo_a[0] > geo_b[0] else (geo_b, where_b)
    assert next_merge_blocked(S, geo, where), (geo_a, geo_b)


@pytest.mark.parametrize("K", [1, 7, 64])
def test_linear_growth_and_contraction_match_oracle(H, K):
    """Pre-batch expansion and post-batch contraction (Section IV-C): the
    bucket count, index mask and split pointer after every batch equal the
    oracle's, and every key stays reachable.  Splits never abort, so growth
    matches exactly; a merge stops at the first pair whose entries do not fit
    the low bucket, which depends on the physical layout (not part of the
    contract), so once the GPU's layout blocks a merge the test checks that
    the block is real instead of comparing geometry."""
    S, nb0, mb = 16, 8, 4096
    t = linear_table(H, nb0, mb, K)
    o2 = oracle.O2(S, 8, 256, oracle.ADDR_LINEAR, nb0, max_buckets=mb, resize_k=K)
    o1 = oracle.O1()
    ks = wl.KeyStream(50 + K)
    n_batch = 3000
    for b in range(6):
        case(f"linear K={K} insert batch {b}")
        keys = ks.range(b * n_batch, (b + 1) * n_batch)
        vals = wl.values_for(keys)
        o2.policy_pre(n_batch)
        o2.insert(keys, vals)
        o2.policy_post()
        o1.insert(keys, vals)
        t.insert(dev(keys), dev(vals), flags=H.HIVE_UNIQUE)
        st = t.stats()
        assert st["status"] == H.HIVE_OK, st
        assert same_geometry(st, o2), (geometry(st), o2.stats())
        assert st["live"] == len(o1)
    allk = ks.range(0, 6 * n_batch + 500)
    v, f = t.lookup(dev(allk))
    ov, of = o1.lookup(allk)
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    rng = np.random.default_rng(K)
    order = rng.permutation(6 * n_batch)
    diverged = False
    for b in range(5):
        case(f"linear K={K} delete batch {b}")
        dk = allk[order[b * 3400:(b + 1) * 3400]]
        d = t.delete(dev(dk), flags=H.HIVE_UNIQUE)
        o2.delete(dk)
        o2.policy_post()
        assert np.array_equal(host(d), o1.delete(dk))
        st = t.stats()
        check_post_policy(t, S, initial=nb0)
        if not diverged and not same_geometry(st, o2):
            ost = o2.stats()
            _, ow = o2.dump(with_where=True)
            _, gw = t.dump(with_where=True)
            check_divergence(S, geometry(st), gw, (ost["n_buckets"], ost["index_mask"], ost["split_ptr"]), ow)
            diverged = True
        assert st["live"] == len(o1)
        v, f = t.lookup(dev(allk))
        ov, of = o1.lookup(allk)
        assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
    words, where = t.dump(with_where=True)
    assert np.array_equal(words, o1.dump())
    check_placement(words, where, S, nb0, oracle.ADDR_LINEAR, mb, geo=t.stats()["n_buckets"])
    t.close()


def test_linear_explicit_split_merge_and_stash_drain(H):
    """hive_resize(+d) splits d pairs, hive_resize(-d) merges d pairs top
    down; stash entries survive splits (drained and re-placed) and merges."""
    S, nb0, mb = 16, 4, 256
    t = linear_table(H, nb0, mb, 4, pre=0, post=0, stash=512)
    o1 = oracle.O1()
    ks = wl.KeyStream(77)
    keys = ks.range(0, 80)  # 80 keys into 64 slots: the stash must hold some
    vals = wl.values_for(keys)
    t.insert(dev(keys), dev(vals), flags=H.HIVE_UNIQUE)
    o1.insert(keys, vals)
    st = t.stats()
    assert st["stash_count"] + st["pending_count"] > 0 and st["live"] == 80
    for delta, exp_nb in ((5, 9), (40, 49), (-3, 46), (100, 146), (-50, 96)):
        case(f"explicit resize {delta}")
        t.resize(delta)
        st = t.stats()
        assert st["n_buckets"] == exp_nb, (delta, st)
        v, f = t.lookup(dev(keys))
        ov, of = o1.lookup(keys)
        assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
        words, where = t.dump(with_where=True)
        assert np.array_equal(words, o1.dump())
        check_placement(words, where, S, nb0, oracle.ADDR_LINEAR, mb, geo=st["n_buckets"])
    t.close()


def test_drain_stash_drain_after_splits(H):
    """The executor's stash-drain and re-place phases: a LINEAR table whose
    stash holds entries takes insert batches through the executor with
    pre-batch expansion, so splits drain the stash and re-place it; lookups,
    contents and geometry equal the plain path's and the dictionary's."""
    import torch
    S, nb0, mb = 16, 64, 2048

    def table():  # no cuckoo kicks, growth only above 96%: the first 980 keys leave some in the stash
        return H.Table(nb0, addressing=H.HIVE_LINEAR, max_buckets=mb, resize_k=16, pre_expand=1, post_policy=0,
                       lf_expand_pct=96, lf_contract_pct=25, max_evictions=0, stash_capacity=512,
                       pending_capacity=1024)
    o1 = oracle.O1()
    ks = wl.KeyStream(78)
    keys = ks.range(0, 980)
    vals = wl.values_for(keys)
    plain, drained = table(), table()
    for t in (plain, drained):
        t.insert(dev(keys), dev(vals), flags=H.HIVE_UNIQUE)
        assert t.stats()["n_buckets"] == nb0
    o1.insert(keys, vals)
    assert drained.stats()["stash_count"] > 0
    # each later batch grows the table first: splits, then the stash drain
    d = H.hive_drain_create(16, 0, 16, 4, 10_000_000)
    keep, plan = [], []
    for b in range(4):
        bk = ks.range(1000 + b * 700, 1000 + (b + 1) * 700)
        bv = wl.values_for(bk)
        k_, v_ = dev(bk), dev(bv)
        keep += [k_, v_]
        assert H.hive_drain_submit(d, drained.h, H.HIVE_OP_INSERT, k_, v_, flags=H.HIVE_UNIQUE) is not None
        plan.append((bk, bv))
    case("drain launch, stash drain after splits")
    H.hive_drain_launch(d, 0)
    torch.cuda.synchronize()
    for bk, bv in plan:
        plain.insert(dev(bk), dev(bv), flags=H.HIVE_UNIQUE)
        o1.insert(bk, bv)
    q = np.concatenate([keys] + [bk for bk, _ in plan] + [ks.range(9000, 9500)])
    ov, of = o1.lookup(q)
    for t in (plain, drained):
        v, f = t.lookup(dev(q))
        assert np.array_equal(host(f), of) and np.array_equal(host(v), ov)
        assert np.array_equal(t.dump(), o1.dump())
    assert geometry(plain.stats()) == geometry(drained.stats())
    H.hive_drain_destroy(d)
    for t in (plain, drained):
        t.close()


def test_linear_merge_stops_when_pair_does_not_fit(H):
    """A full low bucket blocks its merge: the top pairs merge, the call
    stops at the first pair that does not fit."""
    S, nb0, mb = 16, 2, 64
    t = linear_table(H, nb0, mb, 1, pre=0, post=0)
    t.resize(30)  # 32 buckets
    assert t.stats()["n_buckets"] == 32
    o2 = oracle.O2(S, 8, 16, oracle.ADDR_LINEAR, nb0, max_buckets=mb)
    o2.split(30)
    # fill bucket 1 completely with keys whose two candidates are both 1, and
    # put one key in its partner 17 (both candidates 17)
    ks = wl.KeyStream(91)
    cand = ks.range(0, 200000)
    c1, c2 = o2.candidates(cand)
    in1 = cand[(c1 == 1) & (c2 == 1)][:16]
    in17 = cand[(c1 == 17) & (c2 == 17)][:1]
    assert in1.size == 16 and in17.size == 1
    ins = np.concatenate([in1, in17])
    t.insert(dev(ins), dev(wl.values_for(ins)), flags=H.HIVE_UNIQUE)
    # merging 20 pairs from the top: pairs (15,31)..(2,18) fit, (1,17) does not
    t.resize(-20)
    st = t.stats()
    assert st["n_buckets"] == 18, st
    v, f = t.lookup(dev(ins))
    assert host(f).all()
    t.close()


# ---------------------------------------------------------------- executor
def _mixed_batches(seed, n_batches, n_ops, universe, ks):
    return [wl.mixed_batch(seed, b, n_ops, universe, stream=ks, value_salt=b + 1) for b in range(n_batches)]


@pytest.mark.parametrize("bpc", [0, 1])  # full occupancy, one resident block per CU
def test_drain_matches_plain_and_oracle_mixed(H, bpc):
    """The persistent executor gives the same per-batch outputs and final
    contents as one plain launch sequence per batch, and as the dictionary."""
    import torch
    universe, nb = 1 << 16, 2048
    ks = wl.KeyStream(61)
    pre = ks.keys(wl.DomainPerm(61, universe).sample(int(0.85 * nb * 16)))
    batches = _mixed_batches(61, 6, 1 << 13, universe, ks)
    plain = H.Table(nb, stash_capacity=2048, max_batch=1 << 13)
    drained = H.Table(nb, stash_capacity=2048, max_batch=1 << 13)
    o = oracle.O1()
    for t in (plain, drained):
        t.insert(dev(pre), dev(wl.values_for(pre)), flags=H.HIVE_UNIQUE)
    o.insert(pre, wl.values_for(pre))
    d = H.hive_drain_create(16, bpc, 64, 8, 10_000_000)
    outs, tickets, keep = [], [], []
    for mb in batches:
        o_, k_, v_ = dev(mb["ops"]), dev(mb["keys"]), dev(mb["vals"])
        vo = torch.full((k_.numel(),), 7, dtype=torch.uint32, device="cuda")
        fo = torch.full((k_.numel(),), 9, dtype=torch.uint8, device="cuda")
        keep += [o_, k_, v_]
        tickets.append(H.hive_drain_submit(d, drained.h, H.HIVE_OP_MIXED, k_, v_, o_, vo, fo))
        outs.append((vo, fo))
    case(f"drain launch, 6 mixed batches, {bpc} blocks per CU")
    H.hive_drain_launch(d, 0)
    torch.cuda.synchronize()
    assert all(H.hive_drain_poll(d, t) for t in tickets)
    done, live_after = H.hive_drain_results(d, tickets)
    assert done.all()
    assert [int(x) for x in live_after] == [H.hive_drain_result(d, t)[1] for t in tickets]
    with pytest.raises(H.HiveError):
        H.hive_drain_results(d, [tickets[-1] + 1])  # never submitted
    for b, mb in enumerate(batches):
        pv, pf = plain.mixed(dev(mb["ops"]), dev(mb["keys"]), dev(mb["vals"]))
        ov, of = o.apply(mb["ops"], mb["keys"], mb["vals"])
        assert np.array_equal(host(outs[b][1]), of) and np.array_equal(host(outs[b][0]), ov), f"batch {b}"
        assert np.array_equal(host(pf), of) and np.array_equal(host(pv), ov)
    assert np.array_equal(drained.dump(), o.dump()) and np.array_equal(plain.dump(), o.dump())
    assert drained.stats()["live"] == len(o)
    H.hive_drain_destroy(d)


def test_drain_empty_batches_change_nothing(H):
    """Empty batches of every mode complete through the executor and leave
    the table as the plain entry points do (which return at once): a LINEAR
    table grown by hand below its contraction threshold keeps its buckets."""
    import torch
    tabs = [linear_table(H, 8, 4096, 4) for _ in range(2)]
    keys = wl.KeyStream(90).range(0, 600)
    for t in tabs:
        t.insert(dev(keys), dev(wl.values_for(keys)), flags=H.HIVE_UNIQUE)
        t.resize(400)  # 600 keys in well over 400 buckets: far under 25%
    drained, plain = tabs
    before = drained.stats()
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    e8 = torch.empty(0, dtype=torch.uint8, device="cuda")
    d = H.hive_drain_create(16, 1, 16, 2, 10_000_000)
    tickets = [H.hive_drain_submit(d, drained.h, mode, e, e, e8, e, e8)
               for mode in (H.HIVE_OP_INSERT, H.HIVE_OP_DELETE, H.HIVE_OP_LOOKUP, H.HIVE_OP_MIXED)]
    tickets.append(H.hive_drain_submit(d, drained.h, H.HIVE_OP_LOOKUP, dev(keys), None, None, e.new_empty(600),
                                       e8.new_empty(600)))
    case("drain launch, empty batches")
    H.hive_drain_launch(d, 0)
    torch.cuda.synchronize()
    done, _ = H.hive_drain_results(d, tickets)
    assert done.all()
    plain.insert(e, e)
    plain.delete(e)
    plain.lookup(e)
    plain.mixed(e8, e, e)
    after, ref = drained.stats(), plain.stats()
    assert geometry(after) == geometry(before) == geometry(ref), (before, after, ref)
    assert after["live"] == ref["live"] == keys.size
    assert np.array_equal(drained.dump(), plain.dump())
    H.hive_drain_destroy(d)


@pytest.mark.parametrize("bpc", [0, 1])
def test_drain_multi_table_linear_policies(H, bpc):
    """Interleaved batches on three LINEAR tables with pre-batch expansion
    and post-batch contraction: outputs equal the dictionary's and the
    geometry equals that of the same sequence run with plain launches."""
    import torch
    S, nb0, mb_ = 16, 8, 2048
    names = range(3)
    tabs = {i: linear_table(H, nb0, mb_, 4) for i in names}
    refs = {i: linear_table(H, nb0, mb_, 4) for i in names}
    o1 = {i: oracle.O1() for i in names}
    d = H.hive_drain_create(16, bpc, 128, 8, 10_000_000)
    ks = {i: wl.KeyStream(70 + i) for i in names}
    plan = []
    for step in range(5):
        for i in names:
            plan.append((i, H.HIVE_OP_INSERT, ks[i].range(step * 900, (step + 1) * 900)))
    for i in names:
        plan.append((i, H.HIVE_OP_LOOKUP, ks[i].range(0, 5000)))
    for step in range(4):
        for i in names:
            plan.append((i, H.HIVE_OP_DELETE, ks[i].range(step * 1100, (step + 1) * 1100)))
    for i in names:
        plan.append((i, H.HIVE_OP_LOOKUP, ks[i].range(0, 5000)))
    keep, outs = [], []
    for i, mode, keys in plan:
        k_ = dev(keys)
        v_ = dev(wl.values_for(keys)) if mode == H.HIVE_OP_INSERT else None
        vo = torch.empty(keys.size, dtype=torch.uint32, device="cuda")
        fo = torch.empty(keys.size, dtype=torch.uint8, device="cuda")
        keep += [k_, v_]
        t = H.hive_drain_submit(d, tabs[i].h, mode, k_, v_, None, vo, fo, flags=H.HIVE_UNIQUE)
        assert t is not None
        outs.append((vo, fo))
    case(f"drain launch, multi-table linear, {bpc} blocks per CU")
    H.hive_drain_launch(d, 0)
    torch.cuda.synchronize()
    for (i, mode, keys), (vo, fo) in zip(plan, outs):
        t = refs[i]
        if mode == H.HIVE_OP_INSERT:
            t.insert(dev(keys), dev(wl.values_for(keys)), flags=H.HIVE_UNIQUE)
            o1[i].insert(keys, wl.values_for(keys))
        elif mode == H.HIVE_OP_DELETE:
            pf = t.delete(dev(keys), flags=H.HIVE_UNIQUE)
            assert np.array_equal(host(fo), o1[i].delete(keys)) and np.array_equal(host(pf), host(fo))
        else:
            t.lookup(dev(keys))
            ov, of = o1[i].lookup(keys)
            assert np.array_equal(host(fo), of) and np.array_equal(host(vo), ov)
    for i in names:
        check_post_policy(tabs[i], S, initial=nb0)
        check_post_policy(refs[i], S, initial=nb0)
        check_divergence(S, geometry(tabs[i].stats()), tabs[i].dump(with_where=True)[1],
                         geometry(refs[i].stats()), refs[i].dump(with_where=True)[1])
        assert np.array_equal(tabs[i].dump(), o1[i].dump())
    H.hive_drain_destroy(d)


def test_drain_resident_incremental_and_backpressure(H):
    """A resident grid serves batches submitted while it runs; a full ring
    refuses submissions until earlier batches complete."""
    import time

    import torch
    t = H.Table(1024, max_batch=4096)
    o = oracle.O1()
    d = H.hive_drain_create(16, 0, 4, 4, 10_000_000)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()  # the resident grid must not block torch's own stream
    H.hive_drain_launch(d, 1, side)
    ks = wl.KeyStream(80)
    keep = []
    refused = 0
    for b in range(12):
        keys = ks.range(b * 1000, b * 1000 + 1000)
        vals = wl.values_for(keys)
        k_, v_ = dev(keys), dev(vals)
        torch.cuda.current_stream().synchronize()
        keep += [k_, v_]
        case(f"resident submit {b}")
        deadline = time.time() + 30
        while True:
            tk = H.hive_drain_submit(d, t.h, H.HIVE_OP_INSERT, k_, v_, flags=H.HIVE_UNIQUE)
            if tk is not None:
                break
            refused += 1
            assert time.time() < deadline, "ring never drained"
            time.sleep(0.0005)
        o.insert(keys, vals)
        if b % 3 == 2:  # a lookup batch; wait for it before the next submission
            q = dev(ks.range(0, 13000))
            vo = torch.empty(13000, dtype=torch.uint32, device="cuda")
            fo = torch.empty(13000, dtype=torch.uint8, device="cuda")
            torch.cuda.current_stream().synchronize()
            keep += [q, vo, fo]
            while (lt := H.hive_drain_submit(d, t.h, H.HIVE_OP_LOOKUP, q, None, None, vo, fo)) is None:
                assert time.time() < deadline, "lookup batch never admitted"
                time.sleep(0.0005)
            while not H.hive_drain_poll(d, lt):
                assert time.time() < deadline, "lookup batch never completed"
                time.sleep(0.0002)
            ov, of = o.lookup(ks.range(0, 13000))
            assert np.array_equal(host(fo), of) and np.array_equal(host(vo), ov)
    # an insert batch larger than the table's preallocated worklist is
    # refused on the host while the grid runs (its scratch cannot grow)
    big = dev(ks.range(20000, 25000))
    with pytest.raises(H.HiveError):
        H.hive_drain_submit(d, t.h, H.HIVE_OP_INSERT, big, big, flags=H.HIVE_UNIQUE)
    H.hive_drain_stop(d, side)
    assert np.array_equal(t.dump(), o.dump())
    H.hive_drain_destroy(d)


# ---------------------------------------------------------------- serving
_SERVED = {}


def _served_setup():
    """Tables, requests and the dictionary's answers, made once: 32 LINEAR
    tables of 2^U(12,18) keys at 85% load, 2,000 mixed requests (50% lookup,
    25% insert, 25% delete, uniform or Zipf keys) of 2^U(0,16) operations on
    random tables.  The expected outputs replay each table's requests, in
    submission order, through a dictionary loaded with that table's keys."""
    if not _SERVED:
        from paper_2510_15095_amd import serve as sv
        specs = sv.make_specs(32, 9, log2_min=12, log2_max=18)
        reqs = sv.make_requests(specs, 2000, 9, rate=20000.0, log2_max_size=16)
        dicts, expect = {}, []
        for r in reqs:
            if r.table not in dicts:
                sp = specs[r.table]
                keys = wl.KeyStream(sp.seed).range(0, sp.n_keys)
                dicts[r.table] = oracle.O1(2 * sp.n_keys)
                dicts[r.table].insert(keys, wl.values_for(keys))
            expect.append(dicts[r.table].apply(r.ops, r.keys, r.vals))
        _SERVED.update(specs=specs, reqs=reqs, expect=expect,
                       final={t: o.dump() for t, o in dicts.items()})
    return _SERVED


@pytest.mark.parametrize("bpc", [1, 0])  # the server's default, then full occupancy
def test_served_results_equal_the_dictionary_alone_and_in_the_mix(H, bpc):
    """Each request's outputs equal the dictionary's, whether it runs alone
    (one at a time, in submission order) or in the mix served by the
    persistent executor or by plain per-request launches on several streams;
    after each run every table holds the dictionary's final contents."""
    from paper_2510_15095_amd import serve as sv
    d = _served_setup()
    specs, reqs, expect = d["specs"], d["reqs"], d["expect"]
    srv = sv.Server(specs, 2 * sv.footprint_bytes(specs), max_request=1 << 16, ring=256, streams=4,
                    blocks_per_cu=bpc)
    runs = []
    for mode in ("alone", "persistent", "plain"):
        case(f"served: {mode}, {bpc} blocks per CU")
        srv.load()
        if mode == "alone":
            runs.append((mode, srv.run_alone(reqs)))
        else:
            res = srv.run(reqs, mode, outputs=True, timeout_s=120)
            print(mode, {k: v for k, v in res.items() if k != "results"})
            runs.append((mode, res["results"]))
        for t, words in d["final"].items():
            assert np.array_equal(srv.tables[t].dump(), words), f"{mode}: table {t} contents differ"
    for mode, results in runs:
        for i, ((v, f), (ov, of)) in enumerate(zip(results, expect)):
            assert np.array_equal(f, of) and np.array_equal(v, ov), f"{mode}: request {i} differs"
    srv.close()
