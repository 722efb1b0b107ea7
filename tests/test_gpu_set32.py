"""GPU parity of the 32-bit-entry variant: a key-only set with 32-slot
buckets of 4-byte entries (one 128-byte line per bucket, Section III-A).

The dictionary with every value 0 is the oracle: found and deleted flags,
the live count and the final key set must equal it, and every bucket entry
must sit in one of its two candidate buckets (BitHash1/2 modulo the bucket
count, from the oracle's transcriptions).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2510_15095_amd import workload as wl

pytestmark = pytest.mark.gpu

S = 32


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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def make_set(H, nb, **kw):
    return H.Table(nb, slots_per_bucket=S, entry_bits=32, **kw)


def zeros(n):
    return np.zeros(n, np.uint32)


def check_contents(t, o, nb):
    words, where = t.dump(with_where=True)
    assert np.array_equal(words, o.dump()), "key sets differ"
    keys = (words & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    inb = where >= 0
    c1 = np.array([oracle.bithash1(int(k)) % nb for k in keys[inb]], np.int64)
    c2 = np.array([oracle.bithash2(int(k)) % nb for k in keys[inb]], np.int64)
    bad = (where[inb] != c1) & (where[inb] != c2)
    assert not bad.any(), f"{bad.sum()} entries outside their candidate buckets"


@pytest.mark.parametrize("lf,E,stash", [(0.5, 8, 1024), (0.95, 8, 1024), (0.99, 2, 64), (0.995, 0, 8)])
def test_set_insert_lookup_delete(H, lf, E, stash):
    nb = 257
    n = int(S * nb * lf)
    case(f"set32 lf={lf} E={E} stash={stash}")
    ks = wl.KeyStream(200 + E)
    keys = ks.range(0, n)
    t = make_set(H, nb, max_evictions=E, stash_capacity=stash, pending_capacity=4096)
    o = oracle.O1()
    t.insert(dev(keys), dev(zeros(n)), flags=H.HIVE_UNIQUE)
    o.insert(keys, zeros(n))
    st = t.stats()
    assert st["status"] in (H.HIVE_OK, H.HIVE_WARN_PENDING) and st["live"] == n, st
    assert st["full_chains"] == st["stash_inserts"] + st["pending_inserts"], st
    q = ks.range(0, n + 500)
    _, f = t.lookup(dev(q))
    assert np.array_equal(host(f), o.lookup(q)[1])
    # inserting present keys again changes nothing
    t.insert(dev(keys[::2]), dev(zeros(keys[::2].size)), flags=H.HIVE_UNIQUE)
    assert t.stats()["live"] == n
    check_contents(t, o, nb)
    dk = keys[1::3]
    assert np.array_equal(host(t.delete(dev(dk), flags=H.HIVE_UNIQUE)), o.delete(dk))
    _, f = t.lookup(dev(q))
    assert np.array_equal(host(f), o.lookup(q)[1])
    assert t.stats()["live"] == len(o)
    check_contents(t, o, nb)
    t.close()


def test_set_repeats_reserved_keys_and_empty_batches(H):
    import torch
    case("set32 repeats")
    rng = np.random.default_rng(5)
    base = wl.KeyStream(210).range(0, 3000)
    keys = np.concatenate([base[rng.integers(0, base.size, 20000)], np.array([0, 0xFFFFFFFF], np.uint32)])
    t = make_set(H, 256)
    o = oracle.O1()
    t.insert(dev(keys), None)  # values are not read
    o.insert(keys, zeros(keys.size))
    assert t.stats()["live"] == len(o) and t.stats()["invalid_keys"] == 2
    dkeys = base[rng.integers(0, base.size, 5000)]
    assert np.array_equal(host(t.delete(dev(dkeys))), o.delete(dkeys))
    check_contents(t, o, 256)
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    t.insert(e, e)
    t.lookup(e)
    t.delete(e)
    assert t.stats()["live"] == len(o)
    t.close()


def test_set_mixed_batches(H):
    """Mixed batches (Zipf keys, repeated inserts, dedupe on): flags equal
    the dictionary's, inserts report 0."""
    nb, universe = 2048, 1 << 17
    ks = wl.KeyStream(220)
    pre = ks.keys(wl.DomainPerm(220, universe).sample(int(0.9 * nb * S)))
    t = make_set(H, nb, stash_capacity=4096)
    o = oracle.O1()
    t.insert(dev(pre), None, flags=H.HIVE_UNIQUE)
    o.insert(pre, zeros(pre.size))
    for b in range(5):
        case(f"set32 mixed batch {b}")
        mb = wl.mixed_batch(220, b, 1 << 14, universe, stream=ks)
        _, f = t.mixed(dev(mb["ops"]), dev(mb["keys"]), dev(mb["vals"]))
        _, of = o.apply(mb["ops"], mb["keys"], zeros(mb["keys"].size))
        assert np.array_equal(host(f), of), f"batch {b}"
        assert t.stats()["live"] == len(o)
    check_contents(t, o, nb)
    t.close()


def test_set_bulk_95pct(H):
    """2^22 unique keys into a set at 95% load, 50%-hit queries, delete
    half, re-query: expected flags from the generator's closed form, and the
    dump is exactly the inserted keys minus the deleted ones."""
    n = 1 << 22
    nb = int(np.ceil(n / (0.95 * S)))
    case(f"set32 bulk n={n} buckets={nb}")
    w = wl.bulk_workload(12, n)
    t = make_set(H, nb)
    t.insert(dev(w["ins_keys"]), None, flags=H.HIVE_UNIQUE)
    st = t.stats()
    assert st["live"] == n and st["status"] == H.HIVE_OK, st
    present = w["query_idx"] < n
    _, f = t.lookup(dev(w["query_keys"]))
    assert np.array_equal(host(f).astype(bool), present)
    d = t.delete(dev(w["del_keys"]), flags=H.HIVE_UNIQUE)
    assert host(d).all()
    deleted = np.zeros(n, bool)
    deleted[w["del_idx"]] = True
    still = present.copy()
    still[present] = ~deleted[w["query_idx"][present]]
    _, f = t.lookup(dev(w["query_keys"]))
    assert np.array_equal(host(f).astype(bool), still)
    words = t.dump()
    idx = w["stream"].index_of((words & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    assert idx.size == n - w["del_keys"].size and np.unique(idx).size == idx.size
    assert not deleted[idx].any() and (idx < n).all() and not (words >> np.uint64(32)).any()
    t.close()


def test_set_config_limits(H):
    for bad in (dict(slots_per_bucket=16), dict(addressing=1), dict(hash_pair=1), dict(probe_both=1)):
        cfg = dict(slots_per_bucket=S, entry_bits=32)
        cfg.update(bad)
        with pytest.raises(H.HiveError):
            H.Table(64, **cfg)
    t = make_set(H, 64)
    keys = wl.KeyStream(230).range(0, 1900)
    t.insert(dev(keys), None, flags=H.HIVE_UNIQUE)
    first, second, overflow = t.placement()
    assert first + second + overflow >= 1900 and first + second <= 1900 and first > second
    t.close()
