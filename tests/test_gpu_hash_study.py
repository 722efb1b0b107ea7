"""Hash-function study on the GPU against the oracle (Section III-C): every
key's bucket bit-exact for each hash, and the collision count Y exact, at
sizes up to the study's largest (2048^2 keys over 512^2 buckets)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2510_15095_amd import workload as wl

pytestmark = pytest.mark.gpu

KINDS = ("bithash1", "bithash2", "crc32", "crc64", "murmur3", "city32")
EDGE = np.array([0, 1, 2, 0x7F, 0x80, 0xFF, 0x7F7F7F7F, 0x80808080, 0xFF000000, 0x00FF00FF, 0xFFFFFFFE, 0xFFFFFFFF],
                np.uint32)


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


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("m", [512 * 512, 4415057, 1, 3])
def test_buckets_match_oracle(H, kind, m):
    import torch
    keys = np.concatenate([EDGE, wl.KeyStream(91).range(0, 100_000), np.arange(1, 5000, dtype=np.uint32)])
    out = torch.empty(keys.size, dtype=torch.uint32, device="cuda")
    print(f"[case] buckets {kind} m={m}", flush=True)
    H.hive_hash_buckets(kind, dev(keys), m, out)
    assert np.array_equal(out.cpu().numpy(), oracle.hash_buckets(kind, keys, m))


@pytest.mark.parametrize("kind", KINDS)
def test_collisions_match_oracle(H, kind):
    import torch
    m = 512 * 512
    scratch = torch.empty(2 + m // 32, dtype=torch.uint32, device="cuda")
    uniform = wl.KeyStream(92).range(0, 2048 * 2048)
    sequential = np.arange(1, 2048 * 2048 + 1, dtype=np.uint32)
    for name, keys in (("uniform", uniform), ("sequential", sequential)):
        for n in (0, 1, 512, 8192, 262144, 2048 * 2048):
            print(f"[case] collisions {kind} {name} n={n}", flush=True)
            got = H.hive_hash_collisions(kind, dev(keys[:max(n, 1)])[:n], m, scratch)
            want = oracle.collisions(oracle.hash_buckets(kind, keys[:n], m), m)
            assert got == want, (name, n)
    # one bucket: every key but the first collides
    scratch1 = torch.empty(3, dtype=torch.uint32, device="cuda")
    assert H.hive_hash_collisions(kind, dev(uniform[:1000]), 1, scratch1) == 999


def test_unaligned_and_ragged_arrays_take_the_scalar_path(H):
    import torch
    keys = wl.KeyStream(93).range(0, 10_007)
    d = dev(keys)
    for kind in KINDS:
        out = torch.zeros(keys.size, dtype=torch.uint32, device="cuda")
        print(f"[case] unaligned {kind}", flush=True)
        H.hive_hash_buckets(kind, d[1:], 4415057, out[1:])  # 4-byte offsets: not 16-byte aligned
        assert np.array_equal(out[1:].cpu().numpy(), oracle.hash_buckets(kind, keys[1:], 4415057))
        assert int(out[0]) == 0
        H.hive_hash_buckets(kind, d[:7], 512 * 512, out[:7])  # fewer than one 4-key group past 4
        assert np.array_equal(out[:7].cpu().numpy(), oracle.hash_buckets(kind, keys[:7], 512 * 512))


def pair_candidates(pair, keys, nb):
    """The candidate buckets of every key under a table's hash choice, from
    the oracle's transcriptions (CRC-64 contributes its low 32 bits; the
    three-candidate choice is BitHash1, BitHash2 and CityHash32)."""
    le = [int(k).to_bytes(4, "little") for k in keys]
    if pair == 1:
        hs = [[oracle.crc32_bytes(b) for b in le], [oracle.crc64_bytes(b) & 0xFFFFFFFF for b in le]]
    elif pair == 2:
        hs = [[oracle.murmur3_bytes(b, 0) for b in le], [oracle.city32_bytes(b) for b in le]]
    else:
        hs = [[oracle.bithash1(int(k)) for k in keys], [oracle.bithash2(int(k)) for k in keys],
              [oracle.city32_bytes(b) for b in le]]
    return [np.array(h, np.int64) % nb for h in hs]


def check_in_candidates(t, pair, nb, o):
    words, where = t.dump(with_where=True)
    assert np.array_equal(words, o.dump())
    k = (words & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    cands = pair_candidates(pair, k, nb)
    inb = where >= 0
    ok = np.zeros(int(inb.sum()), bool)
    for c in cands:
        ok |= where[inb] == c[inb]
    assert ok.all(), f"{(~ok).sum()} entries outside their candidate buckets"


@pytest.mark.parametrize("pair", [1, 2, 3])
@pytest.mark.parametrize("lf,E,stash", [(0.5, 8, 1024), (0.97, 8, 1024), (0.99, 2, 64)])
def test_table_with_other_hash_pair_matches_oracle(H, pair, lf, E, stash):
    """A FIXED table addressed by CRC-32/CRC-64, MurmurHash3/CityHash32 or
    three candidates (BitHash1, BitHash2, CityHash32): every lookup, delete
    and the final contents equal the dictionary's, and every bucket entry
    sits in one of its candidates under that choice."""
    S, nb = 16, 97
    n = int(S * nb * lf)
    ks = wl.KeyStream(95 + pair)
    keys = ks.range(0, n)
    vals = wl.values_for(keys)
    print(f"[case] pair {pair} lf {lf} E {E} stash {stash}", flush=True)
    t = H.Table(nb, hash_pair=pair, max_evictions=E, stash_capacity=stash, pending_capacity=4096)
    o = oracle.O1()
    t.insert(dev(keys), dev(vals))
    o.insert(keys, vals)
    st = t.stats()
    assert st["status"] in (H.HIVE_OK, H.HIVE_WARN_PENDING) and st["live"] == n, st
    q = ks.range(0, n + 300)
    v, f = t.lookup(dev(q))
    ov, of = o.lookup(q)
    assert np.array_equal(f.cpu().numpy(), of) and np.array_equal(v.cpu().numpy(), ov)
    check_in_candidates(t, pair, nb, o)
    dk = keys[::3]
    assert np.array_equal(t.delete(dev(dk), flags=H.HIVE_UNIQUE).cpu().numpy(), o.delete(dk))
    v, f = t.lookup(dev(q))
    ov, of = o.lookup(q)
    assert np.array_equal(f.cpu().numpy(), of) and np.array_equal(v.cpu().numpy(), ov)
    assert np.array_equal(t.dump(), o.dump())
    with pytest.raises(H.HiveError):
        t.placement()
    t.close()


@pytest.mark.parametrize("pair", [1, 2, 3])
def test_mixed_batches_under_other_hash_choices(H, pair):
    """Mixed batches (Zipf keys with repeated inserts, deletes, lookups, dedupe
    on) on a FIXED table at about 90% load under each hash choice: outputs,
    key counts and contents equal the dictionary's, entries in candidates."""
    S, nb, universe = 16, 2048, 1 << 16
    ks = wl.KeyStream(120 + pair)
    pre = ks.keys(wl.DomainPerm(120 + pair, universe).sample(int(0.88 * nb * S)))
    t = H.Table(nb, hash_pair=pair, stash_capacity=2048, pending_capacity=2048)
    o = oracle.O1()
    t.insert(dev(pre), dev(wl.values_for(pre)), flags=H.HIVE_UNIQUE)
    o.insert(pre, wl.values_for(pre))
    for b in range(4):
        print(f"[case] pair {pair} mixed batch {b}", flush=True)
        mb = wl.mixed_batch(120 + pair, b, 1 << 13, universe, stream=ks, value_salt=b + 1)
        v, f = t.mixed(dev(mb["ops"]), dev(mb["keys"]), dev(mb["vals"]))
        ov, of = o.apply(mb["ops"], mb["keys"], mb["vals"])
        assert np.array_equal(f.cpu().numpy(), of) and np.array_equal(v.cpu().numpy(), ov), f"batch {b}"
        assert t.stats()["live"] == len(o)
    check_in_candidates(t, pair, nb, o)
    t.close()


def test_executor_refuses_other_hash_pairs(H):
    import torch
    t = H.Table(64, hash_pair=1)
    d = H.hive_drain_create(16, 0, 8, 2, 0)
    k = dev(np.arange(1, 65, dtype=np.uint32))
    with pytest.raises(H.HiveError):
        H.hive_drain_submit(d, t.h, H.HIVE_OP_LOOKUP, k, None, None, torch.empty(64, dtype=torch.uint32,
                                                                                 device="cuda"))
    H.hive_drain_destroy(d)
    t.close()


def test_gather_lines_xor_of_each_line(H):
    """The gather-ceiling kernel: out[i] is the XOR of the 16 words of line
    idx[i]; an index past the table gives 0; ragged lengths are covered."""
    import torch
    rng = np.random.default_rng(11)
    n_lines = 5003
    table = rng.integers(0, 2 ** 63, size=(n_lines, 16), dtype=np.int64).view(np.uint64)
    idx = rng.integers(0, n_lines, size=100_003).astype(np.uint32)
    idx[::997] = n_lines + 7  # past the table
    out = torch.empty(idx.size, dtype=torch.uint64, device="cuda")
    H.hive_gather_lines(dev(table.reshape(-1)), dev(idx), out)
    safe = np.minimum(idx, n_lines - 1)
    want = np.bitwise_xor.reduce(table[safe], axis=1)
    want[idx >= n_lines] = 0
    assert np.array_equal(out.cpu().numpy(), want)
