"""The allocation-free mixed batch (hive_mixed_batch_noalloc) against
hive_mixed_batch and the dictionary.

Two tables built the same way take the same batches, one through each entry
point: per-operation outputs, contents and geometry must be equal, and equal
to the dictionary's.  The second call is smaller than the first, so it runs
on the shared scratch array that the first call left filled.  The tables are
LINEAR with the pre- and post-batch rules at 95% load, so the calls also
split, drain the stash and re-place it.
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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def test_noalloc_equals_mixed_batch_and_dictionary(H):
    import torch
    S, nb, universe = 16, 8192, 1 << 20
    big, small = (1 << 17) + 333, (1 << 13) + 77

    def table():
        return H.Table(nb, addressing=H.HIVE_LINEAR, max_buckets=4 * nb, lf_expand_pct=95, pre_expand=1,
                       post_policy=1, resize_k=64, stash_capacity=4096, max_batch=big)

    ks = wl.KeyStream(123)
    pre = ks.keys(wl.DomainPerm(123, universe).sample(int(0.94 * nb * S)))
    ref, na = table(), table()
    o1 = oracle.O1()
    for t in (ref, na):
        t.insert(dev(pre), dev(wl.values_for(pre)), flags=H.HIVE_UNIQUE)
    o1.insert(pre, wl.values_for(pre))
    for b, n in enumerate((big, small, small // 3)):
        mb = wl.mixed_batch(123, b, n, universe, stream=ks, value_salt=b + 1)
        ops, keys, vals = dev(mb["ops"]), dev(mb["keys"]), dev(mb["vals"])
        case(f"noalloc batch {b}: {n} mixed ops")
        rv, rf = ref.mixed(ops, keys, vals)
        nv = torch.full((n,), 7, dtype=torch.uint32, device="cuda")
        nf = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
        H.hive_mixed_batch_noalloc(na.h, ops, keys, vals, nv, nf)
        ov, of = o1.apply(mb["ops"], mb["keys"], mb["vals"])
        assert np.array_equal(host(nf), host(rf)) and np.array_equal(host(nv), host(rv)), f"batch {b}"
        assert np.array_equal(host(nf), of) and np.array_equal(host(nv), ov), f"batch {b}"
        sr, sn = ref.stats(), na.stats()
        assert sn["status"] == H.HIVE_OK, sn
        geo = lambda s: (s["n_buckets"], s["index_mask"], s["split_ptr"])  # noqa: E731
        assert geo(sn) == geo(sr) and sn["live"] == sr["live"] == len(o1)
        assert np.array_equal(na.dump(), o1.dump())
    assert na.stats()["n_buckets"] > nb, "the batches never split the table"
    for t in (ref, na):
        t.close()


def test_noalloc_refuses_what_would_allocate(H):
    import torch
    n = (1 << 22) + 1
    t = H.Table(1024, max_batch=1 << 12)
    ops = torch.full((n,), H.HIVE_OP_LOOKUP, dtype=torch.uint8, device="cuda")
    keys = torch.arange(1, n + 1, dtype=torch.int64, device="cuda").to(torch.uint32)
    vout = torch.empty(n, dtype=torch.uint32, device="cuda")
    fout = torch.empty(n, dtype=torch.uint8, device="cuda")
    case("noalloc: batch beyond the table's worklist")
    with pytest.raises(H.HiveError) as e:
        H.hive_mixed_batch_noalloc(t.h, ops[:5000], keys[:5000], keys[:5000], vout, fout)
    assert e.value.status == H.HIVE_ERR_BUDGET
    t.close()
    t = H.Table(1024, max_batch=n)
    case("noalloc: dedupe beyond the scratch array")
    with pytest.raises(H.HiveError) as e:
        H.hive_mixed_batch_noalloc(t.h, ops, keys, keys, vout, fout)
    assert e.value.status == H.HIVE_ERR_BUDGET
    # the same batch without dedupe needs no scratch: all lookups miss
    H.hive_mixed_batch_noalloc(t.h, ops, keys, keys, vout, fout, flags=H.HIVE_UNIQUE)
    assert not host(fout).any() and (host(vout) == M32).all()
    assert t.stats()["live"] == 0
    t.close()
