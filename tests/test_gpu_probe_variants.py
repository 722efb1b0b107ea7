"""GPU parity of the probe-kernel variants (hive_config.probe_tuning,
probe_grid): every variant of every operation kind, and probe launches
capped at a few blocks (each block then strides over many tiles, the last
one ragged), give the dictionary's results (O1).

A FIXED table of 16-slot buckets is built to 95% load (Section V-C-1's bulk
shape, scaled down so the oracle keeps up) with repeated keys in the insert
batch, then takes lookups with 50% hits, deletes of a third of the keys and
Zipf mixed batches with dedupe on.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2510_15095_amd import workload as wl

pytestmark = pytest.mark.gpu

NB = 4099
S = 16


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


def run_all_kinds(H, tuning, grid):
    n = int(0.95 * NB * S)
    ks = wl.KeyStream(400)
    keys = ks.range(0, n)
    rng = np.random.default_rng(401)
    # inserts with repeats (dedupe on): the last occurrence's value wins
    rep = keys[rng.integers(0, n, n // 8)]
    ins = np.concatenate([keys, rep])
    vals = wl.values_for(ins) ^ np.arange(ins.size, dtype=np.uint32)
    t = H.Table(NB, probe_tuning=tuning, probe_grid=grid, max_batch=ins.size)
    o = oracle.O1()
    t.insert(dev(ins), dev(vals))
    o.insert(ins, vals)
    st = t.stats()
    assert st["status"] == H.HIVE_OK and st["live"] == len(o) == n, st
    q = np.concatenate([keys[::2], ks.range(n, n + n // 2)])
    v, f = t.lookup(dev(q))
    ov, of = o.lookup(q)
    assert np.array_equal(host(f), of) and np.array_equal(host(v), ov), "lookup"
    dk = np.concatenate([keys[::3], ks.range(2 * n, 2 * n + 999)])
    assert np.array_equal(host(t.delete(dev(dk))), o.delete(dk)), "delete"
    for b in range(3):
        mb = wl.mixed_batch(402, b, 8_001, 2 * n, stream=ks, value_salt=b + 1)
        v, f = t.mixed(dev(mb["ops"]), dev(mb["keys"]), dev(mb["vals"]))
        ov, of = o.apply(mb["ops"], mb["keys"], mb["vals"])
        assert np.array_equal(host(f), of) and np.array_equal(host(v), ov), f"mixed batch {b}"
        assert t.stats()["live"] == len(o)
    assert np.array_equal(t.dump(), o.dump())
    t.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
def test_variant_matches_dictionary(H, variant):
    ins = variant if variant in H.PROBE_INSERT_VARIANTS else 0
    tuning = H.probe_tuning(insert=ins, delete=variant, lookup=variant, mixed=variant)
    case(f"probe variant {variant} {H.PROBE_VARIANTS[variant]} (insert {ins}) tuning={tuning:#x}")
    run_all_kinds(H, tuning, 0)


@pytest.mark.parametrize("grid", [1, 7, 300])
def test_capped_probe_grid_matches_dictionary(H, grid):
    # 1 block: every tile through one block; 7 and 300: strides with a
    # ragged remainder of tiles
    case(f"probe grid cap {grid}")
    run_all_kinds(H, H.probe_tuning(3, 2, 4, 1) if grid == 300 else 0, grid)
