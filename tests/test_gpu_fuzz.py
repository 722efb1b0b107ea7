"""Differential fuzz of the HIP path against the dictionary.

Each seed draws a small table configuration -- FIXED or LINEAR addressing
(with random pre- and post-batch rules and resize step K), 16, 32 or 64
slots per bucket, eviction bound, stash and pending capacities, 64-bit
entries or key-only sets of 32-bit entries, plain launches or the
persistent executor -- fills it close to full, then runs Zipf mixed batches
with repeated keys and dedupe on, comparing every output and the key count
with the dictionary after every batch and the contents at the end.  The
seeds run are FUZZ_SEEDS="first:last" (environment; default a short range
that the GPU suite runs every time).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2510_15095_amd import workload as wl

pytestmark = pytest.mark.gpu


def seed_range():
    a, b = os.environ.get("FUZZ_SEEDS", "0:8").split(":")
    return range(int(a), int(b))


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


def draw_config(rng, H):
    kind = rng.choice(["fixed", "linear", "set32"], p=[0.4, 0.45, 0.15])
    cfg = dict(max_evictions=int(rng.integers(0, 9)), stash_capacity=int(rng.choice([4, 16, 64, 256, 1024])),
               pending_capacity=4096)
    if kind == "set32":
        cfg.update(slots_per_bucket=32, entry_bits=32)
        nb = int(rng.integers(8, 200))
    elif kind == "fixed":
        cfg.update(slots_per_bucket=int(rng.choice([16, 16, 32, 64])))
        nb = int(rng.integers(8, 200))
    else:
        nb = int(rng.integers(4, 64))
        cfg.update(slots_per_bucket=16, addressing=H.HIVE_LINEAR, max_buckets=nb * 64,
                   resize_k=int(rng.choice([1, 3, 16, 64])), pre_expand=int(rng.integers(0, 2)), post_policy=1,
                   lf_expand_pct=int(rng.choice([85, 90, 95])), lf_contract_pct=int(rng.choice([10, 25])))
    path = "plain" if kind == "set32" or cfg.get("slots_per_bucket") != 16 else rng.choice(["plain", "persistent"])
    return kind, nb, cfg, path


@pytest.mark.parametrize("seed", list(seed_range()))
def test_fuzz_against_dictionary(H, seed):
    import torch
    rng = np.random.default_rng(1_000_003 + seed)
    kind, nb, cfg, path = draw_config(rng, H)
    S = cfg["slots_per_bucket"]
    set32 = kind == "set32"
    grows = kind == "linear" and cfg["pre_expand"] == 1
    fill = float(rng.uniform(0.3, 1.5)) if grows else float(rng.uniform(0.85, 0.99))
    if kind == "linear" and not grows:
        fill = float(rng.uniform(0.5, 0.9))
    n_pre = max(1, int(fill * nb * S))
    universe = max(4 * n_pre, 4096)
    n_batches = int(rng.integers(3, 7))
    n_ops = int(rng.choice([64, 257, 1000, 4096]))
    if grows and nb >= 48 and rng.random() < 0.5:
        # ten dedupe chunks over two segments; the universe leaves room for
        # a batch's per-type disjoint keys, and its 40,000 keys fit the
        # table's growth room (at least 49,152 slots)
        n_ops = 20_000
        universe = max(universe, 2 * n_ops)
    if not grows:
        # the new keys of all batches must fit the free slots, the stash and
        # the pending list of a table that cannot grow before a batch
        room = (1.0 - fill) * nb * S + cfg["stash_capacity"] + cfg["pending_capacity"]
        n_ops = max(16, min(n_ops, int(room / (n_batches * 0.6))))
    print(f"[case] fuzz seed {seed}: {kind} nb={nb} {cfg} path={path} prefill={n_pre} {n_batches} batches of "
          f"{n_ops} ops", flush=True)
    sys.stdout.flush()
    t = H.Table(nb, **cfg)
    o = oracle.O1()
    ks = wl.KeyStream(5000 + seed)
    pre = ks.keys(wl.DomainPerm(5000 + seed, universe).sample(n_pre))
    pv = np.zeros(n_pre, np.uint32) if set32 else wl.values_for(pre)
    t.insert(dev(pre), dev(pv), flags=H.HIVE_UNIQUE)
    o.insert(pre, pv)
    assert t.stats()["status"] >= 0
    drain = H.hive_drain_create(16, int(rng.integers(0, 2)), 16, 2, 10_000_000) if path == "persistent" else None
    for b in range(n_batches):
        mb = wl.mixed_batch(5000 + seed, b, n_ops, universe, frac_insert=float(rng.choice([0.25, 0.4, 0.6])),
                            frac_delete=0.3, zipf_s=float(rng.choice([0.99, 0.5])) if rng.random() < 0.7 else None,
                            stream=ks, value_salt=b + 1)
        vals = np.zeros(n_ops, np.uint32) if set32 else mb["vals"]
        if drain is None:
            v, f = t.mixed(dev(mb["ops"]), dev(mb["keys"]), dev(vals))
        else:
            o_, k_, v_ = dev(mb["ops"]), dev(mb["keys"]), dev(vals)
            v = torch.empty(n_ops, dtype=torch.uint32, device="cuda")
            f = torch.empty(n_ops, dtype=torch.uint8, device="cuda")
            tk = H.hive_drain_submit(drain, t.h, H.HIVE_OP_MIXED, k_, v_, o_, v, f)
            H.hive_drain_launch(drain, 0)
            torch.cuda.synchronize()
            assert H.hive_drain_poll(drain, tk)
        ov, of = o.apply(mb["ops"], mb["keys"], vals)
        assert np.array_equal(f.cpu().numpy(), of), f"seed {seed} batch {b}: flags differ"
        if not set32:
            assert np.array_equal(v.cpu().numpy(), ov), f"seed {seed} batch {b}: values differ"
        st = t.stats()
        assert st["status"] >= 0, (seed, b, st)
        assert st["live"] == len(o), f"seed {seed} batch {b}: key count {st['live']} vs {len(o)}"
    if drain is not None:
        H.hive_drain_destroy(drain)
    assert np.array_equal(t.dump(), o.dump()), f"seed {seed}: contents differ"
    t.close()
