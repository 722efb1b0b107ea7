"""Host-side logic that needs no GPU: the serving loop's table and request
generators, and the autotuner's cache."""
from __future__ import annotations

import json
import math

import numpy as np
import pytest

from paper_2510_15095_amd import workload as wl


@pytest.fixture(scope="module")
def sv():
    from paper_2510_15095_amd import serve
    return serve


def test_table_specs_sizes_and_reservations(sv):
    specs = sv.make_specs(200, 7, log2_min=10, log2_max=16, load=0.85, headroom=1.25)
    assert [s.tid for s in specs] == list(range(200))
    for s in specs:
        assert 2 ** 10 <= s.n_keys <= 2 ** 16
        assert s.buckets == max(1, math.ceil(s.n_keys / (0.85 * 16)))
        assert s.arena == max(s.buckets + 1, math.ceil(s.buckets * 1.25))
        assert s.universe == 2 * s.n_keys
    # log-uniform sizes: the median sits near the geometric middle
    med = np.median([math.log2(s.n_keys) for s in specs])
    assert 12 < med < 14
    assert sv.footprint_bytes(specs) == sum(s.arena for s in specs) * 128
    again = sv.make_specs(200, 7, log2_min=10, log2_max=16)
    assert [(s.n_keys, s.seed) for s in again] == [(s.n_keys, s.seed) for s in specs]


def test_requests_shape_mix_and_determinism(sv):
    specs = sv.make_specs(16, 3, log2_min=10, log2_max=13)
    reqs = sv.make_requests(specs, 400, 3, rate=1000.0, log2_max_size=12)
    assert len(reqs) == 400
    arr = np.array([r.arrival for r in reqs])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    # Poisson arrivals at 1000/s: mean gap about 1 ms
    assert 0.7e-3 < np.diff(arr).mean() < 1.3e-3
    counts = np.zeros(3)
    for r in reqs:
        assert 1 <= r.n <= min(2 ** 12, specs[r.table].n_keys)
        assert r.ops.shape == r.keys.shape == r.vals.shape == (r.n,)
        assert r.n_ins == int((r.ops == wl.OP_INSERT).sum())
        # one op type per key within a request
        for a in (wl.OP_INSERT, wl.OP_DELETE):
            ka = set(r.keys[r.ops == a].tolist())
            kb = set(r.keys[(r.ops != a)].tolist())
            assert not (ka & kb)
        assert len(set(r.keys[r.ops == wl.OP_DELETE].tolist())) == int((r.ops == wl.OP_DELETE).sum())
        counts += [(r.ops == o).sum() for o in (wl.OP_INSERT, wl.OP_DELETE, wl.OP_LOOKUP)]
    frac = counts / counts.sum()
    assert abs(frac[0] - 0.25) < 0.03 and abs(frac[1] - 0.25) < 0.03 and abs(frac[2] - 0.5) < 0.03
    again = sv.make_requests(specs, 400, 3, rate=1000.0, log2_max_size=12)
    for a, b in zip(reqs, again):
        assert a.table == b.table and a.n == b.n and np.array_equal(a.keys, b.keys)
        assert np.array_equal(a.ops, b.ops) and np.array_equal(a.vals, b.vals)


def test_requests_all_at_once_when_rate_is_zero(sv):
    specs = sv.make_specs(4, 1, log2_min=10, log2_max=11)
    reqs = sv.make_requests(specs, 50, 1, rate=0, log2_max_size=8)
    assert all(r.arrival == 0.0 for r in reqs)


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    from paper_2510_15095_amd import autotune
    path = tmp_path / "tuned.json"
    monkeypatch.setenv("HIVE_TUNE_CACHE", str(path))
    monkeypatch.setattr(autotune, "gpu_arch", lambda: "gfx950")
    monkeypatch.setattr(autotune, "SHIPPED_DIR", str(tmp_path / "none"))
    assert autotune.load("resize") is None
    path.write_text(json.dumps({"gfx950": {"resize": {"resize_k": 256}},
                                "gfx942": {"resize": {"resize_k": 64}}}))
    assert autotune.load("resize") == {"resize_k": 256}
    assert autotune.load("executor") is None
    path.write_text("not json")
    assert autotune.load("resize") is None


def test_autotune_falls_back_to_shipped_values(tmp_path, monkeypatch):
    """Without a cache on this machine, load() returns the values shipped for
    the architecture; a cached section takes precedence.  The shipped probe
    word is one the library accepts (one known variant per kind, inserts
    only the variants without register spills)."""
    from paper_2510_15095_amd import autotune
    from paper_2510_15095_amd import hive as H
    monkeypatch.setenv("HIVE_TUNE_CACHE", str(tmp_path / "absent.json"))
    monkeypatch.setattr(autotune, "gpu_arch", lambda: "gfx950")
    pk = autotune.load("probe_kernel")
    assert pk is not None and 0 <= pk["probe_grid"] <= 1 << 20
    word = pk["probe_tuning"]
    nib = [(word >> (4 * i)) & 15 for i in range(4)]
    assert word >> 16 == 0 and nib[0] in H.PROBE_INSERT_VARIANTS and all(x < len(H.PROBE_VARIANTS) for x in nib)
    assert [tuple(pk["variants"][k]) for k in H.PROBE_KINDS] == [H.PROBE_VARIANTS[x] for x in nib]
    assert autotune.load("resize")["resize_k"] >= 1
    (tmp_path / "absent.json").write_text(json.dumps({"gfx950": {"resize": {"resize_k": 64}}}))
    assert autotune.load("resize") == {"resize_k": 64}
    monkeypatch.setattr(autotune, "gpu_arch", lambda: "gfx90a")
    assert autotune.load("probe_kernel") is None


def test_autotune_keeps_default_within_margin():
    from paper_2510_15095_amd import autotune
    assert autotune._pick({0: 100.0, 1: 101.9, 2: 99.0}, 0) == 0
    assert autotune._pick({0: 100.0, 1: 102.1, 2: 103.0}, 0) == 2
    assert autotune._pick({16: 50.0, 32: 40.0}, 16) == 16
