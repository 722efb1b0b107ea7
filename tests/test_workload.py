"""Pins for the seeded workload generator (shared by oracle and GPU tests)."""
import numpy as np
import pytest

from paper_2510_15095_amd import workload as wl


def test_keystream_native_matches_numpy_and_inverts():
    for seed in (1, 2, 3, 0xDEADBEEF):
        ks, ksn = wl.KeyStream(seed), wl.KeyStream(seed, native=False)
        rng = np.random.default_rng(seed)
        idx = np.concatenate([np.arange(4096), rng.integers(0, wl.KeyStream.N_VALID, 4096),
                              [wl.KeyStream.N_VALID - 1, ks._a, ks._b, ks._a - 1, ks._b - 1]])
        idx = idx[(idx >= 0) & (idx < wl.KeyStream.N_VALID)]
        k = ks.keys(idx)
        assert np.array_equal(k, ksn.keys(idx))
        assert np.array_equal(ks.index_of(k), idx)
        assert np.array_equal(ksn.index_of(k), idx)
        assert not np.any((k == 0) | (k == 0xFFFFFFFF))


def test_keystream_is_injective_on_a_large_prefix():
    k = wl.KeyStream(2).range(0, 1 << 22)
    assert np.unique(k).size == k.size


def test_keystream_skips_reserved_keys_exactly():
    ks = wl.KeyStream(5)
    # the two reserved images are skipped: the index just below each skip
    # and just above map to valid, distinct keys
    around = np.array([ks._a - 1, ks._a, ks._b - 2, ks._b - 1], np.int64)
    around = around[around >= 0]
    k = ks.keys(around)
    assert np.unique(k).size == k.size and not np.any((k == 0) | (k == 0xFFFFFFFF))


def test_splitmix64_stream_is_successive_outputs():
    # SplitMix64: state += golden; output = mix(state).  Output i of a stream
    # seeded with s therefore equals the first output seeded with
    # s + i * golden.
    golden = 0x9E3779B97F4A7C15
    s = 12345
    stream = wl.splitmix64_stream(s, 5)
    for i in range(5):
        assert int(stream[i]) == int(wl.splitmix64_first(np.uint64((s + i * golden) % (1 << 64))))


def test_values_native_matches_numpy():
    k = wl.KeyStream(9).range(0, 100000)
    assert np.array_equal(wl.values_for(k), wl.values_for(k, native=False))


def test_zipf_matches_pmf_small_n():
    z = wl.Zipf(16, 0.99)
    rng = np.random.default_rng(7)
    n = 400000
    s = z.sample(rng, n)
    assert s.min() >= 1 and s.max() <= 16
    freq = np.bincount(s, minlength=17)[1:] / n
    p = z.pmf(np.arange(1, 17))
    # each frequency within 5 standard errors of the exact probability
    se = np.sqrt(p * (1 - p) / n)
    assert np.all(np.abs(freq - p) < 5 * se)


def test_zipf_large_universe_head_mass():
    n_univ = 1 << 26
    z = wl.Zipf(n_univ, 0.99)
    s = z.sample(np.random.default_rng(1), 1 << 20)
    # P(rank 1) = 1 / sum_{k<=N} k^-0.99; the sum is evaluated directly
    harmonic = np.sum(np.arange(1, n_univ + 1, dtype=np.float64) ** -0.99)
    p1 = 1.0 / harmonic
    freq1 = np.mean(s == 1)
    assert abs(freq1 - p1) < 5 * np.sqrt(p1 * (1 - p1) / s.size)


def test_domain_perm_is_a_permutation():
    for n in (1, 2, 3, 17, 1000, 4096, 100003):
        d = wl.DomainPerm(11, n)
        a = d(np.arange(n))
        assert np.array_equal(np.sort(a), np.arange(n))
        assert np.array_equal(a, d(np.arange(n), native=False))


def test_bulk_workload_shape_and_membership():
    w = wl.bulk_workload(4, 5000, n_queries=3001, n_deletes=2500)
    assert w["ins_keys"].size == 5000 and np.unique(w["ins_keys"]).size == 5000
    assert np.array_equal(w["ins_vals"], wl.values_for(w["ins_keys"]))
    present = w["query_idx"] < 5000
    assert present.sum() == 1500
    assert np.unique(w["del_keys"]).size == 2500
    assert np.all(w["del_idx"] < 5000)
    assert np.array_equal(w["stream"].keys(w["query_idx"]), w["query_keys"])


def test_tiny_workload_is_deterministic():
    a, b = wl.tiny_workload(1), wl.tiny_workload(1)
    for k in ("ins_keys", "ins_vals", "query_keys", "del_keys"):
        assert np.array_equal(a[k], b[k])
    assert a["ins_keys"].size == 1 << 16 and a["del_keys"].size == 1 << 15


@pytest.mark.parametrize("zipf_s", [0.99, None])
def test_mixed_batch_counts_and_disjointness(zipf_s):
    b = wl.mixed_batch(3, 0, 20000, 1 << 16, zipf_s=zipf_s)
    ops, ranks = b["ops"], b["ranks"]
    assert (ops == wl.OP_INSERT).sum() == 8000 and (ops == wl.OP_DELETE).sum() == 8000
    types_per_rank = {}
    for o, r in zip(ops.tolist(), ranks.tolist()):
        types_per_rank.setdefault(r, set()).add(o)
    assert all(len(t) == 1 for t in types_per_rank.values())
    del_ranks = ranks[ops == wl.OP_DELETE]
    assert np.unique(del_ranks).size == del_ranks.size


@pytest.mark.parametrize("zipf_s", [0.99, 0.5, 1.2, None])
def test_mixed_batch_native_equals_reference(zipf_s):
    """The C generator equals the pure-Python statement of the same steps
    (stream, shuffle, rank draws, disjointness redraws, keys, values),
    including universes small enough that many ranks are redrawn."""
    for seed, b, n, u in [(3, 0, 5000, 1 << 16), (7, 2, 3000, 4000), (11, 1, 1, 5), (5, 5, 20000, 1 << 26),
                          (9, 3, 600, 700)]:
        a = wl.mixed_batch(seed, b, n, u, zipf_s=zipf_s, value_salt=b)
        r = wl.mixed_batch_reference(seed, b, n, u, zipf_s=zipf_s, value_salt=b)
        for f in ("ops", "keys", "vals", "ranks"):
            assert np.array_equal(a[f], r[f]), (seed, b, n, u, f)


def test_mixed_batches_equal_one_at_a_time():
    jobs = [dict(seed=4, batch=b, n_ops=n, universe=1 << 16, zipf_s=z)
            for b, (n, z) in enumerate([(4096, 0.99), (0, None), (77, None), (9000, 0.99)])]
    many = wl.mixed_batches(jobs)
    for j, m in zip(jobs, many):
        one = wl.mixed_batch(**j)
        for f in ("ops", "keys", "vals", "ranks"):
            assert np.array_equal(m[f], one[f])


def test_mixed_batch_ranks_follow_zipf():
    """All-insert batches (no disjointness redraws): the native sampler's
    ranks follow the Zipf pmf (chi-square over the first ranks + the tail)."""
    n, N = 400_000, 1000
    r = wl.mixed_batch(21, 0, n, N, frac_insert=1.0, frac_delete=0.0)["ranks"]
    pmf = wl.Zipf(N, 0.99).pmf(np.arange(1, N + 1))
    head = 50
    obs = np.concatenate([np.bincount(r, minlength=N + 1)[1:head + 1], [np.sum(r > head)]])
    exp = np.concatenate([pmf[:head], [pmf[head:].sum()]]) * n
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < 100.0, chi2  # 50 degrees of freedom: p < 1e-4 beyond ~ 95
