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
