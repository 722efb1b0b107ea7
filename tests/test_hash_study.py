"""Pins of the hash-study oracle (Section III-C): the hash transcriptions
against published check values, the collision count against its definition,
and the uniform-hashing expectation against exact enumeration."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle


def test_crc32_check_value():
    # the standard check value of the reflected 0x04C11DB7 CRC (zlib, IEEE 802.3)
    assert oracle.crc32_bytes(b"123456789") == 0xCBF43926
    assert oracle.crc32_bytes(b"") == 0


def test_crc64_check_value():
    # the check value of CRC-64/XZ (ECMA-182 polynomial, reflected, all-ones init and xor)
    assert oracle.crc64_bytes(b"123456789") == 0x995DC9BBDF1939FA
    assert oracle.crc64_bytes(b"") == 0


@pytest.mark.parametrize("data,seed,want", [
    (b"", 0, 0x00000000),
    (b"", 1, 0x514E28B7),
    (b"", 0xFFFFFFFF, 0x81F16F39),
    (b"\0\0\0\0", 0, 0x2362F9DE),
    (b"aaaa", 0x9747B28C, 0x5A97808A),
    (b"abc", 0, 0xB3DD93FA),
    (b"Hello, world!", 0x9747B28C, 0x24884CBA),
])
def test_murmur3_published_vectors(data, seed, want):
    assert oracle.murmur3_bytes(data, seed) == want


def test_city32_empty_input():
    # CityHash32 of the empty string, as checked by published ports; it pins
    # the mixing rounds and the finalizer, not the folding of input bytes
    assert oracle.city32_bytes(b"") == 0xDC56D17A


def test_city32_folds_bytes_as_signed():
    # a byte >= 0x80 enters as a negative signed char: 0x80 folds as
    # 0xFFFFFF80, so it differs from any positive byte's contribution
    assert oracle.city32_bytes(b"\x80") != oracle.city32_bytes(b"\x7f")
    assert len({oracle.city32_bytes(bytes([b])) for b in range(256)}) == 256


def test_key_buckets_use_little_endian_bytes():
    keys = np.array([0, 1, 0x12345678, 0xFFFFFFFE, 0x80808080], np.uint32)
    m = 1000003
    le = [int(k).to_bytes(4, "little") for k in keys]
    assert list(oracle.hash_buckets("crc32", keys, m)) == [oracle.crc32_bytes(b) % m for b in le]
    assert list(oracle.hash_buckets("crc64", keys, m)) == [oracle.crc64_bytes(b) % m for b in le]
    assert list(oracle.hash_buckets("murmur3", keys, m)) == [oracle.murmur3_bytes(b, 0) % m for b in le]
    assert list(oracle.hash_buckets("city32", keys, m)) == [oracle.city32_bytes(b) % m for b in le]
    assert list(oracle.hash_buckets("bithash1", keys, m)) == [oracle.bithash1(int(k)) % m for k in keys]
    assert list(oracle.hash_buckets("bithash2", keys, m)) == [oracle.bithash2(int(k)) % m for k in keys]
    with pytest.raises(ValueError):
        oracle.hash_buckets("crc32", keys, 0)


def test_collision_count_definition():
    # loads 2, 1, 0, 3 over four buckets: (2-1) + 0 + 0 + (3-1) = 3
    assert oracle.collisions([0, 0, 1, 3, 3, 3], 4) == 3
    assert oracle.collisions([], 4) == 0
    assert oracle.collisions(list(range(10)), 10) == 0
    # Y = n - (occupied buckets), for any assignment
    rng = np.random.default_rng(1)
    b = rng.integers(0, 50, 200)
    assert oracle.collisions(b, 50) == 200 - len(set(b.tolist()))


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (2, 3), (3, 4), (4, 3), (5, 5)])
def test_expected_collisions_equals_enumeration(m, n):
    total = 0
    for assign in itertools.product(range(m), repeat=n):
        total += n - len(set(assign))
    exact = total / m ** n
    assert oracle.expected_collisions(n, m) == pytest.approx(exact, rel=1e-12, abs=1e-12)


def test_expected_collisions_limits():
    m = 512 * 512
    assert oracle.expected_collisions(0, m) == 0.0
    assert oracle.expected_collisions(1, m) == pytest.approx(0.0, abs=1e-9)
    # n << m: E[Y] ~ n^2 / (2m) (the theorem's Poisson limit)
    n = 512
    assert oracle.expected_collisions(n, m) == pytest.approx(n * n / (2 * m), rel=0.01)
    # one bucket: every key after the first collides
    assert oracle.expected_collisions(7, 1) == pytest.approx(6.0)


def test_uniform_random_buckets_agree_with_expectation():
    # a seeded uniform assignment stands in for an ideal hash: CSR near 1
    m, n = 4096, 8192
    b = np.random.default_rng(5).integers(0, m, n)
    csr = oracle.expected_collisions(n, m) / oracle.collisions(b, m)
    assert 0.95 < csr < 1.05


@pytest.mark.parametrize("n,m", [(0, 7), (1, 7), (5, 1), (512, 512 * 512), (2048 * 2048, 512 * 512),
                                 (10 ** 6, 4415057)])
def test_package_expectation_equals_oracle(n, m):
    from paper_2510_15095_amd import hash_study as hs
    assert hs.expected_collisions(n, m) == pytest.approx(oracle.expected_collisions(n, m), rel=1e-12, abs=1e-9)


def test_csr_definition():
    from paper_2510_15095_amd import hash_study as hs
    assert hs.csr(100, 10, 0) == float("inf")
    assert hs.csr(8192, 4096, 4000) == pytest.approx(oracle.expected_collisions(8192, 4096) / 4000)

