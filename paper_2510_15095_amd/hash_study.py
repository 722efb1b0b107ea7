"""The hash-function study of Section III-C: collision counts measured on
the GPU (hive_hash_collisions) against the uniform-hashing expectation.

For n keys thrown independently and uniformly into m buckets the theorem
there gives E[Y] = n - m (1 - (1 - 1/m)^n) for Y = sum over buckets of
(load - 1)+; the collision speedup ratio CSR = E[Y] / Y is 1 for a hash
that spreads like uniform hashing, above 1 for fewer collisions and below 1
for more.  Only this host-side arithmetic lives here; hashing and counting
run in the library's kernels.
"""
from __future__ import annotations

import math


def expected_collisions(n: int, m: int) -> float:
    """E[Y] under uniform hashing; (1 - 1/m)^n is taken as exp(n log1p(-1/m))."""
    if m < 1:
        raise ValueError("m must be positive")
    if m == 1:
        return float(max(n - 1, 0))
    return n + m * math.expm1(n * math.log1p(-1.0 / m))


def csr(n: int, m: int, observed: int) -> float:
    """E[Y] / Y; infinite when no key collides."""
    e = expected_collisions(n, m)
    return e / observed if observed else math.inf
