"""Host-side checks of the C ABI library (no GPU needed).

* the library loads and exports every entry point include/hive.h declares;
* its host copies of the device hash and reduction agree with independent
  definitions: the BitHash listing evaluated as printed, the oracle's
  transcription and Python's `%`;
* argument errors are reported before any device work.
"""
import ctypes
import os
import random
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hive.h")


@pytest.fixture(scope="module")
def H():
    from paper_2510_15095_amd import build
    from paper_2510_15095_amd import hive as H_  # noqa: F401  (ImportError if the library is missing)
    assert os.path.exists(os.path.join(ROOT, "paper_2510_15095_amd", "libhive.so")), build.__file__
    return H_


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hive_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_problem_statement_calls():
    names = declared_functions()
    for required in ("hive_create", "hive_insert_batch", "hive_lookup_batch", "hive_delete_batch",
                     "hive_resize", "hive_stats"):
        assert required in names


def test_library_exports_every_declared_symbol(H):
    lib = ctypes.CDLL(H.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_mirrors_every_declared_symbol(H):
    missing = [n for n in declared_functions() if not hasattr(H, n)]
    assert not missing, f"no Python binding for: {missing}"


def test_device_hash_matches_oracle_transcription(H):
    import oracle
    rng = random.Random(0)
    for x in [0, 1, 2, 0xFFFFFFFF, 0x80000000] + [rng.getrandbits(32) for _ in range(20000)]:
        assert H.hive_bithash1(x) == oracle.bithash1(x)
        assert H.hive_bithash2(x) == oracle.bithash2(x)


def test_device_hash_matches_listing_as_printed(H):
    """The device hashes (host-compiled copy of the same source) against the
    Section III-C listing evaluated statement by statement as printed."""
    import oracle_pins as P
    rng = random.Random(5)
    for x in P.LISTING_EDGE_KEYS + [rng.getrandbits(32) for _ in range(100_000)]:
        assert H.hive_bithash1(x) == P.listing_bithash1(x), hex(x)
        assert H.hive_bithash2(x) == P.listing_bithash2(x), hex(x)


def test_fastmod_equals_modulo(H):
    rng = random.Random(1)
    divisors = list(range(1, 1 << 12)) + [rng.randrange(1, 1 << 32) for _ in range(300)] + [
        (1 << 32) - 1, (1 << 31), (1 << 31) + 1, 4415057, 1103765, 8192]
    for d in divisors:
        m = H.hive_fastmod_magic(d)
        for a in [0, 1, d - 1, d, d + 1, (1 << 32) - 1] + [rng.getrandbits(32) for _ in range(8)]:
            a &= 0xFFFFFFFF
            assert H.hive_fastmod(a, m, d) == a % d, (a, d)


def test_config_defaults(H):
    cfg = H.hive_config_default()
    assert cfg.slots_per_bucket == 16 and cfg.max_evictions == 8
    assert cfg.lf_expand_pct == 90 and cfg.lf_contract_pct == 25 and cfg.addressing == H.HIVE_FIXED


@pytest.mark.parametrize("bad", [
    dict(slots_per_bucket=15), dict(slots_per_bucket=0), dict(addressing=7), dict(lf_expand_pct=0),
    dict(lf_expand_pct=101), dict(lf_contract_pct=95), dict(max_evictions=5000),
    # hash choices other than BitHash1/2: 16-slot FIXED tables, plain probing only
    dict(hash_pair=4), dict(hash_pair=1, addressing=1), dict(hash_pair=2, slots_per_bucket=32),
    dict(hash_pair=1, probe_both=1), dict(hash_pair=3, addressing=1), dict(hash_pair=3, slots_per_bucket=64),
    # 32-bit entries: 32-slot FIXED BitHash tables only
    dict(entry_bits=32), dict(entry_bits=48), dict(entry_bits=32, slots_per_bucket=32, addressing=1),
    dict(entry_bits=32, slots_per_bucket=32, hash_pair=2),
    # probe-kernel variants: 16-slot BitHash tables without probe_both only;
    # inserts refuse the variants that would spill; unknown variants and bits
    dict(probe_tuning=1), dict(probe_tuning=2), dict(probe_tuning=5 << 8), dict(probe_tuning=1 << 16),
    dict(probe_tuning=3 << 4, slots_per_bucket=32), dict(probe_tuning=3, hash_pair=3),
    dict(probe_tuning=3 << 12, probe_both=1), dict(probe_tuning=3, entry_bits=32, slots_per_bucket=32),
    dict(probe_grid=(1 << 20) + 1),
])
def test_create_rejects_bad_config_without_touching_the_device(H, bad):
    cfg = H.hive_config_default(**bad)
    h = ctypes.c_void_p()
    assert H.lib.hive_create(ctypes.byref(cfg), 1024, None, ctypes.byref(h)) == H.HIVE_ERR_ARG
    assert not h.value


def test_create_rejects_zero_buckets_and_fixed_growth(H):
    h = ctypes.c_void_p()
    cfg = H.hive_config_default()
    assert H.lib.hive_create(ctypes.byref(cfg), 0, None, ctypes.byref(h)) == H.HIVE_ERR_ARG
    cfg = H.hive_config_default(max_buckets=2048)  # FIXED tables cannot grow
    assert H.lib.hive_create(ctypes.byref(cfg), 1024, None, ctypes.byref(h)) == H.HIVE_ERR_ARG
    cfg = H.hive_config_default(addressing=H.HIVE_LINEAR, max_buckets=(1 << 31) + 1)
    assert H.lib.hive_create(ctypes.byref(cfg), 1024, None, ctypes.byref(h)) == H.HIVE_ERR_ARG


def test_null_handle_and_arguments_rejected(H):
    lib = H.lib
    assert lib.hive_insert_batch(None, None, None, 0, 0, None) == H.HIVE_ERR_ARG
    assert lib.hive_lookup_batch(None, None, 0, None, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_delete_batch(None, None, 0, 0, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_mixed_batch(None, None, None, None, 0, 0, None, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_resize(None, 1, None) == H.HIVE_ERR_ARG
    assert lib.hive_stats(None, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_destroy(None) == H.HIVE_ERR_ARG
    assert lib.hive_drain_results(None, None, 0, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_drain_result(None, 0, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_phase_timing(None, 1) == H.HIVE_ERR_ARG
    assert lib.hive_phase_times(None, None) == H.HIVE_ERR_ARG
    assert lib.hive_hash_buckets(H.HIVE_HASH_KINDS, None, 0, 8, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_hash_buckets(0, None, 0, 0, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_hash_buckets(0, None, 0, (1 << 32) + 1, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_hash_buckets(0, None, 0, 8, None, None) == H.HIVE_OK  # empty: nothing to launch
    assert lib.hive_hash_collisions(0, None, 0, 8, None, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_gather_lines(None, 16, None, 5, None, None) == H.HIVE_ERR_ARG
    assert lib.hive_gather_lines(None, 0, None, 0, None, None) == H.HIVE_OK  # empty: nothing to launch
    assert lib.hive_status_string(H.HIVE_ERR_LOST).decode().startswith("pending")


def test_status_strings_cover_all_codes(H):
    for s in (0, -1, -2, -3, -4, -5, 1, 2):
        assert H.lib.hive_status_string(s).decode() != "unknown status"


def test_binding_loads_one_hip_runtime():
    """Importing the binding in a fresh process maps exactly one HIP and one
    HSA runtime (two copies in one process leave the second without a
    device)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2510_15095_amd import hive\n"
            "maps = open('/proc/self/maps').read().split(chr(10))\n"
            "hip = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
            "hsa = {l.split()[-1] for l in maps if 'libhsa-runtime64' in l}\n"
            "print(len(hip), len(hsa))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[-2:] == ["1", "1"], out.stdout
