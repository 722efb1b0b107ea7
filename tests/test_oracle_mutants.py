"""Plant mistakes in copies of the CPU oracle; some pin must catch each one.

Every mutant is a textual edit of oracle/hive_oracle.c compiled into a
temporary library; nothing here touches the GPU or the built oracle."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle
import oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "hive_oracle.c")

MUTANTS = {
    "bithash1_constant": ("{ST_AFFINE, 2057u, 0u},", "{ST_AFFINE, 2053u, 0u},"),
    "bithash2_dropped_step": ("    {ST_XORSHR, 19u, 0xc761c23cu},\n", ""),
    "bithash2_wrong_shift": ("{ST_ADDXORSHL, 9u, 0xd3a2646cu},", "{ST_ADDXORSHL, 8u, 0xd3a2646cu},"),
    "two_choice_tie_to_second": ("(f2 > f1) ? c2 : c1, second = (f2 > f1) ? c1 : c2",
                                 "(f2 >= f1) ? c2 : c1, second = (f2 >= f1) ? c1 : c2"),
    "alt_bucket_always_second": ("return (b == c1) ? c2 : c1;", "return c2;"),
    "lookup_skips_second_bucket": ("if (j == 1 && c2 == c1) break;", "if (j == 1) break;"),
    "delete_keeps_free_bit_clear": ("      t->free_mask[loc.bucket] |= 1ull << loc.index;\n", ""),
    "split_rule_inverted": ("(h[j] & next_mask) == src) stay = 1;", "(h[j] & next_mask) == dst) stay = 1;"),
    "merge_first_free_slot_only": ("nth_set_bit(lo_free, rank++)", "nth_set_bit(lo_free, 0)"),
    "stash_capacity_off_by_one": ("if (t->stash_tail - t->stash_head < t->stash_cap) {",
                                  "if (t->stash_tail - t->stash_head <= t->stash_cap) {"),
    "o1_delete_does_not_unlink": ("            *link = d->pool[idx].next;\n", ""),
    "linear_address_no_split_check": ("if (a < t->sp) a = h & (2 * t->im + 1);", ""),
    "round_not_doubled": ("t->im = 2 * t->im + 1;\n      t->sp = 0;\n    }\n    done++;",
                          "t->sp = 0;\n    }\n    done++;"),
    "evict_no_reroute": ("b = alt_bucket(t, key_of(kv), b);", "(void)0;"),
    "replace_not_checked_in_stash": ("    if (w != O_TOMB && key_of(w) == key) {", "    if (0) {"),
}


def _build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutant {name}: pattern not found in the oracle"
    src = os.path.join(tmpdir, f"{name}.c")
    with open(src, "w") as f:
        f.write(text.replace(old, new, 1))
    lib = os.path.join(tmpdir, f"{name}.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", src, "-o", lib], check=True)
    return lib


_BATTERY = """
import sys
import oracle, oracle_pins as P
L = oracle.bind(sys.argv[1])
for pin in P.ALL_PINS:
    try:
        pin(L)
    except Exception as e:  # any failure of a pin is a detection
        print("caught by", pin.__name__, repr(e)[:200])
        sys.exit(1)
print("caught by none")
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_some_pin_catches_mutant(name):
    here = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([os.path.dirname(here), here]))
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(name, tmp)
        try:
            r = subprocess.run([sys.executable, "-c", _BATTERY, lib], env=env, timeout=30,
                               capture_output=True, text=True)
        except subprocess.TimeoutExpired:
            return  # the pins hang on this mutant: detected
        assert r.returncode != 0, f"no pin detects the planted mistake {name!r}: {r.stdout}{r.stderr}"
