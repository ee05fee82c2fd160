"""Planted mistakes in copies of the oracle: each must fail at least one pin.

Every mutant is a textual edit of ``oracle/ckpp_oracle.c`` compiled into a
temporary directory and exercised in a child process (a mutant may crash).
This shows that the pins catch the plausible slips they are meant to catch:
a dropped term, a wrong sign or index, a swapped operand.
"""

import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ckpp_oracle.c")

MUTANTS = [
    ("bloom_bits_not_set", "t->buckets[p].bloom |= m;", "(void)m;"),
    ("bloom_not_reset", "if (t->buckets[p].moved == 0) t->buckets[p].bloom = 0;", ";"),
    ("moved_counts_twice", "t->buckets[p].moved += 1;", "t->buckets[p].moved += 2;"),
    ("second_bloom_bit_equals_first", "out->b2 = (uint32_t)((h >> 30) & 63);",
     "out->b2 = (uint32_t)((h >> 24) & 63);"),
    ("alternate_may_equal_primary", "if (out->a == out->p) out->a ^= 1;", ";"),
    ("large_tables_keep_small_split", "if (log2_buckets <= 24) {", "if (1) {"),
    ("bloom_prune_inverted", "probe_secondary = orc_bloom_pass(t, sp.p, sp.bloom_mask);",
     "probe_secondary = !orc_bloom_pass(t, sp.p, sp.bloom_mask);"),
    ("no_home_preference", "if (nhome > 0)", "if (0)"),
    ("big_endian_words", "for (int i = 7; i >= 0; i--) lo = (lo << 8) | key[i];",
     "for (int i = 0; i < 8; i++) lo = (lo << 8) | key[i];"),
    ("tag_off_by_one", "out->tag = (uint32_t)(h >> 48);", "out->tag = (uint32_t)(h >> 47);"),
    ("secondary_insert_not_marked", "orc_place(t, sp.a, s, key, value, sp.tag, sp.p, 1, expiry);",
     "orc_place(t, sp.a, s, key, value, sp.tag, sp.p, 0, expiry);"),
    ("delete_keeps_moved_count", "if ((bk->sec >> s) & 1) orc_bloom_remove(t, bk->other[s]);",
     ";"),
    ("move_maintenance_swapped", "    if (was_secondary)\n        orc_bloom_remove",
     "    if (!was_secondary)\n        orc_bloom_remove"),
    ("key_compare_8_bytes", "if (memcmp(orc_rec(t, b, s)->key, key, 16) == 0) return s;",
     "if (memcmp(orc_rec(t, b, s)->key, key, 8) == 0) return s;"),
    ("plain_lookup_one_bucket", "uint32_t bl = (mode == ORC_MODE_BOTH) ? 2 : 1, kl = 0;",
     "uint32_t bl = 1, kl = 0;"),
    ("seed_ignored", "return orc_fmix64(orc_fmix64(lo ^ seed) ^ hi);",
     "return orc_fmix64(orc_fmix64(lo) ^ hi);"),
    # timers (Sec. 4.2)
    ("timer_window_off_by_one", "return (uint16_t)(e - now) >= ORC_MAX_DELAY;",
     "return (uint16_t)(e - now) > ORC_MAX_DELAY;"),
    ("timer_difference_reversed", "return (uint16_t)(e - now) >= ORC_MAX_DELAY;",
     "return (uint16_t)(now - e) >= ORC_MAX_DELAY;"),
    ("lookup_sees_expired", "int s = orc_find_in(t, sp.p, sp.tag, key, &kl, ORC_ALIVE, now);",
     "int s = orc_find_in(t, sp.p, sp.tag, key, &kl, ORC_ANY, now);"),
    ("insert_ignores_expired_slots",
     "if (!(bk->busy & (1u << s)) || orc_expired(t, b, s, now)) return s;",
     "if (!(bk->busy & (1u << s))) return s;"),
    ("refresh_not_written", "if (refresh && t->timed) orc_rec(t, b, s)->pad = expiry;", ";"),
    ("scan_keeps_expired", "orc_remove_slot(t, b, s);\n                removed++;", "removed++;"),
    ("timed_value_shares_time_word", "    r->value = value;\n",
     "    r->value = t->timed ? ((value & 0xFFFFFFFFFFFFull) | ((uint64_t)expiry << 48)) : value;\n"),
    ("update_keeps_old_expiry", "if (t->timed) orc_rec(t, b, s)->pad = expiry;\n", "\n"),
]

RUNNER = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
from oracle import oracle as O
import oracle_pins as P
lib = O.load({lib!r})
failed = P.run_quick(lib)
print("FAILED_PINS", failed)
sys.exit(1 if failed else 0)
"""


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = os.path.join(d, "libmutant.so")
        subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", lib, path],
                       check=True, capture_output=True)
        code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           timeout=600)
        assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"


def test_unmutated_oracle_passes_quick_pins():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle_pins as P
    from oracle import oracle as O
    assert P.run_quick(O.load()) == []
