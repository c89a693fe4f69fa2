"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in a private copy of the oracle's C source (on the CPU), builds it,
points the oracle binding at it, and requires that at least one of the pin
checks fails.  The real oracle is restored afterwards."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle_bulk as TB
from tests import test_oracle_fullkeys as TF
from tests import test_oracle_hash as TH
from tests import test_oracle_migration as TM
from tests import test_oracle_mulshift as TMS
from tests import test_oracle_strings as TS
from tests import test_oracle_table as TT

SRC = os.path.join(os.path.dirname(oracle.__file__), "lpht_oracle.c")

# (name, function the mistake is planted in or None for whole file, old, new)
MUTANTS = [
    ("crc32_poly_instead_of_crc32c", None, "0x82F63B78u", "0xEDB88320u"),
    ("hash_seeds_swapped", "orc_hash", "orc_crc32c_word(seed_hi, key", "orc_crc32c_word(seed_lo, key"),
    ("position_low_bits", "orc_home", "return h >> (64 - log2c);",
     "return h & ((1ull << log2c) - 1);"),
    ("insert_reuses_tombstones", "op_insert", "if (cur == ORC_EMPTY) {",
     "if (cur == ORC_EMPTY || cur == ORC_TOMB) {"),
    ("find_stops_at_tombstone", "op_find", "if (cur == ORC_EMPTY) return 0;",
     "if (cur == ORC_EMPTY || cur == ORC_TOMB) return 0;"),
    ("erase_keeps_live_count", "op_erase", "t->live--;", ";"),
    ("upsert_add_assigns", "apply_up", "(op == ORC_ADD) ? cur + d : d", "d"),
    ("probe_wrap_wrong", "op_insert", "i = (i + 1) & (t->cap - 1);", "i = (i + 1) % (t->cap - 1);"),
    ("migrate_scan_from_zero", "orc_migrate", "e = i;\n      break;", "break;"),
    ("migrate_keeps_tombstones", "orc_migrate", "if (k == ORC_EMPTY || k == ORC_TOMB) continue;",
     "if (k == ORC_EMPTY) continue;"),
    ("growth_single_doubling", "grow_before_batch", "} while (!within_fill(t, t->live + b, t->cap));",
     "} while (0);"),
    ("growth_never_cleans", "grow_before_batch", "return orc_migrate(t, target);",
     "return orc_migrate(t, t->log2c + 1);"),
    ("growth_never_shrinks", "grow_before_batch",
     "while (target > t->log2_min && fits_quarter(t, t->live + b, 1ull << target)) --target;", ";"),
    ("shrink_below_created_capacity", "grow_before_batch", "target > t->log2_min && ", ""),
    ("shrink_one_step_too_far", "grow_before_batch", "fits_quarter(t, t->live + b, 1ull << target)",
     "within_fill(t, t->live + b, 1ull << target)"),
    ("special_erase_keeps_key", "op_erase", "t->sp_present[k] = 0;", ";"),
    ("special_upsert_assigns", "sp_insert", "if (is_upsert) t->sp_val[k] = apply_up(t, t->sp_val[k], v, op);",
     "if (is_upsert) t->sp_val[k] = v;"),
    ("string_prefix_equal", "str_eq", "return t->len[i] == len && (len == 0 || memcmp(t->str[i], s, len) == 0);",
     "return len <= t->len[i] && (len == 0 || memcmp(t->str[i], s, len) == 0);"),
    ("string_find_stops_at_tombstone", "str_op", "if (r != 1 && str_eq(t, r, s, len)) {",
     "if (r == 1 && kind >= 2) return 0;\n    if (r != 1 && str_eq(t, r, s, len)) {"),
    ("string_hash_one_seed", "orc_str_hash", "orc_crc32c_bytes(seed_lo, s, len)", "orc_crc32c_bytes(seed_hi, s, len)"),
    ("bulk_keeps_first", "orc_bulk_merge", ": it[i].v;", ": it[d - 1].v;"),
    ("bulk_sorted_by_key", "item_cmp",
     "if ((x->h >> 32) != (y->h >> 32)) return (x->h >> 32) < (y->h >> 32) ? -1 : 1;",
     "if (x->k != y->k) return x->k < y->k ? -1 : 1;"),
    ("bulk_order_by_whole_hash", "item_cmp",
     "if ((x->h >> 32) != (y->h >> 32)) return (x->h >> 32) < (y->h >> 32) ? -1 : 1;",
     "if (x->h != y->h) return x->h < y->h ? -1 : 1;"),
    ("mulshift_32bit_product", "orc_mulshift", "return key * mul;",
     "return (uint64_t)(uint32_t)key * (uint32_t)mul;"),
    ("mulshift_ignored_by_table", "table_hash", "if (t->hash_kind == ORC_HASH_MULSHIFT) return orc_mulshift(k, t->mul);",
     ";"),
    ("bulk_add_drops_table_value", "orc_bulk_merge", "it[m].v = val_at(t, t->cells, i);", "it[m].v = 0;"),
    ("bulk_no_dedup", "orc_bulk_merge", "if (d > 0 && it[d - 1].k == it[i].k) {", "if (0) {"),
    ("bulk_never_grows", "orc_bulk_merge", "while (!within_fill(t, old_n + n, 1ull << log2c)) {",
     "while (0) {"),
    ("bulk_probe_skips_home", "orc_bulk_merge", "uint64_t i = orc_home(it[j].h, log2c);",
     "uint64_t i = (orc_home(it[j].h, log2c) + 1) & (cap - 1);"),
]


def _plant(src, func, old, new):
    if func is None:
        assert old in src
        return src.replace(old, new)
    start = src.index(func + "(")
    # the function body: from its name to the next line that is a lone "}"
    end = src.index("\n}\n", start)
    body = src[start:end]
    assert old in body, (func, old)
    return src[:start] + body.replace(old, new, 1) + src[end:]


def _pins():
    """Quick versions of the pin checks; each raises on a violation."""
    yield lambda: [TH.test_crc32c_published_vectors(*v) for v in TH._golden_vectors()]
    yield TH.test_crc32c_matches_sse42_instruction_bytes_and_words
    yield TH.test_scaling_map_closed_form
    yield lambda: TH.test_hash_matches_sse42_on_1e6_keys(8)
    yield lambda: TH.test_hash_matches_sse42_on_1e6_keys(4)
    for layout in TT.LAYOUTS:
        yield lambda layout=layout: TT.test_random_sequences_match_dict_model(layout, 4)
        yield lambda layout=layout: TT.test_brute_force_histogram_of_upserts(layout)
        yield lambda layout=layout: TM.test_wraparound_cluster_migrates_in_order(layout)
        yield lambda layout=layout: TM.test_migration_equals_insert_in_scan_order(layout, 1, 0.5, 0.2)
        yield lambda layout=layout: TM.test_growth_insert_only_final_capacity_closed_form(layout)
        yield lambda layout=layout: TM.test_tombstone_cleanup_same_size(layout)
        yield lambda layout=layout: TM.test_cleanup_shrinks_to_hand_computed_capacity(layout)
        yield lambda layout=layout: TM.test_cleanup_never_shrinks_below_created_capacity(layout)
        yield lambda layout=layout: TM.test_explicit_shrink_keeps_contents_and_order_free_occupancy(layout, 2)
        for op in (oracle.ASSIGN, oracle.ADD):
            for seed in range(3):
                yield lambda layout=layout, op=op, seed=seed: TB.test_build_matches_dict_model_and_invariants(
                    layout, op, seed)
                yield lambda layout=layout, op=op, seed=seed: TB.test_merge_matches_dict_model_with_tombstones(
                    layout, op, seed)
        yield lambda layout=layout: TB.test_occupancy_equals_insertion_in_random_order(layout)
        yield lambda layout=layout: TB.test_hand_worked_wrapping_example(layout)
        yield lambda layout=layout: TB.test_capacity_rule_and_full_tables(layout)
        for seed in range(3):
            yield lambda layout=layout, seed=seed: TF.test_sequences_with_keys_0_and_1_match_dict_model(layout, seed)
        yield lambda layout=layout: TF.test_special_keys_survive_migration_and_follow_bulk_rules(layout)
    yield TMS.test_mulshift_closed_form
    for layout in TT.LAYOUTS:
        yield lambda layout=layout: TMS.test_keys_with_distinct_homes_sit_at_their_homes(layout, TMS.MULS[0])
        yield lambda layout=layout: TMS.test_bulk_build_order_upper_half_then_key(layout)
    yield TS.test_string_hash_equals_word_hash_and_seed_closed_form
    for seed in range(3):
        yield lambda seed=seed: TS.test_sequences_match_dict_model(seed)
    yield TS.test_occupancy_independent_of_order_and_migration


@pytest.mark.parametrize("name,func,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, func, old, new):
    src = open(SRC).read()
    bad = _plant(src, func, old, new)
    assert bad != src
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(bad)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(c)], check=True)
    saved = oracle._lib
    oracle._lib = oracle.load(str(so))
    caught = []
    try:
        for pin in _pins():
            try:
                with np.errstate(all="ignore"):
                    pin()
            except Exception as e:  # noqa: BLE001 - any failure counts as caught
                caught.append(type(e).__name__)
                break
    finally:
        oracle._lib = saved
    assert caught, f"planted mistake '{name}' passed every pin"
