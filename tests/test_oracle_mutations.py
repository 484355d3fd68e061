"""Planted mistakes: each plausible slip in the C oracle must make a pin fail.

Every case copies oracle/lms_oracle.c, plants one mistake with a textual
replacement, compiles the copy into a temporary library and runs the pins of
tests/test_oracle_pins.py against it.  The pins must reject every mutant
(the unmodified oracle passes them, see that module).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins
import test_oracle_query_pins as qpins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lms_oracle.c")

MUTANTS = {
    "window_end_inclusive": ("origin + k * S + len > ts", "origin + k * S + len >= ts"),
    "floor_div_truncates": ("if ((a % b) != 0 && a < 0) q -= 1;", ""),
    "avg_wrong_count": ("out_f[k * cap + g] = s / (double)cnt;", "out_f[k * cap + g] = s / (double)(cnt + 1);"),
    "min_max_swapped": ("(afn[k] == ORC_MIN ? mn : mx)", "(afn[k] == ORC_MIN ? mx : mn)"),
    "le_as_lt": ("case ORC_LE: return v <= c;", "case ORC_LE: return v < c;"),
    "projection_not_truncated": ("return (int64_t)(int32_t)(uint32_t)raw;", "return (int64_t)raw;"),
    "join_first_match_only": ("for (int64_t j = lo; j < nb && rows[j].key == k; ++j)",
                              "for (int64_t j = lo; j < nb && j < lo + 1 && rows[j].key == k; ++j)"),
    "runs_ignore_key": ("mem[b].wstart == mem[a].wstart && mem[b].key == mem[a].key",
                        "mem[b].wstart == mem[a].wstart"),
    "sum_of_first_row": ("s += (uint64_t)v;", "s = (uint64_t)v;"),
    "tuple_ignores_last_key": ("if (x->key[j] != y->key[j]) return 0;",
                               "if (j + 1 < nkey && x->key[j] != y->key[j]) return 0;"),
    "tuple_keys_unsorted": ("if (x->key[j] != y->key[j]) return x->key[j] < y->key[j] ? -1 : 1;", ""),
    "self_join_ordered_pairs_only": ("for (int64_t y = r; y < e; ++y) {", "for (int64_t y = x; y < e; ++y) {"),
    "self_join_runs_ignore_key": ("while (e < wend && mem[e].key == mem[r].key) ++e;\n      for (int64_t x",
                                  "while (e < wend) ++e;\n      for (int64_t x"),
}


def battery():
    """The pins, run in sequence; returns the list of failures."""
    failures = []
    checks = [
        *[(lambda s=s: pins.test_window_agg_matches_brute_force(s)) for s in range(12)],
        *[(lambda s=s: pins.test_filter_project_matches_brute_force_and_numpy(s)) for s in range(8)],
        pins.test_projection_wraps_int32,
        pins.test_window_sum_of_wrapping_projection,
        pins.test_predicate_nan_semantics,
        pins.test_tumbling_single_key_equals_bincount,
        lambda: pins.test_sliding_count_invariant(10, 1),
        lambda: pins.test_sliding_equals_merge_of_tumbling_panes(10, 2, 3),
        *[(lambda s=s: pins.test_join_matches_brute_force(s)) for s in range(8)],
        pins.test_join_pandas_merge_and_unique_keys,
        *[(lambda s=s: qpins.test_composite_key_query_matches_brute_force(s)) for s in range(8)],
        qpins.test_composite_key_equals_single_key_on_tuple_ids,
        *[(lambda s=s: qpins.test_self_join_matches_brute_force(s)) for s in range(6)],
        qpins.test_self_join_counts_are_squares_of_window_counts,
    ]
    for c in checks:
        try:
            c()
        except AssertionError as e:  # a pin rejected the oracle
            failures.append(repr(e)[:80])
    return failures


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, "mutation anchor vanished from the oracle source"
    src = tmp_path / "mut.c"
    src.write_text(text.replace(old, new, 1))
    lib_path = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(lib_path), str(src)])
    lib = ctypes.CDLL(str(lib_path))
    for fn in ("orc_filter_project", "orc_window_agg", "orc_window_group", "orc_hash_join", "orc_window_agg_keys",
               "orc_window_self_join"):
        getattr(lib, fn).restype = ctypes.c_int64
    saved = oracle._load()
    oracle._lib = lib
    try:
        failures = battery()
    finally:
        oracle._lib = saved
    assert failures, f"no pin caught the planted mistake {name}"


def test_unmutated_oracle_passes_battery():
    assert battery() == []
