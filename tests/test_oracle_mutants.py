"""Plant one plausible mistake at a time in a copy of the oracle source (on
the CPU), rebuild it, and check that the pin suite rejects every mutant."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ccq_oracle.cpp")

MUTANTS = {
    "range_upper_inclusive": ("h = q.preds[p].lo <= v && v < q.preds[p].hi",
                              "h = q.preds[p].lo <= v && v <= q.preds[p].hi"),
    "range_lower_exclusive": ("h = q.preds[p].lo <= v && v < q.preds[p].hi",
                              "h = q.preds[p].lo < v && v < q.preds[p].hi"),
    "not_ignored": ("return (op == ORC_NOT_RANGE || op == ORC_NOT_IN) ? !h : h;", "return h;"),
    "or_clause_as_and": ("bool any = false;\n                for (size_t p : q.clauses[c]) any = any || holds(p);",
                         "bool any = true;\n                for (size_t p : q.clauses[c]) any = any && holds(p);"),
    "or_clause_first_only": ("for (size_t p : q.clauses[c]) any = any || holds(p);",
                             "any = holds(q.clauses[c][0]);"),
    "rle_run_one_row_long": ("int64_t stop = std::min(c.run_ends[i], r1);",
                             "int64_t stop = std::min(c.run_ends[i] + 1, r1);"),
    "rle_value_of_next_run": ("int64_t stop = std::min(c.run_ends[i], r1);\n            int64_t v = value_at(c, i);",
                              "int64_t stop = std::min(c.run_ends[i], r1);\n"
                              "            int64_t v = value_at(c, i + 1 < c.n ? i + 1 : i);"),
    "index_unlisted_rows_one": ("for (int64_t k = 0; k < len; k++) out[k] = 0;\n        for (int64_t i = first_point_at_or_after(c, r0)",
                                "for (int64_t k = 0; k < len; k++) out[k] = 1;\n        for (int64_t i = first_point_at_or_after(c, r0)"),
    "index_value_shifted": ("out[position_at(c, i) - r0] = value_at(c, i);",
                            "out[position_at(c, i) - r0] = value_at(c, i > 0 ? i - 1 : i);"),
    "bitpacked_drops_base": ("out[r - r0] = c.base + (int64_t)code;", "out[r - r0] = (int64_t)code;"),
    "bitpacked_no_high_word": ("uint64_t two = (uint64_t)c.packed[word] | ((uint64_t)c.packed[word + 1] << 32);",
                               "uint64_t two = (uint64_t)c.packed[word];"),
    "key_ignores_shift": ("int64_t v = x[q.slot[q.keys[k].col]][r] >> q.keys[k].shift;",
                          "int64_t v = x[q.slot[q.keys[k].col]][r];"),
    "sum_counts_rows": ("v = x[q.slot[ag.col]][r];", "v = 1;"),
    "min_as_max": ("if (a.func == ORC_MIN) v = std::min(v, x);", "if (a.func == ORC_MIN) v = std::max(v, x);"),
    "add_as_sub": ("if (ag.op == ORC_OP_ADD) ok = !__builtin_add_overflow(v, w, &v);",
                   "if (ag.op == ORC_OP_ADD) ok = !__builtin_sub_overflow(v, w, &v);"),
    "mul_as_add": ("else ok = !__builtin_mul_overflow(v, w, &v);", "else ok = !__builtin_add_overflow(v, w, &v);"),
    "window_ignores_begin": ("int64_t c0 = q.row_begin + ch * CH;", "int64_t c0 = ch * CH;"),
    "groups_descending": ("for (auto& kv : all) {   /* std::map", "for (auto& kv : std::map<std::vector<int64_t>, Acc, std::greater<std::vector<int64_t>>>(all.begin(), all.end())) {   /* std::map"),
    "thread_merge_drops_counts": ("it->second.count += kv.second.count;", "it->second.count = kv.second.count;"),
    "in_list_first_only": ("q.in_sets[p].insert(q.preds[p].in_list[i]);",
                           "if (i == 0) q.in_sets[p].insert(q.preds[p].in_list[i]);"),
    "composite_points_ignored": ("out[point_position(c, i) - r0] = point_value(c, i);", "(void)0;"),
    "composite_point_value_shifted": ("out[point_position(c, i) - r0] = point_value(c, i);",
                                      "out[point_position(c, i) - r0] = point_value(c, i + 1 < c.pt_n ? i + 1 : i);"),
    "composite_run_value_of_next_run": (
        "int64_t v = value_at(c, i);\n            for (int64_t r = std::max(c.run_starts[i], r0)",
        "int64_t v = value_at(c, i + 1 < c.n ? i + 1 : i);\n            for (int64_t r = std::max(c.run_starts[i], r0)"),
}


def _build(text, out):
    with open(out + ".cpp", "w") as f:
        f.write(text)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", out + ".cpp", "-o", out, "-lpthread"])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation anchor not found: %s" % name
    so = str(tmp_path / ("mut_%s.so" % name))
    _build(src.replace(old, new), so)
    env = dict(os.environ, CCQ_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_composite.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])
