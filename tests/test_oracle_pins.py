"""Pins for the CPU oracle: the paper's worked examples, closed forms,
invariants, round trips through the generator's encoder, brute force and
sqlite3 on tiny tables.  None of these compares the oracle with itself."""
import bisect
import glob
import json
import os

import numpy as np
import pytest

import datagen
from oracle import oracle
from tests import brute
from tests.cases import tiny_query as _tiny_query, tiny_table as _tiny_table

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _as_np_column(c):
    c = dict(c)
    if c["enc"] == "rle":
        c["values"] = np.array(c["values"], dtype=np.int64)
        c["run_ends"] = np.array(c["run_ends"], dtype=np.int64)
    elif c["enc"] == "index":
        c["positions"] = np.array(c["positions"], dtype=np.int32)
        c["values"] = np.array(c["values"], dtype=np.int64)
    else:
        c["packed"] = np.array(c["packed"], dtype=np.uint32)
    return c


def _as_query(q, n_rows):
    return {"preds": [tuple(p) for p in q["preds"]], "keys": [tuple(k) for k in q["keys"]],
            "aggs": [tuple(tuple(x) if isinstance(x, list) else x for x in a) for a in q["aggs"]],
            "window": tuple(q.get("window", (0, n_rows)))}


def _norm(res):
    return {"keys": [tuple(k) for k in res["keys"]], "counts": list(res["counts"]),
            "aggs": [tuple(a) for a in res["aggs"]]}


# ------------------------------------------------------------------ worked examples

def test_rle_encoding_example():
    g = _load("rle_encoding.json")
    col = _as_np_column(g["column"])
    # paper (start, end) inclusive <-> our exclusive run ends
    assert list(col["run_ends"]) == [e + 1 for e in g["paper_end"]]
    assert [0] + list(col["run_ends"][:-1]) == g["paper_start"]
    assert list(oracle.decode(col, g["n_rows"])) == g["expect_rows"]


def test_bitwidth_example_packing_and_decode():
    g = _load("bitwidth.json")
    packed = datagen.pack_codes(np.array(g["codes"], dtype=np.uint32), g["w"])
    assert list(packed) == g["packed_words"]
    col = {"enc": "bitpacked", "packed": packed, "w": g["w"], "base": g["base"]}
    assert list(oracle.decode(col, g["n_rows"])) == g["expect_rows"]
    assert brute.decode_rows(col, g["n_rows"]) == g["expect_rows"]


@pytest.mark.parametrize("name", ["range_intersect.json", "idx_in_rle.json", "alignment.json", "groupby.json"])
def test_paper_query_examples(name):
    g = _load(name)
    table = {"n_rows": g["n_rows"], "columns": {k: _as_np_column(v) for k, v in g["columns"].items()}}
    for q in g["queries"]:
        query = _as_query(q, g["n_rows"])
        exp = _norm(q["expect"])
        assert _norm(oracle.run(table, query, n_threads=1)) == exp, (name, q)
        assert _norm(oracle.run(table, query, n_threads=4)) == exp, (name, q)
        assert _norm(brute.run(table, query)) == exp, (name, q)


def test_range_intersect_example_matches_paper_ranges():
    """The groups of the range_intersect fixture are exactly the paper's
    intersection ranges s=[2,4,6], e=[3,5,7]: recompute the lengths e-s+1."""
    g = _load("range_intersect.json")
    lengths = [e - s + 1 for s, e in zip(g["paper_result_start"], g["paper_result_end"])]
    assert g["queries"][1]["expect"]["counts"] == lengths


def test_alignment_example_matches_paper_aligned_runs():
    g = _load("alignment.json")
    lengths = [e - s + 1 for s, e in zip(g["paper_aligned_start"], g["paper_aligned_end"])]
    by_pair = dict(zip(zip(g["paper_r1"], g["paper_r2"]), lengths))
    q = g["queries"][2]["expect"]
    assert {tuple(k): c for k, c in zip(q["keys"], q["counts"])} == by_pair
    assert [a + b for a, b in zip(g["paper_r1"], g["paper_r2"])] == g["paper_r1_plus_r2"]


def test_bucketize_reading_matches_worked_examples():
    """Reading of bucketize: right=False is lower_bound, right=True is
    upper_bound.  The worked examples of Algorithms 1, 3 and 5 fix it."""
    lower = lambda xs, b: [bisect.bisect_left(b, x) for x in xs]
    upper = lambda xs, b: [bisect.bisect_right(b, x) for x in xs]
    assert lower([2], [3, 5, 8]) == [0]                       # Algorithm 1 step 1
    assert upper([7], [1, 4, 6]) == [3]                       # Algorithm 1 step 2
    assert upper([2, 4, 7], [0, 6]) == [1, 1, 2]              # Algorithm 3 step 1
    assert lower([0, 6], [2, 4, 7]) == [0, 2]                 # Algorithm 5 step 1
    assert upper([2, 7], [2, 4, 7]) == [1, 3]                 # Algorithm 5 step 2


# ------------------------------------------------------------------ encodings round trip

@pytest.mark.parametrize("w", list(range(1, 33)))
def test_bitpacked_round_trip_all_widths(w):
    rng = np.random.default_rng(w)
    n = 1000 + w  # not a multiple of 32: ragged last group
    codes = rng.integers(0, 1 << w, size=n, dtype=np.uint64).astype(np.uint32)
    packed = datagen.pack_codes(codes, w)
    base = int(rng.integers(-(1 << 40), 1 << 40))
    col = {"enc": "bitpacked", "packed": packed, "w": w, "base": base}
    got = oracle.decode(col, n)
    np.testing.assert_array_equal(got, codes.astype(np.int64) + base)
    part = oracle.decode(col, n, 37, 700)
    np.testing.assert_array_equal(part, codes[37:700].astype(np.int64) + base)
    if w in (1, 7, 14, 20, 32):
        assert brute.decode_rows(col, 200) == list(codes[:200].astype(np.int64) + base)


def test_generated_packed_column_matches_codes():
    n = 50_000
    col = datagen.packed_column(5, 77, n, 14, "zipf", 10000)
    codes = datagen.zipf_codes(5, 77, 1.1, 10000, n)
    np.testing.assert_array_equal(oracle.decode(col, n), codes.astype(np.int64))


def test_rle_round_trip_and_generator_invariants():
    n = 300_001
    for dist, mean in (("geometric", 16), ("lognormal", 64), ("lognormal", 1000)):
        c = datagen.rle_column(3, 500, n, dist, mean, 0, 1000)
        e = c["run_ends"]
        assert e[-1] == n and np.all(np.diff(e) > 0) and e[0] > 0
        lens = np.diff(np.r_[0, e])
        assert lens.sum() == n                                   # run lengths sum to N
        assert abs(lens[:-1].mean() / mean - 1) < 0.1
        rows = oracle.decode(c, n)
        np.testing.assert_array_equal(rows, np.repeat(c["values"].astype(np.int64), lens))
        np.testing.assert_array_equal(oracle.decode(c, n, 1234, 99_999), rows[1234:99_999])


def test_index_round_trip_and_generator_invariants():
    n = 200_000
    c = datagen.sparse_column(9, 600, n, 0.01, 1, 1_000_000)
    p = c["positions"]
    assert np.all(np.diff(p) > 0) and p[0] >= 0 and p[-1] < n
    assert abs(len(p) / (0.01 * n) - 1) < 0.1
    dense = np.zeros(n, dtype=np.int64)
    dense[p] = c["values"]
    np.testing.assert_array_equal(oracle.decode(c, n), dense)
    np.testing.assert_array_equal(oracle.decode(c, n, 777, 150_000), dense[777:150_000])
    c64 = dict(c, positions=p.astype(np.int64))
    np.testing.assert_array_equal(oracle.decode(c64, n), dense)


def test_generator_is_thread_count_independent():
    import subprocess
    import sys
    code = ("import datagen,hashlib;c=datagen.config_c2(n_rows=3_000_000);"
            "h=hashlib.sha256();[h.update(a.tobytes()) for v in c['columns'].values() for a in v.values() "
            "if hasattr(a,'tobytes')];print(h.hexdigest())")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = set()
    for t in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.add(subprocess.check_output([sys.executable, "-c", code], cwd=root, env=env).strip())
    assert len(outs) == 1


# ------------------------------------------------------------------ closed forms and invariants

def _rle_table(seed, n, specs):
    cols = {}
    for i, (name, dist, mean, lo, hi, dt) in enumerate(specs):
        cols[name] = datagen.rle_column(seed, 100 * (i + 1), n, dist, mean, lo, hi, dt)
    return {"n_rows": n, "columns": cols}


def test_sum_over_rle_closed_form_and_single_run():
    """SUM over an RLE column is the sum of value * run length; one run of N
    rows gives v * N."""
    n = 500_000
    t = _rle_table(11, n, [("m", "lognormal", 32, -10**6, 10**6 + 1, np.int64)])
    c = t["columns"]["m"]
    lens = np.diff(np.r_[0, c["run_ends"]])
    closed = int(np.sum(c["values"].astype(np.int64) * lens))
    r = oracle.run(t, {"preds": [], "keys": [], "aggs": [("sum", "m"), ("count",)], "window": (0, n)})
    assert r["aggs"][0] == (closed, n) and r["counts"] == [n]
    one = {"n_rows": n, "columns": {"x": {"enc": "rle", "values": np.array([-7], dtype=np.int64),
                                           "run_ends": np.array([n], dtype=np.int64)}}}
    r = oracle.run(one, {"preds": [], "keys": [], "aggs": [("sum", "x")], "window": (0, n)})
    assert r["aggs"][0] == (-7 * n,)


def test_aligned_boundaries_are_the_union_of_run_ends():
    """GROUP BY the run numbers of every RLE column: each group is one aligned
    run, so the groups' boundaries must be the union of all run ends and each
    COUNT the gap between consecutive union points (coarsest common refinement)."""
    n = 120_000
    t = _rle_table(12, n, [("a", "geometric", 16, 0, 10, np.int32), ("b", "lognormal", 40, 0, 10, np.int32),
                           ("c", "lognormal", 300, 0, 10, np.int32)])
    ids = {}
    for name, c in list(t["columns"].items()):
        R = len(c["run_ends"])
        ids[name + "_run"] = {"enc": "rle", "values": np.arange(R, dtype=np.int64), "run_ends": c["run_ends"]}
    t["columns"].update(ids)
    keys = [(k, 0, len(v["run_ends"])) for k, v in ids.items()]
    r = oracle.run(t, {"preds": [], "keys": keys, "aggs": [("count",)], "window": (0, n)})
    union = np.unique(np.concatenate([c["run_ends"] for c in ids.values()]))
    assert len(r["keys"]) == len(union)
    assert r["counts"] == list(np.diff(np.r_[0, union]))
    assert sum(r["counts"]) == n


def test_complement_and_partition_invariants():
    n = 400_000
    t = _rle_table(13, n, [("a", "lognormal", 64, 0, 1 << 16, np.int32), ("b", "lognormal", 200, 0, 1 << 16, np.int32),
                           ("k", "lognormal", 500, 0, 50, np.int32), ("m", "lognormal", 32, -1000, 1000, np.int64)])
    t["columns"]["s"] = datagen.sparse_column(13, 900, n, 0.01, 1, 10**6)
    base = [("b", "range", 16384, 65536)]
    aggs = [("sum", "m"), ("sum", "s"), ("count",)]
    q = lambda preds, keys=(): {"preds": base + preds, "keys": list(keys), "aggs": aggs, "window": (0, n)}
    inside = oracle.run(t, q([("a", "range", 0, 32768)]))
    below = oracle.run(t, q([("a", "range", -(1 << 63), 0)]))
    above = oracle.run(t, q([("a", "range", 32768, 1 << 62)]))
    every = oracle.run(t, q([]))
    # COUNT(p) + COUNT(not p) = COUNT; same for sums
    for i in range(3):
        assert inside["aggs"][0][i] + below["aggs"][0][i] + above["aggs"][0][i] == every["aggs"][0][i]
    # group sums add up to the ungrouped sums
    grouped = oracle.run(t, q([("a", "range", 0, 32768)], [("k", 0, 50)]))
    assert tuple(map(sum, zip(*grouped["aggs"]))) == inside["aggs"][0]
    assert sum(grouped["counts"]) == inside["counts"][0]
    # IN-list additivity: SUM over S = sum over singletons
    S = [3, 9, 17, 41]
    whole = oracle.run(t, q([("k", "in", S)]))
    parts = [oracle.run(t, q([("k", "in", [s])])) for s in S]
    assert tuple(map(sum, zip(*[p["aggs"][0] for p in parts]))) == whole["aggs"][0]
    # window additivity
    w1 = dict(q([]), window=(0, 123_457))
    w2 = dict(q([]), window=(123_457, n))
    a1, a2 = oracle.run(t, w1), oracle.run(t, w2)
    assert tuple(x + y for x, y in zip(a1["aggs"][0], a2["aggs"][0])) == every["aggs"][0]
    # thread count does not matter
    assert oracle.run(t, q([], [("k", 0, 50)]), n_threads=1) == oracle.run(t, q([], [("k", 0, 50)]), n_threads=7)


def test_multi_chunk_group_counts_closed_form():
    """Several 2^20-row chunks and several threads: per-group COUNT and SUM of
    an RLE key / RLE measure pair must equal the run-level closed forms
    (COUNT(k) = sum of lengths of the aligned runs with key k)."""
    n = 3_500_000
    t = _rle_table(14, n, [("k", "lognormal", 4000, 0, 16, np.int32), ("m", "lognormal", 3000, -50, 50, np.int64)])
    k, m = t["columns"]["k"], t["columns"]["m"]
    union = np.union1d(k["run_ends"], m["run_ends"])
    starts = np.r_[0, union[:-1]]
    lens = union - starts
    kv = k["values"][np.searchsorted(k["run_ends"], starts, side="right")].astype(np.int64)
    mv = m["values"][np.searchsorted(m["run_ends"], starts, side="right")].astype(np.int64)
    counts = np.bincount(kv, weights=lens, minlength=16).astype(np.int64)
    sums = np.zeros(16, dtype=np.int64)
    np.add.at(sums, kv, mv * lens)
    q = {"preds": [], "keys": [("k", 0, 16)], "aggs": [("sum", "m"), ("count",)], "window": (0, n)}
    for threads in (1, 3, 8):
        r = oracle.run(t, q, n_threads=threads)
        assert r["keys"] == [(i,) for i in range(16) if counts[i] > 0]
        assert r["counts"] == [int(c) for c in counts if c > 0]
        assert r["aggs"] == [(int(sums[i]), int(counts[i])) for i in range(16) if counts[i] > 0]


# ------------------------------------------------------------------ brute force and sqlite3

@pytest.mark.parametrize("seed", range(60))
def test_oracle_matches_brute_force_and_sqlite(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 300))
    t, wd = _tiny_table(rng, n)
    for _ in range(4):
        q = _tiny_query(rng, n, wd)
        got = _norm(oracle.run(t, q, n_threads=1 + seed % 3))
        assert got == _norm(brute.run(t, q)), q
        assert got == _norm(brute.run_sqlite(t, q)), q


def test_hypothesis_tables():
    hyp = pytest.importorskip("hypothesis")
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=60, deadline=None)
    @given(st.integers(1, 200), st.integers(0, 2**31 - 1))
    def inner(n, seed):
        rng = np.random.default_rng(seed)
        t, wd = _tiny_table(rng, n)
        q = _tiny_query(rng, n, wd)
        assert _norm(oracle.run(t, q)) == _norm(brute.run(t, q))

    inner()


# ------------------------------------------------------------------ validation and errors

def test_validation_errors():
    good_rle = {"enc": "rle", "values": np.array([1, 2], dtype=np.int32), "run_ends": np.array([3, 5], dtype=np.int64)}
    q = {"preds": [], "keys": [], "aggs": [("count",)], "window": (0, 5)}
    bad = [
        {"x": dict(good_rle, run_ends=np.array([3, 3], dtype=np.int64))},
        {"x": dict(good_rle, run_ends=np.array([3, 6], dtype=np.int64))},
        {"x": dict(good_rle, run_ends=np.array([0, 5], dtype=np.int64))},
        {"x": {"enc": "index", "positions": np.array([1, 5], dtype=np.int32), "values": np.array([1, 1], dtype=np.int64)}},
        {"x": {"enc": "index", "positions": np.array([2, 2], dtype=np.int32), "values": np.array([1, 1], dtype=np.int64)}},
        {"x": {"enc": "bitpacked", "packed": np.zeros(8, dtype=np.uint32), "w": 0, "base": 0}},
        {"x": {"enc": "bitpacked", "packed": np.zeros(8, dtype=np.uint32), "w": 33, "base": 0}},
    ]
    for cols in bad:
        with pytest.raises(oracle.OracleError):
            oracle.run({"n_rows": 5, "columns": cols}, q)
    t = {"n_rows": 5, "columns": {"x": good_rle}}
    with pytest.raises(oracle.OracleError, match="domain"):
        oracle.run(t, {"preds": [], "keys": [("x", 0, 2)], "aggs": [], "window": (0, 5)})
    with pytest.raises(oracle.OracleError, match="window"):
        oracle.run(t, dict(q, window=(0, 6)))
    big = {"n_rows": 4, "columns": {"x": {"enc": "rle", "values": np.array([2**62], dtype=np.int64),
                                          "run_ends": np.array([4], dtype=np.int64)}}}
    with pytest.raises(oracle.OracleError, match="overflow"):
        oracle.run(big, {"preds": [], "keys": [], "aggs": [("sum", "x")], "window": (0, 4)})


def test_empty_results():
    t = {"n_rows": 10, "columns": {"x": {"enc": "rle", "values": np.array([1, 2], dtype=np.int32),
                                         "run_ends": np.array([4, 10], dtype=np.int64)}}}
    r = oracle.run(t, {"preds": [("x", "range", 5, 9)], "keys": [], "aggs": [("sum", "x"), ("count",)],
                       "window": (0, 10)})
    assert r == {"keys": [()], "counts": [0], "aggs": [(0, 0)]}
    r = oracle.run(t, {"preds": [("x", "range", 5, 9)], "keys": [("x", 0, 4)], "aggs": [("count",)],
                       "window": (0, 10)})
    assert r == {"keys": [], "counts": [], "aggs": []}
    r = oracle.run(t, {"preds": [], "keys": [], "aggs": [("count",)], "window": (3, 3)})
    assert r["counts"] == [0]


# ---- NOT (Section 5.3): the mask algorithms against the paper's worked
# examples and against a row-by-row complement; negated predicates in the
# oracle against brute force and SQL

def test_not_mask_algorithms_paper_examples():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "not_masks.json")))
    a = g["not_rle"]
    assert oracle.not_rle(a["start"], a["end"], a["total_size"]) == (a["start_out"], a["end_out"])
    b = g["not_index"]
    assert oracle.not_index(b["pos"], b["total_size"]) == (b["start_out"], b["end_out"])


def _rows_of_ranges(start, end, n):
    m = [False] * n
    for s, e in zip(start, end):
        for r in range(s, e + 1):
            m[r] = True
    return m


@pytest.mark.parametrize("seed", range(40))
def test_not_masks_are_row_complements(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    rows = sorted(set(int(x) for x in rng.integers(0, n, size=int(rng.integers(0, n + 1)))))
    # an RLE mask: maximal ranges of the chosen rows
    start, end = [], []
    for r in rows:
        if end and end[-1] == r - 1:
            end[-1] = r
        else:
            start.append(r)
            end.append(r)
    want = [not x for x in _rows_of_ranges(start, end, n)]
    s2, e2 = oracle.not_rle(start, end, n)
    assert _rows_of_ranges(s2, e2, n) == want
    assert all(a <= b for a, b in zip(s2, e2)) and all(e2[i] + 1 < s2[i + 1] for i in range(len(s2) - 1))
    s3, e3 = oracle.not_index(rows, n)
    assert _rows_of_ranges(s3, e3, n) == want


@pytest.mark.parametrize("seed", range(30))
def test_negated_predicates_match_brute_force_and_sqlite(seed):
    from tests.cases import tiny_query_with_not
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(1, 300))
    t, wd = _tiny_table(rng, n)
    for _ in range(4):
        q = tiny_query_with_not(rng, n, wd)
        got = _norm(oracle.run(t, q, n_threads=1 + seed % 3))
        assert got == _norm(brute.run(t, q)), q
        assert got == _norm(brute.run_sqlite(t, q)), q


# ---- OR (Section 5.2): mask forms against the paper's example and against
# row sets; OR clauses in the oracle against brute force and SQL

def _ranges_of_rows(rows):
    start, end = [], []
    for r in rows:
        if end and end[-1] == r - 1:
            end[-1] = r
        else:
            start.append(r)
            end.append(r)
    return start, end


def test_or_plain_paper_example():
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "or_masks.json")))["or_plain"]
    assert oracle.or_plain(g["m1"], g["m2"]) == g["out"]


@pytest.mark.parametrize("seed", range(40))
def test_or_masks_are_row_unions(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 60))
    a = sorted(set(int(x) for x in rng.integers(0, n, size=int(rng.integers(0, n + 1)))))
    b = sorted(set(int(x) for x in rng.integers(0, n, size=int(rng.integers(0, n + 1)))))
    want = sorted(set(a) | set(b))
    # RLE masks: arbitrary (not necessarily maximal) cuts of the row sets
    sa, ea = _ranges_of_rows(a)
    sb, eb = _ranges_of_rows(b)
    s, e = oracle.range_union(sa, ea, sb, eb)
    assert _rows_of_ranges(s, e, n) == [r in set(want) for r in range(n)]
    # the output is maximal: disjoint, sorted, no two ranges touch
    assert all(x <= y for x, y in zip(s, e)) and all(e[i] + 1 < s[i + 1] for i in range(len(s) - 1))
    assert (s, e) == _ranges_of_rows(want)
    # De Morgan with the paper's NOT: a OR b = NOT(NOT a AND NOT b)
    na = set(r for r in range(n) if _rows_of_ranges(*oracle.not_rle(sa, ea, n), n)[r])
    nb = set(r for r in range(n) if _rows_of_ranges(*oracle.not_rle(sb, eb, n), n)[r])
    ns, ne = oracle.not_rle(*_ranges_of_rows(sorted(na & nb)), n)
    assert (ns, ne) == (s, e)
    assert oracle.merge_sorted_idx(a, b) == want
    assert oracle.concat_sort(a, b) == want
    ma = [r in set(a) for r in range(n)]
    mb = [r in set(b) for r in range(n)]
    assert oracle.or_plain(ma, mb) == [r in set(want) for r in range(n)]


@pytest.mark.parametrize("seed", range(20))
def test_or_clause_rows_are_the_union_of_the_column_masks(seed):
    # COUNT(*) under (p1 on r0 OR p2 on r1) equals the rows of range_union
    # of the two columns' RLE masks (the runs whose values pass, as ranges)
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, 400))
    t, wd = _tiny_table(rng, n)

    def mask(col, lo, hi):
        c = t["columns"][col]
        ends = [int(x) for x in c["run_ends"]]
        starts = [0] + ends[:-1]
        rows = []
        for s0, e0, v in zip(starts, ends, c["values"]):
            if lo <= int(v) < hi:
                rows += list(range(s0, e0))
        return _ranges_of_rows(rows)

    l0, l1 = int(rng.integers(-6, 20)), int(rng.integers(-6, 20))
    h0, h1 = l0 + int(rng.integers(0, 10)), l1 + int(rng.integers(0, 10))
    s, e = oracle.range_union(*mask("r0", l0, h0), *mask("r1", l1, h1))
    q = {"preds": [], "or": [[("r0", "range", l0, h0), ("r1", "range", l1, h1)]], "keys": [], "aggs": [("count",)]}
    got = oracle.run(t, q, n_threads=1)
    assert got["counts"] == [sum(y - x + 1 for x, y in zip(s, e))]


@pytest.mark.parametrize("seed", range(30))
def test_or_clauses_match_brute_force_and_sqlite(seed):
    from tests.cases import tiny_query_with_or
    rng = np.random.default_rng(9500 + seed)
    n = int(rng.integers(1, 300))
    t, wd = _tiny_table(rng, n)
    for _ in range(4):
        q = tiny_query_with_or(rng, n, wd)
        got = _norm(oracle.run(t, q, n_threads=1 + seed % 3))
        assert got == _norm(brute.run(t, q)), q
        assert got == _norm(brute.run_sqlite(t, q)), q



@pytest.mark.parametrize("seed", range(30))
def test_rle_index_or_clauses_match_brute_force_and_sqlite(seed):
    """An OR clause over RLE columns and the Index column (unlisted rows
    hold 0), in run mode and beside bit-packed columns."""
    from tests.cases import tiny_query_with_rle_index_or
    rng = np.random.default_rng(9800 + seed)
    n = int(rng.integers(1, 300))
    t, wd = _tiny_table(rng, n)
    for _ in range(4):
        q = tiny_query_with_rle_index_or(rng, n, wd)
        got = _norm(oracle.run(t, q, n_threads=1 + seed % 3))
        assert got == _norm(brute.run(t, q)), q
        assert got == _norm(brute.run_sqlite(t, q)), q


# ---- predicates on Index columns: Algorithm 4 (idx_in_idx) against row
# sets; the oracle's per-row Index predicates against brute force and SQL

@pytest.mark.parametrize("seed", range(30))
def test_idx_in_idx_is_the_row_intersection(seed):
    rng = np.random.default_rng(1100 + seed)
    n = int(rng.integers(1, 80))
    a = sorted(set(int(x) for x in rng.integers(0, n, size=int(rng.integers(0, n + 1)))))
    b = sorted(set(int(x) for x in rng.integers(0, n, size=int(rng.integers(0, n + 1)))))
    assert oracle.idx_in_idx(a, b) == sorted(set(a) & set(b))
    assert oracle.idx_in_idx(b, a) == sorted(set(a) & set(b))


@pytest.mark.parametrize("seed", range(20))
def test_and_of_two_index_predicates_counts_idx_in_idx(seed):
    # two Index columns, predicates that 0 fails: the qualifying rows are
    # idx_in_idx of the two columns' Index masks (their passing points)
    rng = np.random.default_rng(1200 + seed)
    n = int(rng.integers(1, 300))
    cols = {}
    masks = []
    for name in ("s1", "s2"):
        pos = np.sort(rng.choice(n, size=int(rng.integers(0, n + 1)), replace=False)).astype(np.int64)
        val = rng.integers(-20, 20, size=len(pos)).astype(np.int64)
        cols[name] = {"enc": "index", "positions": pos, "values": val}
        masks.append([int(p) for p, v in zip(pos, val) if 3 <= v < 15])
    t = {"n_rows": n, "columns": cols}
    q = {"preds": [("s1", "range", 3, 15), ("s2", "range", 3, 15)], "keys": [], "aggs": [("count",)]}
    assert oracle.run(t, q, n_threads=1)["counts"] == [len(oracle.idx_in_idx(masks[0], masks[1]))]


@pytest.mark.parametrize("seed", range(30))
def test_index_predicates_match_brute_force_and_sqlite(seed):
    from tests.cases import tiny_query_with_index_pred
    rng = np.random.default_rng(9800 + seed)
    n = int(rng.integers(1, 300))
    t, wd = _tiny_table(rng, n)
    for _ in range(4):
        q = tiny_query_with_index_pred(rng, n, wd)
        got = _norm(oracle.run(t, q, n_threads=1 + seed % 3))
        assert got == _norm(brute.run(t, q)), q
        assert got == _norm(brute.run_sqlite(t, q)), q


# ---- dictionary decoding of key columns (Section 2.1, dictionary encoding)

def _dict_table(rng, n, values, order):
    """A column of arbitrary int64 values, dictionary-encoded: a dictionary
    of its distinct values (sorted, or permuted when order == 'shuffled')
    and one bit-packed code per row, plus an RLE column to sum."""
    uniq = np.unique(values)
    dic = uniq.copy() if order == "sorted" else rng.permutation(uniq)
    pos = {int(v): i for i, v in enumerate(dic)}
    codes = np.array([pos[int(v)] for v in values], dtype=np.int64)
    w = max(1, int(len(dic) - 1).bit_length())
    ends = np.cumsum(rng.integers(1, 40, size=n)).astype(np.int64)
    ends = ends[ends < n]
    ends = np.append(ends, n)
    cols = {"v": {"enc": "bitpacked", "packed": datagen.pack_codes(codes, w), "w": w, "base": 0, "dict": dic},
            "m": {"enc": "rle", "values": rng.integers(-1000, 1000, size=len(ends)).astype(np.int64),
                  "run_ends": ends}}
    return {"n_rows": n, "columns": cols}, dic, codes


@pytest.mark.parametrize("order", ["sorted", "shuffled"])
@pytest.mark.parametrize("seed", range(6))
def test_dictionary_keys_round_trip(seed, order):
    """GROUP BY a dictionary-encoded column reports the original values:
    with a sorted dictionary the result is np.unique of the decoded column
    (values and counts); with a permuted one the groups come in code order
    and each reports dict[code].  Per-group SUMs of another column are the
    row-level sums over the rows holding that value."""
    rng = np.random.default_rng([seed, 31])
    n = int(rng.integers(1, 5000))
    pool = rng.integers(-(1 << 62), 1 << 62, size=int(rng.integers(1, 300)), dtype=np.int64)
    values = pool[rng.integers(0, len(pool), size=n)]
    t, dic, codes = _dict_table(rng, n, values, order)
    q = {"preds": [], "keys": [("v", 0, len(dic))], "aggs": [("count",), ("sum", "m")], "window": (0, n)}
    got = oracle.run(t, q, n_threads=3)
    m_rows = np.repeat(t["columns"]["m"]["values"],
                       np.diff(np.concatenate([[0], t["columns"]["m"]["run_ends"]])))
    if order == "sorted":
        u, cnt = np.unique(values, return_counts=True)
        assert got["keys"] == [(int(x),) for x in u]
        assert got["counts"] == [int(x) for x in cnt]
    else:
        present = sorted(set(int(c) for c in codes))
        assert got["keys"] == [(int(dic[c]),) for c in present]
        assert got["counts"] == [int((codes == c).sum()) for c in present]
    sums = [int(m_rows[values == k[0]].sum()) for k in got["keys"]]
    assert [a[1] for a in got["aggs"]] == sums


def test_dictionary_rules():
    rng = np.random.default_rng(5)
    t, dic, _ = _dict_table(rng, 100, rng.integers(0, 9, size=100), "sorted")
    base = {"preds": [], "aggs": [("count",)], "window": (0, 100)}
    with pytest.raises(oracle.OracleError):
        oracle.run(t, dict(base, keys=[("v", 1, 4)]))                  # shifted dictionary key
    with pytest.raises(oracle.OracleError):
        oracle.run(t, dict(base, keys=[("v", 0, len(dic) + 1)]))       # domain beyond the dictionary
    with pytest.raises(oracle.OracleError):
        oracle.run(t, dict(base, keys=[], aggs=[("sum", "v")]))        # SUM over dictionary codes


# ------------------------------------------------------------------ MIN, MAX, column arithmetic, AVG / VAR

@pytest.mark.parametrize("seed", range(40))
def test_min_max_and_expressions_match_brute_force_and_sqlite(seed):
    from tests.cases import tiny_query_with_exprs
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(1, 300))
    t, wd = _tiny_table(rng, n)
    for _ in range(4):
        q = tiny_query_with_exprs(rng, n, wd)
        got = _norm(oracle.run(t, q, n_threads=1 + seed % 3))
        assert got == _norm(brute.run(t, q)), q
        assert got == _norm(brute.run_sqlite(t, q)), q


@pytest.mark.parametrize("seed", range(10))
def test_expression_invariants(seed):
    """SUM(a + b) = SUM(a) + SUM(b), SUM(a - b) = SUM(a) - SUM(b); the
    ungrouped MIN / MAX are the extremes of the per-group ones."""
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(50, 400))
    t, wd = _tiny_table(rng, n)
    base = {"preds": [("r0", "range", -3, 12)], "window": (0, n)}
    r = oracle.run(t, dict(base, keys=[], aggs=[("sum", ("r1", "+", "p")), ("sum", "r1"), ("sum", "p"),
                                                 ("sum", ("r1", "-", "p")), ("min", "r1"), ("max", "r1")]))
    a = r["aggs"][0]
    assert a[0] == a[1] + a[2] and a[3] == a[1] - a[2]
    g = oracle.run(t, dict(base, keys=[("d", 0, 1 << wd)], aggs=[("min", "r1"), ("max", "r1")]))
    if g["keys"]:
        assert a[4] == min(x[0] for x in g["aggs"]) and a[5] == max(x[1] for x in g["aggs"])


def test_avg_var_post_processing():
    """AVG and VAR from COUNT, SUM and SUM(x * x): exact on small cases,
    within a few ulps of the exact rational otherwise."""
    from fractions import Fraction
    assert oracle.avg_var(4, 4, 8) == (1.0, 1.0)          # values 0, 2, 0, 2
    assert oracle.avg_var(3, 21, 147) == (7.0, 0.0)        # a constant 7
    assert oracle.avg_var(0, 0, 0) == (0.0, 0.0)
    rng = np.random.default_rng(9)
    for _ in range(200):
        x = rng.integers(-10**6, 10**6, size=int(rng.integers(1, 500)))
        n, s, ss = len(x), int(x.sum()), int((x.astype(object) ** 2).sum())
        avg, var = oracle.avg_var(n, s, ss)
        ea = Fraction(s, n)
        ev = Fraction(ss, n) - ea * ea
        assert abs(Fraction(avg) - ea) <= abs(ea) * Fraction(1, 2**50) + Fraction(1, 2**60)
        assert abs(Fraction(var) - ev) <= abs(Fraction(ss, n)) * Fraction(1, 2**45) + Fraction(1, 2**40)
    # on a table: VAR of r1 from one query's COUNT, SUM(r1) and SUM(r1 * r1)
    rng = np.random.default_rng(10)
    t, wd = _tiny_table(rng, 300)
    r = oracle.run(t, {"preds": [], "keys": [], "aggs": [("count",), ("sum", "r1"), ("sum", ("r1", "*", "r1"))],
                       "window": (0, 300)})
    vals = np.array(brute.decode_rows(t["columns"]["r1"], 300), dtype=np.float64)
    avg, var = oracle.avg_var(*r["aggs"][0])
    assert abs(avg - vals.mean()) < 1e-12 * max(1.0, abs(vals.mean()))
    assert abs(var - vals.var()) < 1e-9 * max(1.0, vals.var())
