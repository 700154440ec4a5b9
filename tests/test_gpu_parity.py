"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle,
element by element, on the same seeded inputs.  Integer results must match
bit for bit."""
import json
import os
import sys

import numpy as np
import pytest

import datagen
from oracle import oracle
from tests.cases import tiny_query, tiny_table

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_10092_amd import ccq
    assert torch.cuda.is_available()
    return ccq.Context(0)


def gpu_run(ctx, table, query, repeat=1):
    from paper_2506_10092_amd import ccq
    dev = ccq.to_device(table["columns"])
    t = ccq.Table(ctx, table["n_rows"], dev)
    p = ccq.Plan(t, query)
    ws, res = p.new_workspace(), p.new_result()
    outs = []
    for _ in range(repeat):
        p.execute(ws, res)
        outs.append(res.to_python())
    for o in outs[1:]:
        assert o == outs[0], "repeated execution differs"
    return outs[0]


def check(ctx, table, query, n_threads=None, repeat=1):
    exp = oracle.run(table, query, n_threads=n_threads)
    got = gpu_run(ctx, table, query, repeat=repeat)
    assert got["status"] == 0, got["status"]
    assert got["keys"] == exp["keys"], "keys differ"
    assert got["counts"] == exp["counts"], "counts differ"
    assert got["aggs"] == exp["aggs"], "aggregates differ"
    return got


def _np_col(c):
    c = dict(c)
    if c["enc"] == "rle":
        c["values"] = np.array(c["values"], dtype=np.int64)
        c["run_ends"] = np.array(c["run_ends"], dtype=np.int64)
    elif c["enc"] == "index":
        c["positions"] = np.array(c["positions"], dtype=np.int32)
        c["values"] = np.array(c["values"], dtype=np.int64)
    return c


@pytest.mark.parametrize("name", ["range_intersect.json", "idx_in_rle.json", "alignment.json", "groupby.json"])
def test_paper_examples(ctx, name):
    g = json.load(open(os.path.join(GOLDEN, name)))
    table = {"n_rows": g["n_rows"], "columns": {k: _np_col(v) for k, v in g["columns"].items()}}
    for q in g["queries"]:
        query = {"preds": [tuple(p) for p in q["preds"]], "keys": [tuple(k) for k in q["keys"]],
                 "aggs": [tuple(tuple(x) if isinstance(x, list) else x for x in a) for a in q["aggs"]],
                 "window": (0, g["n_rows"])}
        got = check(ctx, table, query)
        assert got["counts"] == q["expect"]["counts"]
        assert [list(a) for a in got["aggs"]] == q["expect"]["aggs"]


@pytest.mark.parametrize("seed", range(40))
def test_tiny_random_tables(ctx, seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(1, 5000))
    t, wd = tiny_table(rng, n)
    for _ in range(3):
        q = tiny_query(rng, n, wd)
        say("tiny seed", seed, "n", n, "query", q)
        check(ctx, t, q)


def test_c1_full(ctx):
    c = datagen.config_c1()
    say("c1", c["n_rows"])
    got = check(ctx, c, c["query"], repeat=3)
    assert got["counts"][0] > 0


@pytest.mark.parametrize("window", [None, (0, 2048), (1, 2047), (12_345, 9_876_543), (5_000_000, 5_000_000),
                                    (19_999_990, 20_000_000), (777, 778)])
def test_c2_windows(ctx, window):
    c = datagen.config_c2(n_rows=20_000_003)
    q = dict(c["query"])
    if window:
        q["window"] = window
    say("c2 2e7 window", q["window"])
    check(ctx, c, q)


def test_c2_more_templates(ctx):
    c = datagen.config_c2(n_rows=5_000_017, columns=("r0", "r1", "r2", "s", "d", "p"))
    n = c["n_rows"]
    in_codes = c["query"]["preds"][2][2]
    queries = [
        # RLE-only with sparse SUM (run mode + idx_in_rle probe)
        {"preds": [("r0", "range", 0, 30000)], "keys": [("r2", 12, 16)], "aggs": [("sum", "s"), ("count",)]},
        # SUM over RLE and bit-packed in row mode, RLE key with shift
        {"preds": [("d", "in", in_codes[:7])], "keys": [("r1", 10, 64)], "aggs": [("sum", "r2"), ("sum", "p")]},
        # range on the 20-bit column (no code table), dict key without IN
        {"preds": [("p", "range", -100000, 250000)], "keys": [("d", 0, 10000)], "aggs": [("count",), ("sum", "s")]},
        # three predicates, ungrouped, several sums
        {"preds": [("r0", "range", 1000, 60000), ("r1", "range", 0, 50000), ("p", "range", 0, 1 << 19)],
         "keys": [], "aggs": [("sum", "r0"), ("sum", "p"), ("sum", "s"), ("count",)]},
        # composite predicates on one column (folded), IN on an RLE column
        {"preds": [("r0", "range", 0, 40000), ("r0", "range", 20000, 60000), ("r1", "in", list(range(0, 65536, 7)))],
         "keys": [("r0", 8, 256)], "aggs": [("count",)]},
        # global-table mode: 2 keys, 64k groups
        {"preds": [], "keys": [("r0", 8, 256), ("r1", 8, 256)], "aggs": [("sum", "r2"), ("count",)]},
    ]
    for q in queries:
        q["window"] = (0, n)
        say("c2 template", q)
        check(ctx, c, q)


def test_c3_small(ctx):
    c = datagen.config_c3(n_rows=30_000_001)
    say("c3 3e7")
    check(ctx, c, c["query"])


def _rle(values, ends, dt=np.int64):
    return {"enc": "rle", "values": np.asarray(values, dtype=dt), "run_ends": np.asarray(ends, dtype=np.int64)}


def test_unit_runs_force_short_tiles(ctx):
    """Every run one row long in 8 RLE columns: tiles must end early."""
    n = 300_000
    rng = np.random.default_rng(7)
    cols = {"c%d" % i: _rle(rng.integers(0, 4, n), np.arange(1, n + 1), np.int32) for i in range(8)}
    t = {"n_rows": n, "columns": cols}
    q = {"preds": [("c0", "range", 1, 4), ("c3", "range", 0, 3)], "keys": [("c1", 0, 4), ("c2", 0, 4)],
         "aggs": [("sum", "c4"), ("sum", "c7"), ("count",)], "window": (0, n)}
    check(ctx, t, q)
    q["window"] = (1234, 250_001)
    check(ctx, t, q)


def test_unit_runs_with_packed_column(ctx):
    n = 100_003
    rng = np.random.default_rng(8)
    codes = rng.integers(0, 1 << 9, n).astype(np.uint32)
    cols = {"a": _rle(rng.integers(0, 3, n), np.arange(1, n + 1)),
            "b": _rle(rng.integers(0, 3, n // 3 + 1), np.r_[np.arange(3, n, 3), n]),
            "d": {"enc": "bitpacked", "packed": datagen.pack_codes(codes, 9), "w": 9, "base": 0}}
    t = {"n_rows": n, "columns": cols}
    q = {"preds": [("a", "range", 1, 3), ("d", "range", 100, 400)], "keys": [("d", 5, 16), ("b", 0, 3)],
         "aggs": [("sum", "a"), ("sum", "d"), ("count",)], "window": (0, n)}
    check(ctx, t, q)


def test_single_long_run_and_empty_filters(ctx):
    n = 7_000_001
    t = {"n_rows": n, "columns": {"x": _rle([42], [n]), "y": _rle([1, 2, 3], [10, n - 5, n], np.int32)}}
    for q in [
        {"preds": [], "keys": [], "aggs": [("sum", "x"), ("count",)]},
        {"preds": [("y", "range", 2, 3)], "keys": [("y", 0, 4)], "aggs": [("sum", "x")]},
        {"preds": [("y", "range", 7, 9)], "keys": [], "aggs": [("sum", "x"), ("count",)]},
        {"preds": [("y", "range", 7, 9)], "keys": [("y", 0, 4)], "aggs": [("count",)]},
        {"preds": [("y", "in", [])], "keys": [], "aggs": [("count",)]},
    ]:
        q["window"] = (3, n - 2)
        check(ctx, t, q)


@pytest.mark.parametrize("w", [1, 7, 13, 14, 15, 20, 31, 32])
def test_bit_widths(ctx, w):
    n = 70_001
    rng = np.random.default_rng(w)
    codes = rng.integers(0, 1 << w, n, dtype=np.uint64).astype(np.uint32)
    base = -(1 << (w - 1))
    t = {"n_rows": n, "columns": {
        "p": {"enc": "bitpacked", "packed": datagen.pack_codes(codes, w), "w": w, "base": base},
        "r": _rle(rng.integers(0, 5, n // 50 + 1), np.r_[np.sort(rng.choice(np.arange(1, n), n // 50, replace=False)), n]),
        "s": {"enc": "index", "positions": np.sort(rng.choice(n, 700, replace=False)).astype(np.int64),
              "values": rng.integers(-5, 5, 700).astype(np.int32)}}}
    lo = base + (1 << w) // 5
    hi = base + (1 << w) * 4 // 5 + 1
    shift = max(0, w - 4)
    qs = [{"preds": [("p", "range", lo, hi)], "keys": [], "aggs": [("sum", "p"), ("sum", "s"), ("count",)]},
          {"preds": [("p", "range", 0, 1 << 40)], "keys": [("p", shift, 16)], "aggs": [("sum", "s"), ("count",)]},
          {"preds": [("r", "range", 1, 4)], "keys": [("r", 0, 5)], "aggs": [("sum", "p")]}]
    for q in qs:
        q["window"] = (5, n)
        check(ctx, t, q)


def test_key_domain_violation_sets_status(ctx):
    n = 10_000
    t = {"n_rows": n, "columns": {"x": _rle([0, 1, 9, 2], [100, 200, 300, n])}}
    got = gpu_run(ctx, t, {"preds": [], "keys": [("x", 0, 4)], "aggs": [("count",)], "window": (0, n)})
    assert got["status"] == -4
    # the violating run filtered out: no error
    q = {"preds": [("x", "range", 0, 4)], "keys": [("x", 0, 4)], "aggs": [("count",)], "window": (0, n)}
    check(ctx, t, q)
    codes = np.array([1, 2, 3, 17] * 25, dtype=np.uint32)
    t2 = {"n_rows": 100, "columns": {"d": {"enc": "bitpacked", "packed": datagen.pack_codes(codes, 5), "w": 5, "base": 0}}}
    got = gpu_run(ctx, t2, {"preds": [], "keys": [("d", 0, 8)], "aggs": [("count",)], "window": (0, 100)})
    assert got["status"] == -4


def test_int64_positions_and_int32_values(ctx):
    n = 3_000_000
    c = datagen.config_c2(n_rows=n, columns=("r0", "s", "d"))
    c["columns"]["s"]["positions"] = c["columns"]["s"]["positions"].astype(np.int64)
    c["columns"]["s"]["values"] = c["columns"]["s"]["values"].astype(np.int32)
    q = {"preds": [("r0", "range", 0, 40000), ("d", "in", list(range(0, 200, 3)))], "keys": [("d", 0, 10000)],
         "aggs": [("sum", "s"), ("count",)], "window": (0, n)}
    check(ctx, c, q)


@pytest.mark.parametrize("q", [
    # GROUP BY the 14-bit dictionary column without an IN-list: 10,000 slots
    {"preds": [("r0", "range", 0, 40000)], "keys": [("d", 0, 10000)], "aggs": [("count",), ("sum", "s")]},
    {"preds": [("d", "range", 100, 9000), ("r1", "range", 5000, 60000)], "keys": [("d", 0, 10000)],
     "aggs": [("count",)]},
    # GROUP BY the 20-bit column shifted: 2^20 >> 7 = 8192 slots, window cut mid-word
    {"preds": [("r0", "range", 10000, 50000)], "keys": [("p", 7, 8192)], "aggs": [("sum", "s"), ("count",)]},
    # the key's domain excludes part of the column (domain errors are a status, checked elsewhere)
    {"preds": [("p", "range", -(1 << 19), 0)], "keys": [("p", 6, 16384)], "aggs": [("count",)]},
])
def test_large_group_table_fast_path(ctx, q):
    """Fast row path with a group table too large to replicate: uint32 counts
    in dynamic LDS, slots computed from the code, Index sums added to the
    global table."""
    n = 3_000_017
    t = datagen.config_c2(seed=61, n_rows=n, columns=("r0", "r1", "s", "d", "p"))
    for window in ((0, n), (77, n - 5)):
        qq = dict(q, window=window)
        if q["keys"][0][0] == "p":
            # codes of p reach keys below 0 ((base + code) >> shift < 0): restrict to the non-negative half
            qq["preds"] = [x for x in q["preds"] if x[0] != "p"] + [("p", "range", 0, 1 << 19)]
        got = check(ctx, t, qq)
        say("groups", len(got["keys"]))


def _geometric_runs(rng, n, mean, vlo, vhi, dt=np.int32):
    """RLE column over n rows with geometric run lengths of the given mean."""
    lens = rng.geometric(1.0 / mean, size=int(n / mean * 1.3) + 64)
    ends = np.cumsum(lens)
    ends = ends[ends < n]
    ends = np.r_[ends, n]
    return _rle(rng.integers(vlo, vhi, len(ends)), ends, dt)


def _index_col(rng, n, density):
    keep = rng.random(n) < density
    pos = np.flatnonzero(keep).astype(np.int32)
    return {"enc": "index", "positions": pos, "values": rng.integers(1, 1_000_000, len(pos)).astype(np.int64)}


@pytest.mark.parametrize("mean_run", [1, 5, 64])
@pytest.mark.parametrize("density", [0.05, 0.3, 1.0])
def test_fast_path_short_runs_and_dense_points(ctx, mean_run, density):
    """The single-packed-column row path with runs shorter than a batch per
    tile pass (several run batches per pass) and with more than 64 Index
    points per pass (the batch-by-batch point route); windows cut tiles."""
    n = 1_000_003
    rng = np.random.default_rng(1000 + mean_run * 10 + int(density * 10))
    codes = rng.integers(0, 700, n).astype(np.uint32)
    cols = {"r0": _geometric_runs(rng, n, mean_run, 0, 4),
            "r1": _geometric_runs(rng, n, 200, 0, 4),
            "s": _index_col(rng, n, density),
            "d": {"enc": "bitpacked", "packed": datagen.pack_codes(codes, 14), "w": 14, "base": 0}}
    t = {"n_rows": n, "columns": cols}
    in_codes = [int(x) for x in rng.choice(700, 40, replace=False)]
    q = {"preds": [("r0", "range", 1, 3), ("r1", "range", 0, 3), ("d", "in", in_codes)],
         "keys": [("d", 0, 1 << 14)], "aggs": [("sum", "s"), ("count",)], "window": (0, n)}
    say("fast path mean_run", mean_run, "density", density)
    check(ctx, t, q)
    q["window"] = (12_345, n - 777)
    check(ctx, t, q)


@pytest.mark.parametrize("density", [0.01, 0.5])
def test_fast_path_20bit_code_range(ctx, density):
    """The 20-bit row path without a code table (a code range and a shifted
    key), with RLE predicates and an Index SUM."""
    n = 777_777
    rng = np.random.default_rng(77 + int(density * 100))
    codes = rng.integers(0, 1 << 20, n).astype(np.uint32)
    cols = {"r0": _geometric_runs(rng, n, 30, 0, 8),
            "s": _index_col(rng, n, density),
            "p": {"enc": "bitpacked", "packed": datagen.pack_codes(codes, 20), "w": 20, "base": -(1 << 19)}}
    t = {"n_rows": n, "columns": cols}
    q = {"preds": [("r0", "range", 2, 7), ("p", "range", -100_000, 300_000)],
         "keys": [("p", 14, 64)], "aggs": [("sum", "s"), ("count",)], "window": (0, n)}
    # keys of negative values fall outside [0, card): keep them out with the range
    q["preds"][1] = ("p", "range", 0, 300_000)
    say("20-bit fast path density", density)
    check(ctx, t, q)
    q["window"] = (31, n - 1)
    check(ctx, t, q)


# ---- NOT (Section 5.3): negated predicates, alone and stacked with plain
# ones on one column, on every kernel path

@pytest.mark.parametrize("seed", range(30))
def test_tiny_random_tables_with_not(ctx, seed):
    from tests.cases import tiny_query_with_not
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(1, 5000))
    t, wd = tiny_table(rng, n)
    for _ in range(3):
        q = tiny_query_with_not(rng, n, wd)
        say("tiny NOT seed", seed, "n", n, "query", q)
        check(ctx, t, q)


@pytest.mark.parametrize("seed", range(30))
def test_tiny_random_tables_with_or(ctx, seed):
    from tests.cases import tiny_query_with_or
    rng = np.random.default_rng(7500 + seed)
    n = int(rng.integers(1, 5000))
    t, wd = tiny_table(rng, n)
    for _ in range(3):
        q = tiny_query_with_or(rng, n, wd)
        say("tiny OR seed", seed, "n", n, "query", q)
        check(ctx, t, q)


def test_or_on_fast_path_run_mode_and_generic_paths(ctx):
    """OR clauses over the RLE columns (Section 5.2, range_union): on the
    fast path (dictionary column), in run mode (no bit-packed column) and on
    the generic row path (20-bit column); a column named in the clause-0
    predicates and in two OR clauses (three slots); clauses with a false
    predicate, an always-true predicate, and a clause no row passes."""
    n = 2_000_003
    t = datagen.config_c2(seed=93, n_rows=n, columns=("r0", "r1", "s", "d", "p"))
    in_codes = t["query"]["preds"][2][2]
    fast = {"keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)]}
    queries = [
        dict(fast, preds=[("d", "in", in_codes)], **{"or": [[("r0", "range", 0, 20000), ("r1", "range", 50000, 65536)]]}),
        dict(fast, preds=[("r0", "range", 0, 40000), ("d", "in", in_codes)],
             **{"or": [[("r0", "not_range", 5000, 30000), ("r1", "in", list(range(0, 65536, 3)))]]}),
        dict(fast, preds=[("d", "not_in", in_codes[:5])],
             **{"or": [[("r0", "range", 0, 10000), ("r1", "range", 60000, 65536)],
                       [("r0", "range", 30000, 65536), ("r1", "not_range", 20000, 65536)]]}),
        {"preds": [], "keys": [("r0", 10, 64)], "aggs": [("sum", "r1"), ("count",)],
         "or": [[("r0", "range", 0, 8000), ("r1", "range", 30000, 40000), ("r0", "in", [60000, 60001])]]},
        {"preds": [("p", "range", -200_000, 400_000)], "keys": [], "aggs": [("sum", "p"), ("sum", "s"), ("count",)],
         "or": [[("r1", "range", 0, 16384), ("r0", "not_range", 0, 60000)]]},
        dict(fast, preds=[("d", "in", in_codes)],
             **{"or": [[("r0", "in", []), ("r1", "range", 0, 30000)], [("r1", "not_in", []), ("r0", "range", 0, 10)]]}),
        dict(fast, preds=[("d", "in", in_codes)], **{"or": [[("r0", "in", []), ("r1", "range", 5, 5)]]}),
    ]
    for q in queries:
        for window in ((0, n), (4097, n - 31)):
            qq = dict(q, window=window)
            say("OR query", qq["preds"], qq["or"], window)
            check(ctx, t, qq)


@pytest.mark.parametrize("seed", range(30))
def test_tiny_random_tables_with_index_predicates(ctx, seed):
    from tests.cases import tiny_query_with_index_pred
    rng = np.random.default_rng(7800 + seed)
    n = int(rng.integers(1, 5000))
    t, wd = tiny_table(rng, n)
    for _ in range(3):
        q = tiny_query_with_index_pred(rng, n, wd)
        say("tiny Index-predicate seed", seed, "n", n, "query", q)
        check(ctx, t, q)


def test_or_across_rle_and_bitpacked_columns(ctx):
    """One OR clause over RLE and bit-packed columns (Table 4, RLE mask OR
    Plain mask): its RLE part is a mask of its own and each row is tested on
    its codes; with other clauses, a key on the dictionary column, windows."""
    n = 2_000_003
    t = datagen.config_c2(seed=97, n_rows=n, columns=("r0", "r1", "s", "d", "p"))
    in_codes = t["query"]["preds"][2][2]
    queries = [
        {"preds": [], "keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)],
         "or": [[("r0", "range", 0, 4000), ("d", "in", in_codes[:20])]]},
        {"preds": [("d", "in", in_codes)], "keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)],
         "or": [[("r1", "range", 60000, 65536), ("r0", "in", [5, 6, 7]), ("p", "range", -1000, 20_000)],
                [("r0", "range", 0, 40000), ("r1", "range", 0, 30000)]]},
        {"preds": [("r1", "range", 0, 50000)], "keys": [], "aggs": [("sum", "p"), ("sum", "r0"), ("count",)],
         "or": [[("d", "not_in", in_codes), ("p", "not_range", -400_000, 400_000)]]},
    ]
    for q in queries:
        for window in ((0, n), (4097, n - 31)):
            qq = dict(q, window=window)
            say("mixed OR query", qq["preds"], qq["or"], window)
            check(ctx, t, qq)


@pytest.mark.parametrize("seed", range(30))
def test_tiny_random_tables_with_rle_index_or(ctx, seed):
    from tests.cases import tiny_query_with_rle_index_or
    rng = np.random.default_rng(7900 + seed)
    n = int(rng.integers(1, 5000))
    t, wd = tiny_table(rng, n)
    for _ in range(3):
        q = tiny_query_with_rle_index_or(rng, n, wd)
        say("tiny RLE-Index OR seed", seed, "n", n, "query", q)
        check(ctx, t, q)


def test_or_across_rle_and_index_columns(ctx):
    """One OR clause over RLE columns and the Index column (Table 4, RLE mask
    OR Index mask; unlisted rows hold 0): in run mode (no bit-packed column)
    and on the generic row path, with a predicate 0 fails and one 0 passes,
    beside an OR clause over RLE columns alone, in windows."""
    n = 2_000_003
    t = datagen.config_c2(seed=99, n_rows=n, columns=("r0", "r1", "s", "d", "p"))
    in_codes = t["query"]["preds"][2][2]
    queries = [
        {"preds": [("r1", "range", 0, 50000)], "keys": [], "aggs": [("sum", "s"), ("sum", "r0"), ("count",)],
         "or": [[("r0", "range", 0, 4000), ("s", "range", 1, 300_000)]]},
        {"preds": [], "keys": [("r1", 12, 16)], "aggs": [("sum", "s"), ("count",)],
         "or": [[("r0", "range", 60000, 65536), ("s", "not_range", 100, 200_000)]]},
        {"preds": [("d", "in", in_codes)], "keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)],
         "or": [[("r0", "range", 0, 20000), ("r1", "in", [1, 2, 3]), ("s", "range", 1000, 500_000)]]},
        {"preds": [("p", "range", -200_000, 400_000)], "keys": [], "aggs": [("sum", "p"), ("sum", "s"), ("count",)],
         "or": [[("r0", "range", 0, 30000), ("r1", "range", 0, 30000)],
                [("s", "in", [0]), ("r1", "range", 40000, 65536)]]},
    ]
    for q in queries:
        for window in ((0, n), (4097, n - 31)):
            qq = dict(q, window=window)
            say("RLE-Index OR query", qq["preds"], qq["or"], window)
            check(ctx, t, qq)


def test_index_predicates_run_mode_and_row_mode(ctx):
    """Predicates on the Index column (1% of rows listed, values >= 1, 0
    elsewhere): one that 0 fails (only listed rows can qualify: idx_in_rle),
    one that 0 passes (every unlisted row qualifies: the complement of the
    failing points), with and without the dictionary column, in a window."""
    n = 2_000_003
    t = datagen.config_c2(seed=95, n_rows=n, columns=("r0", "r1", "s", "d", "p"))
    in_codes = t["query"]["preds"][2][2]
    queries = [
        {"preds": [("s", "range", 1, 500_000), ("r0", "range", 0, 32768)], "keys": [("r1", 12, 16)],
         "aggs": [("sum", "s"), ("count",)]},
        {"preds": [("s", "not_range", 1, 300_000), ("r1", "range", 16384, 65536)], "keys": [],
         "aggs": [("sum", "s"), ("sum", "r0"), ("count",)]},
        {"preds": [("s", "range", 250_000, 750_000), ("d", "in", in_codes)], "keys": [("d", 0, 10000)],
         "aggs": [("sum", "s"), ("count",)]},
        {"preds": [("s", "not_in", [1, 2, 3]), ("p", "range", -100_000, 300_000)], "keys": [],
         "aggs": [("sum", "p"), ("count",)], "or": [[("s", "range", 0, 1), ("s", "range", 900_000, 10**6)]]},
    ]
    for q in queries:
        for window in ((0, n), (4097, n - 31)):
            qq = dict(q, window=window)
            say("Index-predicate query", qq["preds"], qq.get("or"), window)
            check(ctx, t, qq)


def test_not_on_fast_path_and_generic_paths(ctx):
    """NOT IN on the dictionary column (folded into its code table on the
    fast path), NOT ranges on RLE columns, and a 20-bit column whose plain
    and negated ranges leave two intervals (the generic row path)."""
    n = 2_000_003
    t = datagen.config_c2(seed=91, n_rows=n, columns=("r0", "r1", "s", "d", "p"))
    base = t["query"]
    in_codes = base["preds"][2][2]
    queries = [
        {"preds": [("r0", "not_range", 0, 32768), ("r1", "range", 16384, 65536), ("d", "in", in_codes)],
         "keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)]},
        {"preds": [("r0", "range", 0, 50000), ("r0", "not_range", 10000, 20000), ("d", "not_in", in_codes[:10]),
                   ("d", "range", 0, 200)],
         "keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)]},
        {"preds": [("p", "range", -200_000, 400_000), ("p", "not_range", -1000, 5000), ("r1", "not_in", [1, 2, 3])],
         "keys": [], "aggs": [("sum", "p"), ("sum", "s"), ("count",)]},
        {"preds": [("r0", "not_in", list(range(0, 65536, 2))), ("r1", "not_range", 0, 100)],
         "keys": [("r0", 10, 64)], "aggs": [("sum", "r1"), ("count",)]},
        # NOT of a range open to the left: every value from 1000 up
        {"preds": [("r1", "not_range", -(1 << 63), 1000), ("d", "in", in_codes)],
         "keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)]},
        {"preds": [("p", "not_range", -(1 << 63), -1000), ("p", "not_range", 2000, 1 << 62)],
         "keys": [], "aggs": [("sum", "p"), ("count",)]},
    ]
    for q in queries:
        for window in ((0, n), (4097, n - 31)):
            qq = dict(q, window=window)
            say("NOT query", qq["preds"], window)
            check(ctx, t, qq)


def test_table_validate_rejects_malformed_columns(ctx):
    """ccq_table_validate: well-formed columns pass; run ends that do not
    increase, a last run end other than the row count and a position out of
    range are rejected, naming the column (also past the 64th)."""
    import torch
    from paper_2506_10092_amd import ccq
    n = 1000
    t = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")

    def table(bad_col=None, bad=None):
        cols = {}
        for i in range(70):
            cols["c%d" % i] = {"enc": "rle", "values": t([1, 2, 3], torch.int32), "run_ends": t([10, 500, n], torch.int64)}
        cols["s"] = {"enc": "index", "positions": t([3, 7, 999], torch.int32), "values": t([1, 2, 3], torch.int64)}
        if bad_col is not None:
            cols[bad_col] = bad
        return ccq.Table(ctx, n, cols)

    table().validate()
    cases = [("c3", {"enc": "rle", "values": t([1, 2, 3], torch.int32), "run_ends": t([10, 10, n], torch.int64)}, 3),
             ("c68", {"enc": "rle", "values": t([1, 2], torch.int32), "run_ends": t([10, n - 1], torch.int64)}, 68),
             ("s", {"enc": "index", "positions": t([3, 7, n], torch.int32), "values": t([1, 2, 3], torch.int64)}, 70),
             ("s", {"enc": "index", "positions": t([3, 3, 9], torch.int32), "values": t([1, 2, 3], torch.int64)}, 70)]
    for name, bad, idx in cases:
        with pytest.raises(ccq.CcqError, match="column %d:" % idx):
            table(name, bad).validate()
    say("table validation: good table passes, %d malformed columns rejected" % len(cases))


@pytest.mark.parametrize("shape", ["fast_in", "fast_big", "generic", "batch"])
def test_dictionary_keys_decode(ctx, shape):
    """GROUP BY a dictionary-encoded column: every kernel path reports
    dict[code] (values unlike the codes, permuted, negative and 64-bit
    wide), equal to the oracle."""
    from paper_2506_10092_amd import ccq
    n = 1_500_007
    t = datagen.config_c2(seed=12, n_rows=n, columns=datagen.C2_COLS)
    rng = np.random.default_rng(77)
    t["columns"]["d"]["dict"] = rng.permutation(
        rng.integers(-(1 << 62), 1 << 62, size=10_000, dtype=np.int64))
    base = t["query"]
    q = {"fast_in": base,
         "fast_big": dict(base, preds=base["preds"][:2], aggs=[("count",)]),
         "generic": dict(base, aggs=[("sum", "p"), ("sum", "s"), ("count",)]),
         "batch": base}[shape]
    say("dictionary case:", shape)
    if shape == "batch":
        tb = ccq.Table(ctx, n, ccq.to_device(t["columns"]))
        qs = [q, dict(q, window=(1000, 700_000)), dict(q, aggs=[("sum", "p"), ("count",)])]
        b = ccq.Batch(ctx, [ccq.Plan(tb, x) for x in qs])
        ws = b.new_workspace()
        b.execute(ws)
        got = b.to_python()
        for x, g in zip(qs, got):
            exp = oracle.run(t, x)
            assert g["status"] == 0
            for k in ("keys", "counts", "aggs"):
                assert g[k] == exp[k], k
        return
    got = check(ctx, t, q)
    assert len(got["keys"]) > 0
    assert all(k[0] in set(int(v) for v in t["columns"]["d"]["dict"]) for k in got["keys"][:20])


def test_dictionary_plan_rules(ctx):
    from paper_2506_10092_amd import ccq
    t = datagen.config_c2(seed=12, n_rows=100_003, columns=("r0", "d"))
    t["columns"]["d"]["dict"] = np.arange(10_000, dtype=np.int64) * 3
    tb = ccq.Table(ctx, t["n_rows"], ccq.to_device(t["columns"]))
    base = {"preds": [], "aggs": [("count",)], "window": (0, t["n_rows"])}
    for bad, status in ((dict(base, keys=[("d", 1, 5000)]), -1), (dict(base, keys=[("d", 0, 10_001)]), -1),
                        (dict(base, keys=[], aggs=[("sum", "d")]), -2)):
        with pytest.raises(ccq.CcqError) as e:
            ccq.Plan(tb, bad)
        assert e.value.status == status


def _generic_table(n, seed=21):
    """Columns that send queries down the generic row path: RLE int32 r
    (predicates, keys), RLE int64 m with values far beyond int32, a 32-bit
    packed column q spanning the whole int32 range (SUM terms that wrap a
    32-bit accumulator often), Zipf dictionary codes d (14 bits, 12000
    codes) and a 20-bit packed column p."""
    cols = {
        "r": datagen.rle_column(seed, 5010, n, "lognormal", 64, 0, 1 << 16),
        "m": datagen.rle_column(seed, 5020, n, "lognormal", 200, -(1 << 40), 1 << 40, np.int64),
        "q": datagen.packed_column(seed, 5030, n, 32, "uniform", 1 << 32, base=-(1 << 31)),
        "d": datagen.packed_column(seed, 5040, n, 14, "zipf", 12000, s=1.1),
        "p": datagen.packed_column(seed, 5050, n, 20, "uniform", 1 << 20, base=-(1 << 19)),
    }
    return {"name": "generic_%d" % n, "n_rows": n, "columns": cols}


GENERIC_CASES = {
    # SUM terms that wrap int32 cells (q) and terms wider than int32 (m)
    "wrap_and_wide": {"preds": [("r", "range", 1000, 60000)], "keys": [("d", 0, 12000)],
                      "aggs": [("sum", "q"), ("sum", "m"), ("count",)]},
    # four SUMs over 12000 groups: only part of the table fits in LDS
    "partial_table": {"preds": [("p", "range", -300000, 400000)], "keys": [("d", 0, 12000)],
                      "aggs": [("sum", "q"), ("sum", "m"), ("sum", "p"), ("sum", "r"), ("count",)]},
    # a range on the key column itself: no code table, slot = key - lowest key
    "range_key_no_table": {"preds": [("d", "range", 3, 9000), ("r", "range", 0, 50000)],
                           "keys": [("d", 0, 12000)], "aggs": [("sum", "p"), ("count",)]},
    # an RLE key with 8192 groups next to a packed SUM: register runs, global table
    "rle_key_global": {"preds": [("p", "range", -400000, 300000)], "keys": [("r", 3, 8192)],
                       "aggs": [("sum", "q"), ("sum", "m"), ("count",)]},
    # two keys: RLE then dictionary
    "two_keys": {"preds": [("q", "range", -(1 << 30), 1 << 30)], "keys": [("r", 12, 16), ("d", 0, 12000)],
                 "aggs": [("sum", "p"), ("count",)]},
}


@pytest.mark.parametrize("case", sorted(GENERIC_CASES))
def test_generic_row_path_tables(ctx, case):
    t = _generic_table(3_000_017)
    q = dict(GENERIC_CASES[case], window=(12_345, 3_000_017 - 999))
    say("generic case:", case)
    got = check(ctx, t, q)
    assert len(got["keys"]) > 1



@pytest.mark.parametrize("seed", range(30))
def test_tiny_random_tables_with_min_max_expressions(ctx, seed):
    """MIN, MAX and SUM / MIN / MAX of a + b, a - b, a * b over RLE and
    bit-packed columns (the generic row path), equal to the oracle."""
    from tests.cases import tiny_query_with_exprs
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(1, 5000))
    t, wd = tiny_table(rng, n)
    for _ in range(3):
        q = tiny_query_with_exprs(rng, n, wd)
        say("expr seed", seed, "n", n, "query", q)
        check(ctx, t, q)


@pytest.mark.parametrize("q", [
    # over the mixed-encoding table: RLE x RLE, RLE x packed, packed x packed; dictionary / RLE / no keys
    {"preds": [("r0", "range", 0, 40000)], "keys": [("d", 0, 10000)],
     "aggs": [("min", "r1"), ("max", ("r1", "-", "p")), ("sum", ("r0", "*", "r1")), ("count",), ("sum", "s")]},
    {"preds": [("p", "range", -200000, 300000)], "keys": [("r2", 10, 64)],
     "aggs": [("sum", ("p", "+", "r0")), ("min", ("p", "*", "r1")), ("max", "p")]},
    {"preds": [], "keys": [], "aggs": [("min", "r0"), ("max", "r0"), ("sum", ("r0", "+", "r1")), ("count",)]},
    {"preds": [("d", "in", [0, 1, 2, 3, 4])], "keys": [("d", 0, 10000)],
     "aggs": [("min", "p"), ("max", "p"), ("sum", ("p", "*", "p"))]},
])
def test_min_max_expressions_2m_rows(ctx, q):
    t = datagen.config_c2(seed=33, n_rows=2_000_003, columns=datagen.C2_COLS)
    q = dict(q, window=(777, 2_000_003 - 55))
    say("expr 2M:", q["aggs"])
    got = check(ctx, t, q)
    assert len(got["keys"]) >= 1


def test_min_max_expressions_in_a_batch(ctx):
    from paper_2506_10092_amd import ccq
    n = 1_000_003
    t = datagen.config_c2(seed=34, n_rows=n, columns=datagen.C2_COLS)
    qs = [{"preds": [("r1", "range", 1000, 50000)], "keys": [("d", 0, 10000)],
           "aggs": [("max", ("r0", "+", "p")), ("count",)], "window": (0, n)},
          {"preds": [], "keys": [], "aggs": [("min", "p"), ("sum", ("r2", "*", "r2"))], "window": (100, n // 2)},
          {"preds": [("r0", "range", 0, 30000)], "keys": [("d", 0, 10000)], "aggs": [("sum", "s"), ("count",)],
           "window": (0, n)}]
    tb = ccq.Table(ctx, n, ccq.to_device(t["columns"]))
    b = ccq.Batch(ctx, [ccq.Plan(tb, q) for q in qs], tiles_per_item=16)
    b.execute(b.new_workspace())
    for q, g in zip(qs, b.to_python()):
        exp = oracle.run(t, q)
        assert g["status"] == 0
        for k in ("keys", "counts", "aggs"):
            assert g[k] == exp[k], k
