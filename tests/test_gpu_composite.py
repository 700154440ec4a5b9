"""GPU parity of composite columns (Section 3.2: RLE + Index, Plain + Index)
against the CPU oracle, through the C-ABI.  The oracle reads the paper's
form (pure runs with starts and ends beside the points); the library reads
the run-ends form that tests.cases.abi_column derives from it.  Results must
match bit for bit, on the single-query kernel and in batches mixed with
plans without composites."""
import json
import os
import sys

import numpy as np
import pytest

import datagen
from oracle import oracle
from tests.cases import abi_column, composite_columns, composite_table, tiny_query_with_composites

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "composite.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_10092_amd import ccq
    assert torch.cuda.is_available()
    return ccq.Context(0)


def device_table(ctx, table):
    from paper_2506_10092_amd import ccq
    n = table["n_rows"]
    cols = {k: abi_column(v, n) for k, v in table["columns"].items()}
    return ccq.Table(ctx, n, ccq.to_device(cols))


def check(ctx, table, query, t=None):
    from paper_2506_10092_amd import ccq
    exp = oracle.run(table, query)
    t = t or device_table(ctx, table)
    p = ccq.Plan(t, query)
    got = p.run()
    assert got["status"] == 0, got["status"]
    assert got["keys"] == exp["keys"], ("keys differ", query)
    assert got["counts"] == exp["counts"], ("counts differ", query)
    assert got["aggs"] == exp["aggs"], ("aggregates differ", query)
    return got


def test_paper_examples(ctx):
    g = json.load(open(GOLDEN))
    pi, ri = g["plain_index"], g["rle_index"]
    n = pi["n_rows"]
    codes = np.array(pi["plain"] + [200] * (n - len(pi["plain"])), dtype=np.uint32)   # never read
    y = {"enc": "plain+index", "packed": datagen.pack_codes(codes, 8), "w": 8, "base": 0,
         "positions": np.array(pi["outlier_positions"], dtype=np.int32),
         "point_values": np.array(pi["outlier_values"], dtype=np.int64)}
    table = {"n_rows": n, "columns": {"y": y}}
    for q in ({"preds": [], "keys": [], "aggs": [("count",), ("sum", "y"), ("min", "y"), ("max", "y")]},
              {"preds": [("y", "range", 2, 1 << 40)], "keys": [], "aggs": [("count",), ("sum", "y")]},
              {"preds": [("y", "range", 0, 100)], "keys": [], "aggs": [("sum", "y")]}):
        got = check(ctx, table, dict(q, window=(0, n)))
    assert got["aggs"] == [(6,)]
    n = ri["n_rows"]
    x = {"enc": "rle+index", "values": np.array(ri["rle_values"], dtype=np.int64),
         "run_starts": np.array(ri["rle_starts"], dtype=np.int64),
         "run_ends": np.array(ri["rle_ends_inclusive"], dtype=np.int64) + 1,
         "positions": np.array(ri["index_positions"], dtype=np.int32),
         "point_values": np.array(ri["index_values"], dtype=np.int64)}
    table = {"n_rows": n, "columns": {"x": x}}
    got = check(ctx, table, {"preds": [], "keys": [], "aggs": [("count",), ("sum", "x"), ("max", "x")],
                             "window": (0, n)})
    assert got["aggs"] == [(7, sum(ri["expect_rows"]), 4)]
    got = check(ctx, table, {"preds": [("x", "in", [1, 3])], "keys": [], "aggs": [("count",)], "window": (0, n)})
    assert got["counts"] == [5]


@pytest.mark.parametrize("seed", range(24))
def test_tiny_composite_tables(ctx, seed):
    rng = np.random.default_rng([seed, 51])
    n = int(rng.integers(1, 300))
    table, wd = composite_table(rng, n)
    t = device_table(ctx, table)
    for _ in range(4):
        check(ctx, table, tiny_query_with_composites(rng, n, wd), t)


@pytest.mark.parametrize("n", [4097, 20011, 70001])
def test_composite_tables_over_several_tiles(ctx, n):
    """Several 2048-row tiles and a ragged tail; windows that start and end
    inside tiles."""
    rng = np.random.default_rng([n, 52])
    table, wd = composite_table(rng, n)
    t = device_table(ctx, table)
    for i in range(10):
        q = tiny_query_with_composites(rng, n, wd)
        say("composite", n, i, q)
        check(ctx, table, q, t)


def test_composite_batch_with_other_plans(ctx):
    """A batch mixing composite plans (their own kernel instance) with
    generic, run-mode and fast-path plans; every answer equal to the
    oracle's, repeated launches equal."""
    from paper_2506_10092_amd import ccq
    rng = np.random.default_rng(53)
    n = 60_000
    table, wd = composite_table(rng, n)
    t = device_table(ctx, table)
    qs = [tiny_query_with_composites(rng, n, wd) for _ in range(12)]
    qs += [{"preds": [("r0", "range", 0, 10), ("r2", "range", 0, 20)], "keys": [("r2", 0, 20)],
            "aggs": [("count",), ("sum", "r1")],
            "window": (0, n)},
           {"preds": [("d", "in", [1, 2, 3])], "keys": [("d", 0, 1 << wd)], "aggs": [("count",)], "window": (0, n)},
           {"preds": [("r1", "range", 0, 12)], "keys": [], "aggs": [("sum", "p"), ("sum", "s")], "window": (5, n - 7)}]
    plans = [ccq.Plan(t, q) for q in qs]
    b = ccq.Batch(ctx, plans, tiles_per_item=2)
    ws = b.new_workspace()
    b.execute(ws)
    got = b.to_python()
    b.execute(ws)
    assert b.to_python() == got
    for q, r in zip(qs, got):
        exp = oracle.run(table, q)
        assert r["status"] == 0 and (r["keys"], r["counts"], r["aggs"]) == (exp["keys"], exp["counts"], exp["aggs"]), q


def test_composite_two_million_rows(ctx):
    """2M rows: an RLE + Index column of mostly pure runs and a Plain + Index
    column with about 1% outliers, beside the mixed table's other columns."""
    rng = np.random.default_rng(54)
    n = 2_000_000
    x, y, _, _ = composite_columns(rng, n, p_single=0.1)
    cols = {"x": x, "y": y,
            "r0": datagen.rle_column(54, 1, n, "lognormal", 64, 0, 20),
            "s": datagen.sparse_column(54, 3, n, 0.01, -100, 100),
            "d": datagen.packed_column(54, 5, n, 6, "uniform", 64)}
    big = {"n_rows": n, "columns": cols}
    t = device_table(ctx, big)
    queries = [
        {"preds": [("x", "range", 0, 10)], "keys": [], "aggs": [("count",), ("sum", "x"), ("sum", "y")]},
        {"preds": [("y", "not_range", -20, 20), ("r0", "range", 0, 12)], "keys": [("d", 0, 64)],
         "aggs": [("count",), ("min", "y"), ("max", "x"), ("sum", "s")]},
        {"preds": [("x", "in", [1, 2, 3, 17])], "keys": [("r0", 0, 20)],
         "aggs": [("sum", ("x", "*", "y")), ("count",)]},
        {"preds": [("d", "in", [5, 9])], "keys": [], "aggs": [("sum", ("y", "-", "x")), ("max", "y")]},
    ]
    for i, q in enumerate(queries):
        say("composite 2M", i)
        for win in ((0, n), (12_345, n - 777)):
            check(ctx, big, dict(q, window=win), t)
