"""Batched execution: every query of a batch must give exactly what the
oracle and its own single-launch execution give, whatever the work-item size,
and a captured hipGraph must give the same answers on every replay."""
import sys

import numpy as np
import pytest

import datagen
from oracle import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2506_10092_amd import ccq
    n = 3_000_017
    t = datagen.config_c2(seed=44, n_rows=n, columns=("r0", "r1", "r2", "s", "d", "p"))
    qs = datagen.c4_queries(44, n, n_queries=160, lo_rows=1_000, hi_rows=n)
    # edge cases: empty window, one row, whole table, a window ending mid-word
    qs += [dict(qs[0], window=(5, 5)), dict(qs[1], window=(77, 78)), dict(qs[2], window=(0, n)),
           dict(qs[3], window=(31, n - 3))]
    # OR clauses over RLE columns (one column in two clauses)
    qs += [dict(qs[4], **{"or": [[("r0", "range", 0, 20000), ("r1", "range", 50000, 65536)]]}),
           dict(qs[5], **{"or": [[("r2", "not_range", 0, 100), ("r0", "in", [1, 2, 3])],
                                 [("r0", "range", 0, 30000), ("r1", "range", 0, 10000)]]}),
           # an OR clause over RLE and bit-packed columns; a predicate on the Index column
           dict(qs[6], **{"or": [[("r1", "range", 0, 20000), ("d", "in", [1, 2, 3, 4, 5])]]}),
           dict(qs[7], preds=qs[7]["preds"] + [("s", "not_range", 1, 500_000)]),
           # OR clauses over RLE columns and the Index column, in run mode and row mode
           {"preds": [("r2", "range", 0, 40000)], "keys": [], "aggs": [("count",), ("sum", "s"), ("sum", "r0")],
            "or": [[("r0", "range", 0, 5000), ("s", "range", 1, 200_000)]], "window": (1000, n - 5)},
           {"preds": [("d", "in", list(range(0, 10000, 7)))], "keys": [("d", 0, 10000)],
            "aggs": [("count",), ("sum", "s")],
            "or": [[("r1", "range", 0, 10000), ("r0", "in", [1, 2]), ("s", "not_in", [0])]], "window": (0, n)}]
    ctx = ccq.Context(0)
    table = ccq.Table(ctx, n, ccq.to_device(t["columns"]))
    plans = [ccq.Plan(table, q) for q in qs]
    torch.cuda.synchronize()
    return {"t": t, "qs": qs, "ctx": ctx, "table": table, "plans": plans}


def _single(plans):
    return [p.run() for p in plans]


def test_batch_equals_oracle_and_single_launch(setup):
    from paper_2506_10092_amd import ccq
    t, qs, plans = setup["t"], setup["qs"], setup["plans"]
    single = _single(plans)
    for tpi in (1, 7, 64, 100000):
        b = ccq.Batch(setup["ctx"], plans, tiles_per_item=tpi)
        ws = b.new_workspace()
        b.execute(ws)
        got = b.to_python()
        say("batch tiles_per_item", tpi, "items", b.n_items)
        assert got == single, "batch differs from single-launch results (tiles_per_item %d)" % tpi
    for i, q in enumerate(qs):
        exp = oracle.run(t, q)
        s = single[i]
        assert s["status"] == 0
        assert (s["keys"], s["counts"], s["aggs"]) == (exp["keys"], exp["counts"], exp["aggs"]), (i, q)


def test_batch_graph_replays(setup):
    import torch
    from paper_2506_10092_amd import ccq
    plans = setup["plans"]
    eager = _single(plans)
    stream = torch.cuda.Stream()
    b = ccq.Batch(setup["ctx"], plans, tiles_per_item=16, use_graph=True)
    ws = b.new_workspace()
    for rep in range(4):
        with torch.cuda.stream(stream):
            b.execute(ws, stream)
        stream.synchronize()
        got = b.to_python()
        assert got == eager, "graph replay %d differs" % rep
        # the program's own eager work between replays
        x = torch.arange(1 << 20, device="cuda").sum().item()
        assert x == (1 << 20) * ((1 << 20) - 1) // 2
        plans[rep].run()


def test_batch_autotune_keeps_results(setup):
    import torch
    from paper_2506_10092_amd import ccq
    plans = setup["plans"]
    eager = _single(plans)
    stream = torch.cuda.Stream()
    b = ccq.Batch(setup["ctx"], plans)
    ws = b.new_workspace()
    best, ms = b.autotune(ws, candidates=(2, 16, 128), reps=2, stream=stream)
    say("autotune best", best, "ms", ms)
    assert best in (2, 16, 128) and ms > 0
    b.execute(ws, stream)
    stream.synchronize()
    assert b.to_python() == eager


def test_autotune_tuning_cache(setup, tmp_path):
    """A second autotune of a batch of the same shape takes the context's
    cached result without timing (the same size and the same time); a fresh
    context that loads the saved cache does the same; a different candidate
    list is a different key and is timed."""
    import torch
    from paper_2506_10092_amd import ccq
    plans = setup["plans"]
    stream = torch.cuda.Stream()
    b = ccq.Batch(setup["ctx"], plans)
    ws = b.new_workspace()
    cand = (4, 32, 256)
    best, ms = b.autotune(ws, candidates=cand, reps=2, stream=stream)
    say("tuned", best, ms)
    b2 = ccq.Batch(setup["ctx"], plans)
    assert b2.autotune(b2.new_workspace(), candidates=cand, reps=2, stream=stream) == (best, ms)
    path = str(tmp_path / "tune.txt")
    assert setup["ctx"].tune_cache_save(path) >= 1
    ctx2 = ccq.Context(0)
    assert ctx2.tune_cache_load(path) >= 1
    t2 = ccq.Table(ctx2, setup["table"].n_rows, setup["table"].columns)
    plans2 = [ccq.Plan(t2, q) for q in setup["qs"]]
    b3 = ccq.Batch(ctx2, plans2)
    ws3 = b3.new_workspace()
    best3, ms3 = b3.autotune(ws3, candidates=cand, reps=2, stream=stream)
    assert best3 == best and abs(ms3 - ms) <= 1e-5 * max(ms, 1.0)     # the file keeps 6 significant digits
    # the cached size is the one that runs, and the answers are unchanged
    b3.execute(ws3, stream)
    stream.synchronize()
    assert b3.to_python() == _single(plans)
    other = b3.autotune(ws3, candidates=(8, 64), reps=1, stream=stream)
    assert other[0] in (8, 64)
