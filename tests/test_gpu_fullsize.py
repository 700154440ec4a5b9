"""Full-size parity: the bench workload (mixed encodings, 1e9 rows) and the
multi-RLE group-by (1e10 rows) against the CPU oracle over the whole window,
in the launch configuration bench.py times (one ccq_execute per query)."""
import os
import sys
import time

import pytest

import datagen
from oracle import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(table, query):
    from paper_2506_10092_amd import ccq
    ctx = ccq.Context(0)
    t = ccq.Table(ctx, table["n_rows"], ccq.to_device(table["columns"]))
    p = ccq.Plan(t, query)
    ws, res = p.new_workspace(), p.new_result()
    p.execute(ws, res)
    p.execute(ws, res)          # a second run on the same workspace must give the same answer
    return res.to_python()


def _compare(got, exp):
    assert got["status"] == 0
    assert got["keys"] == exp["keys"]
    assert got["counts"] == exp["counts"]
    assert got["aggs"] == exp["aggs"]


@pytest.mark.timeout(600)
def test_c2_full_1e9():
    t0 = time.time()
    c = datagen.config_c2()
    say("c2 1e9 generated in %.1fs" % (time.time() - t0))
    got = _gpu(c, c["query"])
    say("gpu done")
    exp = oracle.run(c, c["query"], n_threads=os.cpu_count())
    say("oracle done in %.1fs" % (time.time() - t0))
    _compare(got, exp)
    assert len(got["keys"]) == 50


@pytest.mark.timeout(600)
def test_c2_full_1e9_not_or_and_index_filters():
    """The same table under NOT, OR and Index-column filters (the filters
    bench.py --filter times, plus an Index predicate), over all 1e9 rows."""
    c = datagen.config_c2()
    r0, r1, din = c["query"]["preds"]
    base = dict(c["query"])
    queries = [
        dict(base, preds=[("r0", "not_range", 16384, 49152), r1, din]),
        dict(base, preds=[din], **{"or": [[r0, r1]]}),
        dict(base, preds=[r0, ("s", "range", 1, 500_000)], keys=[("r1", 12, 16)]),
    ]
    from paper_2506_10092_amd import ccq
    ctx = ccq.Context(0)
    t = ccq.Table(ctx, c["n_rows"], ccq.to_device(c["columns"]))
    for q in queries:
        say("query", q["preds"], q.get("or"))
        got = ccq.Plan(t, q).run()
        exp = oracle.run(c, q, n_threads=os.cpu_count())
        _compare(got, exp)


@pytest.mark.timeout(900)
def test_c3_full_1e10():
    t0 = time.time()
    c = datagen.config_c3()
    say("c3 1e10 generated in %.1fs" % (time.time() - t0))
    got = _gpu(c, c["query"])
    say("gpu done, %d groups" % len(got["keys"]))
    # properties that hold at any size, checked before the long oracle run
    m = c["columns"]["m"]
    import numpy as np
    lens = np.diff(np.r_[0, m["run_ends"]])
    assert sum(got["counts"]) == c["n_rows"]
    assert sum(a[0] for a in got["aggs"]) == int(np.sum(m["values"] * lens))
    exp = oracle.run(c, c["query"], n_threads=os.cpu_count())
    say("oracle done in %.1fs" % (time.time() - t0))
    _compare(got, exp)
