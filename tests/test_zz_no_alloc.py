"""ccq_execute_noalloc (the library's fixed device scratch as the
workspace) against ccq_execute (a caller workspace): identical results on
two calls in a row, the second with a smaller input, so the second call
runs over what the first left in the scratch."""
import sys

import pytest

import datagen
from oracle import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_10092_amd import ccq
    assert torch.cuda.is_available()
    return ccq.Context(0)


def both(plan):
    """(ccq_execute, ccq_execute_noalloc) results of one plan."""
    ws, r1, r2 = plan.new_workspace(), plan.new_result(), plan.new_result()
    plan.execute(ws, r1)
    plan.execute_noalloc(r2)
    return r1.to_python(), r2.to_python()


def test_noalloc_matches_execute_on_two_calls(ctx):
    from paper_2506_10092_amd import ccq
    # call 1: 2e6-row four-key RLE GROUP BY (up to 1e6 groups, a 16 MB group
    # table in the scratch); call 2: a 1e5-row window of the mixed-encoding
    # table, 50 groups, over the scratch call 1 left behind
    c3 = datagen.config_c3(n_rows=2_000_003)
    c2 = datagen.config_c2(n_rows=1_000_003)
    t3 = ccq.Table(ctx, c3["n_rows"], ccq.to_device(c3["columns"]))
    t2 = ccq.Table(ctx, c2["n_rows"], ccq.to_device(c2["columns"]))
    q2 = dict(c2["query"], window=(123_457, 223_457))
    for name, table, tb, q in (("c3 2e6", c3, t3, c3["query"]), ("c2 window 1e5", c2, t2, q2)):
        say("noalloc case:", name)
        p = ccq.Plan(tb, q)
        assert p.workspace_bytes <= ccq.NOALLOC_WORKSPACE_BYTES
        a, b = both(p)
        assert a["status"] == 0 and b["status"] == 0
        assert b == a, name
        exp = oracle.run(table, q)
        for k in ("keys", "counts", "aggs"):
            assert b[k] == exp[k], (name, k)


def test_noalloc_rejects_oversized_workspace(ctx):
    from paper_2506_10092_amd import ccq
    c3 = datagen.config_c3(n_rows=100_003)
    t3 = ccq.Table(ctx, c3["n_rows"], ccq.to_device(c3["columns"]))
    # 4096 * 4096 declared groups: a 256 MB group table
    q = dict(c3["query"], keys=[("k0", 0, 4096), ("k1", 0, 4096)])
    p = ccq.Plan(t3, q)
    assert p.workspace_bytes > ccq.NOALLOC_WORKSPACE_BYTES
    with pytest.raises(ccq.CcqError) as e:
        p.execute_noalloc(p.new_result())
    assert e.value.status == -3
