"""Serving loop (ccq_server_*): every query answered through the server --
batched or one launch per query, submitted from one thread or several, with
the HBM budget forcing admission to wait -- must give exactly the CPU
oracle's answer (and so what its own ccq_execute gives, alone); a query whose
workspace exceeds the budget completes with CCQ_E_BUDGET and does not
disturb the others."""
import sys
import threading

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
    n = 2_000_003
    t = datagen.config_c2(seed=55, n_rows=n, columns=("r0", "r1", "r2", "s", "d", "p"))
    qs = datagen.c4_queries(55, n, n_queries=120, lo_rows=1_000, hi_rows=n)
    ctx = ccq.Context(0)
    table = ccq.Table(ctx, n, ccq.to_device(t["columns"]))
    plans = [ccq.Plan(table, q) for q in qs]
    single = [p.run() for p in plans]
    torch.cuda.synchronize()
    # the expected answers come from the CPU oracle; each query alone
    # (ccq_execute) must give them too
    expect = []
    for q in qs:
        e = oracle.run(t, q)
        expect.append({"keys": e["keys"], "counts": e["counts"], "aggs": e["aggs"], "status": 0})
    assert single == expect, "a query alone differs from the CPU oracle"
    return {"ctx": ctx, "table": table, "plans": plans, "single": single, "expect": expect}


def _serve(setup, server, plans, threads=1):
    results = [p.new_result() for p in plans]
    tickets = [None] * len(plans)

    def submit(idx):
        for i in idx:
            tickets[i] = server.submit(plans[i], results[i])

    if threads == 1:
        submit(range(len(plans)))
    else:
        ths = [threading.Thread(target=submit, args=(range(k, len(plans), threads),)) for k in range(threads)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
    server.drain(120.0)
    done = {c["ticket"]: c for c in server.poll(4096)}
    assert sorted(done) == sorted(tickets)
    for c in done.values():
        assert c["t_submit"] <= c["t_start"] <= c["t_done"]
    return [done[t] for t in tickets], [r.to_python() for r in results]


@pytest.mark.parametrize("batching", [True, False])
def test_server_matches_single_launch(setup, batching):
    from paper_2506_10092_amd import ccq
    s = ccq.Server(setup["ctx"], 256 << 20, max_inflight=48, n_streams=2, batching=batching, tiles_per_item=32)
    comps, got = _serve(setup, s, setup["plans"])
    s.close()
    assert all(c["status"] == 0 for c in comps)
    assert got == setup["expect"], "a served answer differs from the CPU oracle"
    say("server batching=%s: %d served answers equal the oracle's" % (batching, len(got)))


def test_server_tight_budget_and_threads(setup):
    """An 8 MiB arena holds only a few group tables at once: admission waits
    for frees; four submitting threads."""
    from paper_2506_10092_amd import ccq
    s = ccq.Server(setup["ctx"], (16 << 20) + (8 << 20), max_inflight=6, n_streams=1, batching=True)
    comps, got = _serve(setup, s, setup["plans"], threads=4)
    s.close()
    assert all(c["status"] == 0 for c in comps)
    assert got == setup["expect"]


def test_server_budget_rejection(setup):
    from paper_2506_10092_amd import ccq
    table = setup["table"]
    # 2^20 groups x (count + one sum) x 8 bytes = 16 MiB of group table > the 8 MiB arena
    big = ccq.Plan(table, {"preds": [], "keys": [("r0", 0, 1 << 16), ("r1", 12, 16)],
                           "aggs": [("count",), ("sum", "s")], "window": (0, table.n_rows)})
    assert big.workspace_bytes > (8 << 20)
    s = ccq.Server(setup["ctx"], (16 << 20) + (8 << 20), max_inflight=8, n_streams=1, batching=True)
    plans = [setup["plans"][0], big, setup["plans"][1]]
    comps, got = _serve(setup, s, plans)
    s.close()
    assert [c["status"] for c in comps] == [0, ccq.E_BUDGET, 0]
    assert got[0] == setup["expect"][0] and got[2] == setup["expect"][1]


def test_server_rejects_bad_config(setup):
    from paper_2506_10092_amd import ccq
    with pytest.raises(ccq.CcqError):
        ccq.Server(setup["ctx"], 1024, max_inflight=4)
    with pytest.raises(ccq.CcqError):
        ccq.Server(setup["ctx"], 256 << 20, max_inflight=0)


@pytest.mark.parametrize("graphs", [True, False])
def test_server_graph_replays_across_rounds(setup, graphs):
    """Batches of at most 8 queries, so launch shapes repeat and each captured
    graph is replayed many times; three rounds with unrelated GPU work and
    synchronisations between them; every answer of every round equals the
    oracle's."""
    import torch
    from paper_2506_10092_amd import ccq
    s = ccq.Server(setup["ctx"], 256 << 20, max_inflight=16, max_batch=8, n_streams=2, batching=True,
                   tiles_per_item=64, graphs=graphs)
    for rnd in range(3):
        comps, got = _serve(setup, s, setup["plans"])
        assert all(c["status"] == 0 for c in comps)
        assert got == setup["expect"], "round %d differs from the oracle (graphs=%s)" % (rnd, graphs)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        torch.cuda.synchronize()
        say("graph replay round", rnd, "graphs", graphs, "ok")
    s.close()
