#!/usr/bin/env python3
"""Benchmark: filter / group-by / aggregate queries over lightweight-encoded
columns resident in HBM.

Default workload (the batched form against the plain path): one table of
1e8 logical rows with the mixed-encoding columns -- RLE int32 r0, r1, r2
(lognormal runs, means 64 / 200 / 1000, values uniform in [0, 2^16)), an
index-encoded int64 column s (1% of rows), dictionary codes d (Zipf s=1.1
over 10k entries, 14 bits) and a 20-bit plain column p -- and 4096 seeded
query templates (windows log-uniform in [1e4, 1e8] rows; 1-3 predicates,
1-2 aggregates, GROUP BY none, d or an RLE value >> shift).  A step is one
execution of the whole batch (work-item size autotuned, replayed as a
hipGraph); the same 4096 queries as 4096 single launches are timed beside
it.  Every answer is checked against the CPU oracle, which is timed on the
host's cores as the CPU baseline.

--config c2 | c3 | c1: one query per step (single-launch path), the
1e9-row mixed-encoding GROUP BY d query, the 1e10-row four-key RLE GROUP
BY, or the 1e6-row two-column query.  --config c5: the serving loop.
--config encode: the device Plain -> RLE encoder on a 1e9-row column.
--config join: a 1e8-row RLE fact column joined with a 65,536-row dimension
key, and a dimension attribute applied over the join.

Prints one JSON line: logical rows/s; the persistent kernels' achieved
compressed-bytes bandwidth against the 8 TB/s HBM peak (bytes = the encoded
bytes each query references inside its window); the CPU oracle's rate.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "logical rows/s + HBM GB/s (% of peak); batched p50/p99 latency vs plain path"
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_10092_amd", "csrc", f)
                  for f in ("ccq_device.h", "ccq_inst.hip", "ccq_kernels.hip", "ccq_plan.h", "ccq_api.cpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(table, query):
    """Encoded bytes the query references inside its window: each RLE run that
    overlaps it (value + 8-byte run end), each Index point inside it
    (position + value) and the packed bits of its rows."""
    import numpy as np
    n0, n1 = query["window"]
    used = {p[0] for p in query["preds"]} | {k[0] for k in query["keys"]} | \
           {a[1] for a in query["aggs"] if a[0] == "sum"} | {p[0] for cl in query.get("or", ()) for p in cl}
    total = 0
    for name in sorted(used):
        c = table["columns"][name]
        if c["enc"] == "rle":
            e = c["run_ends"]
            if n1 > n0:
                lo = int(np.searchsorted(e, n0, side="right"))
                hi = int(np.searchsorted(e, n1 - 1, side="right"))
                total += (hi - lo + 1) * (8 + c["values"].itemsize)
        elif c["enc"] == "index":
            p = c["positions"]
            cnt = int(np.searchsorted(p, n1) - np.searchsorted(p, n0))
            total += cnt * (p.itemsize + c["values"].itemsize)
        else:
            total += int(math.ceil((n1 - n0) * c["w"] / 8.0))
    return total


def make_workload(name, rows):
    import datagen
    if name == "c1":
        return datagen.config_c1(n_rows=rows or 1_000_000)
    if name == "c2":
        return datagen.config_c2(n_rows=rows or 1_000_000_000)
    if name == "c3":
        return datagen.config_c3(n_rows=rows or 10_000_000_000)
    if name == "c4":
        return datagen.config_c4(n_rows=rows or 100_000_000)
    raise SystemExit("unknown --config %s" % name)


def traffic_from_profile(kernel, workload_name):
    """HBM bytes per launch of `kernel` on a workload from the committed
    rocprofv3 counter summary, or None when it is missing or was taken on
    other kernel code."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload_name))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sha") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_threads():
    """Host threads the CPU oracle may use: this process's CPU share (at
    most 16, a one-GPU machine's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def oracle_check(table, queries, answers, what):
    """Every answer against the CPU oracle (exits on the first mismatch);
    returns (rows, seconds, threads) of the oracle work."""
    from oracle import oracle
    threads = cpu_threads()
    rows, t0 = 0, time.time()
    for i, (q, got) in enumerate(zip(queries, answers)):
        exp = oracle.run(table, q, n_threads=threads)
        if got["status"] != 0 or any(got[k] != exp[k] for k in ("keys", "counts", "aggs")):
            raise SystemExit("%s: query %d differs from the CPU oracle (status %d): %r" % (what, i, got["status"], q))
        rows += q["window"][1] - q["window"][0]
    return rows, time.time() - t0, threads


def copy_reference(args):
    """A plain device-to-device copy of known size, timed like a step."""
    import torch
    n = args.copy_bytes // 4
    x = torch.ones(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record()
    for _ in range(args.steps):
        y.copy_(x)
    e.record()
    torch.cuda.synchronize()
    ms = b.elapsed_time(e) / args.steps
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "ms": ms,
                      "GBps_read_plus_write": 2 * n * 4 / (ms * 1e-3) / 1e9}), flush=True)


def bench_batch(args):
    """Many queries in one batched launch sequence (autotuned work items,
    replayed as a hipGraph) against the single-launch path (one ccq_execute
    per query), over one resident table; every answer is checked against
    the CPU oracle."""
    import torch
    import datagen
    from paper_2506_10092_amd import ccq

    n_rows = args.rows or 100_000_000
    t_gen = time.time()
    t = datagen.config_c2(seed=4, n_rows=n_rows, columns=datagen.C2_COLS)
    qs = datagen.c4_queries(4, n_rows, n_queries=args.queries)
    log("generated table + %d queries in %.1fs" % (len(qs), time.time() - t_gen))
    ctx = ccq.Context(0)
    table = ccq.Table(ctx, n_rows, ccq.to_device(t["columns"]))
    plans = [ccq.Plan(table, q) for q in qs]
    log("plans created")
    rows = sum(q["window"][1] - q["window"][0] for q in qs)
    alg = sum(algorithmic_bytes(t, q) for q in qs)
    stream = torch.cuda.Stream()

    # single-launch path: one ccq_execute per query, each with its own
    # buffers; one untimed pass, then one timed pass
    wss = [p.new_workspace() for p in plans]
    res = [p.new_result() for p in plans]
    with torch.cuda.stream(stream):
        for p, w, r in zip(plans, wss, res):
            p.execute(w, r, stream)
    stream.synchronize()
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        b0.record(stream)
        for p, w, r in zip(plans, wss, res):
            p.execute(w, r, stream)
        b1.record(stream)
    stream.synchronize()
    single_ms = b0.elapsed_time(b1)
    single = [r.to_python() for r in res]
    log("single-launch path %.3f ms" % single_ms)

    batch = ccq.Batch(ctx, plans, use_graph=True)
    ws = batch.new_workspace()
    if args.tune_cache:
        log("tuning cache %s: %d entries loaded" % (args.tune_cache, ctx.tune_cache_load(args.tune_cache)))
    best, tuned_ms = batch.autotune(ws, candidates=(8, 32, 128, 512), reps=3, stream=stream)
    log("autotuned tiles_per_item=%d (%.3f ms)" % (best, tuned_ms))
    if args.tune_cache:
        ctx.tune_cache_save(args.tune_cache)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            batch.execute(ws, stream)
    stream.synchronize()
    # the step: whole-batch graph replays
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(args.steps):
            batch.execute(ws, stream)
        e1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    got = batch.to_python()
    if got != single:
        raise SystemExit("batched results differ from the single-launch path")
    # the persistent launches alone (the dominant kernels), timed with events
    # recorded on the launch stream around them
    K = args.steps
    fb = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    fe = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in fb + fe:
        e.record(stream)
    stream.synchronize()
    with torch.cuda.stream(stream):
        for i in range(K):
            batch.execute(ws, stream, fused_events=(fb[i], fe[i]))
    stream.synchronize()
    kernel_ms = sum(fb[i].elapsed_time(fe[i]) for i in range(K)) / K
    if batch.to_python() != single:
        raise SystemExit("batched results (direct launches) differ from the single-launch path")
    log("batch %.3f ms per batch of %d queries (persistent launches %.3f ms); equal to the single-launch path"
        % (ms, len(qs), kernel_ms))

    cpu = None
    if not args.no_cpu_baseline:
        o_rows, o_s, threads = oracle_check(t, qs, got, "c4 batch")
        cpu = {"value": o_rows / o_s, "unit": "rows/s", "cores": threads, "kind": "oracle",
               "sample": "all %d queries of the batch (%d logical rows), %.1f s wall; every batched answer "
                         "equal to the oracle's bit for bit" % (len(qs), o_rows, o_s)}
        log("cpu oracle: %d queries in %.1f s, all equal" % (len(qs), o_s))

    achieved = alg / (kernel_ms * 1e-3) / 1e9
    wl_name = "c4_batch_%d_over_%g" % (len(qs), n_rows)
    traffic = traffic_from_profile("k_batch", wl_name)
    out = {
        "metric": METRIC,
        "value": rows / (ms * 1e-3),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wl_name, "queries": len(qs), "table_rows": n_rows, "rows": rows,
                   "compressed_bytes": alg, "tiles_per_item": best, "graph": True,
                   "step": "one batched execution of all queries (hipGraph replay)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_frac": (traffic / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "kernel": "ccq::k_batch (the batch's persistent launches, timed together)",
                     "kernel_ms": kernel_ms},
        "single_launch": {"ms": single_ms, "rows_per_s": rows / (single_ms * 1e-3),
                          "GBps": alg / (single_ms * 1e-3) / 1e9, "speedup_of_batch": single_ms / ms},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _light_table(t):
    """What algorithmic_bytes needs of a table (run ends, positions, widths,
    value types), without the value arrays and packed words."""
    import numpy as np
    cols = {}
    for name, c in t["columns"].items():
        if c["enc"] == "rle":
            cols[name] = {"enc": "rle", "run_ends": c["run_ends"], "values": np.empty(0, c["values"].dtype)}
        elif c["enc"] == "index":
            cols[name] = {"enc": "index", "positions": c["positions"], "values": np.empty(0, c["values"].dtype)}
        else:
            cols[name] = {"enc": c["enc"], "w": c["w"]}
    return {"n_rows": t["n_rows"], "columns": cols}


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def bench_serve(args):
    """Serving: queries of the batched templates arrive as a Poisson process
    over eight resident tables of the mixed-encoding columns (n_i = scale *
    1e7 * 10^(3i/7) rows, i = 0..7); a server with continuous batching and a
    server that launches every query on its own (the single-launch path)
    answer them under one HBM budget.  Per arrival rate: throughput and
    p50 / p99 latency from arrival to completion, after a warm-up."""
    import numpy as np
    import torch
    import datagen
    from paper_2506_10092_amd import ccq

    sizes = [max(1_000_000, int(round(args.serve_scale * 1e7 * 10 ** (3 * i / 7)))) for i in range(8)]
    cols = ("r0", "r1", "r2", "s", "d", "p")
    ctx = ccq.Context(0)
    tables, light, host = [], [], []
    t_gen = time.time()
    for i, n in enumerate(sizes):
        t = datagen.config_c2(seed=50 + i, n_rows=n, columns=cols)
        tables.append(ccq.Table(ctx, n, ccq.to_device(t["columns"])))
        light.append(_light_table(t))
        host.append(t if not args.no_cpu_baseline else None)   # kept for the oracle check
        del t
        log("table %d: %d rows resident (%.1fs)" % (i, n, time.time() - t_gen))
    torch.cuda.synchronize()

    n_q = args.serve_queries
    rng = np.random.default_rng([5, 5555])
    which = rng.integers(0, 8, size=n_q)
    per = [datagen.c4_queries(500 + i, sizes[i], n_queries=int((which == i).sum())) for i in range(8)]
    nxt = [0] * 8
    queries = []
    for i in which:
        queries.append((int(i), per[i][nxt[i]]))
        nxt[i] += 1
    plans = [ccq.Plan(tables[i], q) for i, q in queries]
    results = [p.new_result() for p in plans]
    rows_q = np.array([q["window"][1] - q["window"][0] for _, q in queries], dtype=np.float64)
    bytes_q = np.array([algorithmic_bytes(light[i], q) for i, q in queries], dtype=np.float64)
    log("%d plans over %d tables (%.1fs)" % (n_q, len(tables), time.time() - t_gen))

    free, _ = torch.cuda.mem_get_info()
    budget = int(min(args.serve_budget_gb * 1e9, free - 4e9))
    # arrival rates; "max" submits every query at once (the saturation throughput)
    levels = [float("inf") if x.strip() == "max" else float(x) for x in args.qps.split(",")]
    warm = min(args.serve_warmup, n_q // 2)
    report = {}
    answers = {}
    for batching in (True, False):
        mode = "batched" if batching else "single_launch"
        report[mode] = {}
        for qps in levels:
            srv = ccq.Server(ctx, budget, max_inflight=args.serve_inflight, n_streams=2, batching=batching,
                             tiles_per_item=args.serve_tpi)
            if math.isinf(qps):
                arr = np.zeros(n_q)
            else:
                arr = np.cumsum(np.random.default_rng([6, int(qps)]).exponential(1.0 / qps, size=n_q))
            base = ccq.now() + 0.005
            sched = {}
            for k in range(n_q):
                due = base + arr[k]
                while ccq.now() < due:
                    pass
                sched[srv.submit(plans[k], results[k])] = (k, due)
            srv.drain(900.0)
            comps = []
            while True:
                got = srv.poll(4096)
                if not got:
                    break
                comps.extend(got)
            srv.close()
            if len(comps) != n_q or any(c["status"] != 0 for c in comps):
                raise SystemExit("server %s at %g QPS: %d completions, statuses %s" %
                                 (mode, qps, len(comps), sorted({c["status"] for c in comps})))
            stat = [(sched[c["ticket"]][0], c["t_done"] - sched[c["ticket"]][1], c["t_done"]) for c in comps]
            stat = [x for x in stat if x[0] >= warm]
            lat = [x[1] for x in stat]
            idx = [x[0] for x in stat]
            t_first = base + arr[warm]
            dur = max(x[2] for x in stat) - t_first
            report[mode]["%g" % qps] = {
                "queries": len(stat), "p50_ms": _pct(lat, 50) * 1e3, "p99_ms": _pct(lat, 99) * 1e3,
                "queries_per_s": len(stat) / dur, "rows_per_s": float(rows_q[idx].sum()) / dur,
                "GBps": float(bytes_q[idx].sum()) / dur / 1e9}
            log("%s %g QPS: p50 %.3f ms p99 %.3f ms, %.0f queries/s" %
                (mode, qps, report[mode]["%g" % qps]["p50_ms"], report[mode]["%g" % qps]["p99_ms"],
                 report[mode]["%g" % qps]["queries_per_s"]))
            if qps == levels[0]:
                answers[mode] = [r.to_python() for r in results]
    if answers["batched"] != answers["single_launch"]:
        raise SystemExit("served results differ between the batched and the single-launch server")
    cpu = None
    if not args.no_cpu_baseline:
        # a seeded sample of the served answers against the CPU oracle
        pick = sorted(np.random.default_rng([7, 7777]).choice(n_q, size=min(args.serve_check, n_q), replace=False))
        o_rows, o_s, threads = 0, 0.0, 1
        for k in pick:
            i, q = queries[k]
            r, s_, threads = oracle_check(host[i], [q], [answers["batched"][k]], "c5 served query %d" % k)
            o_rows += r
            o_s += s_
        cpu = {"value": o_rows / o_s, "unit": "rows/s", "cores": threads, "kind": "oracle",
               "sample": "%d served queries drawn at random (seeded) from the %d of the first arrival rate, "
                         "%d logical rows, %.1f s wall; every sampled answer equal to the oracle's bit for bit"
                         % (len(pick), n_q, o_rows, o_s)}
        log("cpu oracle: %d sampled served answers equal (%.1f s)" % (len(pick), o_s))
    top = "%g" % levels[-1]
    b = report["batched"][top]
    out = {
        "metric": METRIC,
        "value": b["rows_per_s"],
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": n_q,
        "warmup": warm,
        "ms_per_step": 1e3 / b["queries_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "c5_serve_8_tables_%g_rows" % sum(sizes), "tables": sizes, "queries": n_q,
                   "qps": levels, "hbm_budget_bytes": budget, "max_inflight": args.serve_inflight,
                   "tiles_per_item": args.serve_tpi},
        "serving": report,
        "p50_ms": b["p50_ms"],
        "p99_ms": b["p99_ms"],
        "single_launch_p50_ms": report["single_launch"][top]["p50_ms"],
        "single_launch_p99_ms": report["single_launch"][top]["p99_ms"],
        "roofline": {"bound": "hbm", "achieved": b["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b["GBps"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole served load at the top arrival rate (encoded bytes of the completed "
                               "queries / wall time)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_encode(args):
    """The device encoder: Plain -> RLE of an int32 column (the mixed-encoding
    table's r0, decoded: lognormal runs of mean 64) of --rows rows (default
    1e9).  A step is one ccq_plain_to_rle (count, scan, write); the output is
    checked against the CPU oracle's runs."""
    import numpy as np
    import torch
    import datagen
    from oracle import encode as E
    from paper_2506_10092_amd import ccq

    n = args.rows or 1_000_000_000
    src = datagen.rle_column(2, 2010, n, "lognormal", 64, 0, 1 << 16)
    x = E.decode_rle(src["values"], src["run_ends"])
    import ctypes
    ctx = ccq.Context(0)
    d = torch.from_numpy(x).cuda()
    stream = torch.cuda.current_stream()
    # the run count once (outside the timed region), then one ccq_plain_to_rle
    # call per step into outputs of exactly that size
    runs = ccq.plain_to_rle(ctx, d, stream)["values"].numel()
    L = ccq.lib()
    ws = ccq._enc_ws(d)
    rv = torch.empty(runs, dtype=d.dtype, device=d.device)
    re_ = torch.empty(runs, dtype=torch.int64, device=d.device)
    nr = ctypes.c_int64()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())

    def step():
        ccq._check(L.ccq_plain_to_rle(ctx.h, vp(d), ccq._dtype_code(d), n, vp(ws), ws.numel(),
                                      ccq._stream_ptr(stream), vp(rv), vp(re_), runs, ctypes.byref(nr)))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.time() - t0) * 1e3 / args.steps
    out = {"values": rv, "run_ends": re_}
    # the oracle's maximal runs (the generator's runs need not be maximal:
    # neighbouring runs may draw the same value)
    t1 = time.time()
    ev, ee = E.plain_to_rle(x)
    cpu_s = time.time() - t1
    if not (np.array_equal(out["run_ends"].cpu().numpy(), ee) and np.array_equal(out["values"].cpu().numpy(), ev)):
        raise SystemExit("encoded runs differ from the oracle's")
    alg = 4 * n + 12 * runs       # the column read once, the runs written once
    cpu = None
    if not args.no_cpu_baseline:
        cpu = {"value": n / cpu_s, "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": "numpy plain_to_rle over the whole column (%d rows), %.1f s, one thread; its runs "
                         "equal the GPU's" % (n, cpu_s)}
    achieved = alg / (ms * 1e-3) / 1e9
    out = {"metric": METRIC, "value": n / (ms * 1e-3), "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "encode_plain_to_rle_%g" % n, "rows": n, "runs": runs,
                      "step": "one ccq_plain_to_rle call into outputs of the known run count (count, scan, host read "
                              "of the run count, write)"},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "k_enc_count + k_enc_scan + k_enc_write (wall time of the call)"},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def bench_join(args):
    """Joins (Get / Apply Join Index): a fact column joined with a dimension
    key.  Left: the mixed-encoding table's RLE int32 column r0 (lognormal runs
    of mean 64, values uniform in [0, 2^16)) over --rows rows (default 1e8).
    Right: a 65,536-row dimension table, its key a seeded permutation of
    [0, 2^16) bit-packed to 16 bits, and an attribute uniform in [0, 2^20)
    bit-packed to 20 bits.  A step is one ccq_join_index (one block per left
    run) and one ccq_join_apply of the attribute over the blocks (one value
    per left row).  Blocks and values are checked in full against the
    dimension arrays, and a window of the left column against the CPU
    oracle."""
    import ctypes
    import numpy as np
    import torch
    import datagen
    from oracle import join as J
    from paper_2506_10092_amd import ccq

    n = args.rows or 100_000_000
    nd = 1 << 16
    left = datagen.rle_column(2, 2010, n, "lognormal", 64, 0, 1 << 16)
    rng = np.random.default_rng([2, 7001])
    key = rng.permutation(nd).astype(np.uint32)
    attr = rng.integers(0, 1 << 20, size=nd).astype(np.uint32)
    right = {"k": {"enc": "bitpacked", "packed": datagen.pack_codes(key, 16), "w": 16, "base": 0},
             "a": {"enc": "bitpacked", "packed": datagen.pack_codes(attr, 20), "w": 20, "base": 0}}
    ctx = ccq.Context(0)
    tl = ccq.Table(ctx, n, ccq.to_device({"r0": left}))
    tr = ccq.Table(ctx, nd, ccq.to_device(right))
    L = ccq.lib()
    runs = len(left["values"])
    wsb = L.ccq_join_workspace_bytes(tl.h, 0, 0, n, tr.h, 0, 0, nd)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    blocks = torch.empty((runs, 4), dtype=torch.int64, device="cuda")
    ws2b = L.ccq_join_apply_workspace_bytes(runs, n)
    ws2 = torch.empty(ws2b, dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    nb, npairs, nout = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    stream = ccq._stream_ptr(None)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())

    def step():
        ccq._check(L.ccq_join_index(tl.h, 0, 0, n, tr.h, 0, 0, nd, vp(ws), wsb, stream, vp(blocks), runs,
                                    ctypes.byref(nb), ctypes.byref(npairs)))
        ccq._check(L.ccq_join_apply(tr.h, 1, vp(blocks), nb.value, 1, vp(ws2), ws2b, stream, vp(out), n,
                                    ctypes.byref(nout)))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.time() - t0) * 1e3 / args.steps
    # index calls alone, for the split
    t1 = time.time()
    for _ in range(args.steps):
        ccq._check(L.ccq_join_index(tl.h, 0, 0, n, tr.h, 0, 0, nd, vp(ws), wsb, stream, vp(blocks), runs,
                                    ctypes.byref(nb), ctypes.byref(npairs)))
    torch.cuda.synchronize()
    ms_index = (time.time() - t1) * 1e3 / args.steps
    # full check: one block per left run, in left order (one right entry per value)
    inv = np.empty(nd, dtype=np.int64)
    inv[key.astype(np.int64)] = np.arange(nd)
    ends = left["run_ends"]
    starts = np.r_[0, ends[:-1]]
    lv = left["values"].astype(np.int64)
    want = np.stack([starts, ends - starts, inv[lv], np.ones(runs, dtype=np.int64)], axis=1)
    if nb.value != runs or npairs.value != n or not np.array_equal(blocks.cpu().numpy(), want):
        raise SystemExit("join blocks differ from the dimension arrays")
    if nout.value != n or not np.array_equal(out.cpu().numpy(), np.repeat(attr.astype(np.int64)[inv[lv]],
                                                                        ends - starts)):
        raise SystemExit("applied values differ from the dimension arrays")
    # oracle on a window of the left column (bounded sample)
    w = min(n, 10_000_000)
    t2 = time.time()
    ob = J.join_blocks(J.entries(left, n, 0, w), J.entries(right["k"], nd, 0, nd))
    ov = J.apply(ob, right["a"], nd, "right")
    cpu_s = time.time() - t2
    gb, gp = ccq.join_index(tl, 0, tr, 0, (0, w))
    if sorted(map(tuple, gb.cpu().numpy().tolist())) != sorted(ob) or gp != len(ov):
        raise SystemExit("join blocks differ from the CPU oracle")
    if not np.array_equal(ccq.join_apply(tr, 1, torch.tensor(ob, dtype=torch.int64, device="cuda"), "right")
                          .cpu().numpy(), ov):
        raise SystemExit("applied values differ from the CPU oracle")
    # algorithmic bytes: the left runs and both right columns read, the
    # blocks written once and read once, the applied values written
    alg = runs * 12 + nd * 2 + nd * 20 // 8 + runs * 32 * 2 + n * 8
    achieved = alg / (ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        cpu = {"value": w / cpu_s, "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": "oracle join_blocks + apply over the first %d left rows (%d runs), %.1f s, one thread; "
                         "equal to the GPU's" % (w, len(ob), cpu_s)}
    line = {"metric": METRIC, "value": n / (ms * 1e-3), "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": "join_rle_fact_%g_x_dim_%d" % (n, nd), "rows": n, "left_runs": runs,
                       "blocks": nb.value, "pairs": npairs.value, "ms_join_index": ms_index,
                       "step": "one ccq_join_index (bounds, build, count, scan, write) and one ccq_join_apply "
                               "(pair counts, scan, gather) with their host reads of the sizes"},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "every kernel of both calls (wall time of the calls)"},
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def describe_query(wl, query, flt):
    """A short text of a single-launch workload's filter and grouping."""
    if wl["name"].startswith("c2"):
        return {"and": "r0 range AND r1 range AND d IN", "not": "NOT r0 range AND r1 range AND d IN",
                "or": "(r0 range OR r1 range) AND d IN", "or_dict": "r1 range AND (r0 range OR d IN)"}[flt]
    if wl["name"].startswith("c3"):
        return "no filter; GROUP BY k0, k1, k2, k3 -> SUM(m), COUNT(*)"
    return "a < 500 -> SUM(b), COUNT(*)"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c4", choices=["c1", "c2", "c3", "c4", "c5", "encode", "join"])
    ap.add_argument("--queries", type=int, default=4096, help="c4: queries per batch")
    ap.add_argument("--serve-queries", type=int, default=10000, help="c5: queries per arrival rate (after warm-up)")
    ap.add_argument("--serve-warmup", type=int, default=500, help="c5: leading queries left out of the statistics")
    ap.add_argument("--serve-scale", type=float, default=1.0, help="c5: scale of the eight table sizes")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0, help="c5: HBM budget of the servers")
    ap.add_argument("--serve-inflight", type=int, default=512, help="c5: queries admitted or running at once")
    ap.add_argument("--serve-tpi", type=int, default=64, help="c5: batch work-item size in tiles")
    ap.add_argument("--qps", default="200,1000,5000,max",
                    help="c5: Poisson arrival rates; max submits every query at once (saturation)")
    ap.add_argument("--serve-check", type=int, default=1000, help="c5: served answers checked against the oracle")
    ap.add_argument("--rows", type=int, default=0, help="override the logical row count")
    ap.add_argument("--tune-cache", default="",
                    help="c4: a tuning-cache file, loaded before the autotune and saved after it")
    ap.add_argument("--filter", default="and", choices=["and", "not", "or", "or_dict"],
                    help="c2: the workload's filter (and), or the same table under a filter with NOT "
                         "(r0 outside a middle range), an OR of the two RLE ranges (or), or an OR of the "
                         "r0 range and the dictionary IN-list (or_dict)")
    ap.add_argument("--cpu-sample-rows", type=int, default=1_000_000_000,
                    help="rows of the window the CPU oracle runs over (bounded sample)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum wall time of the CPU oracle timing")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the query, time a plain device copy of this many bytes (the "
                         "reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the query would shard by row range with one exchange of partial "
              "group tables). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2506_10092_amd import ccq

    if args.copy_bytes:
        copy_reference(args)
        return

    if args.config == "c4":
        bench_batch(args)
        return
    if args.config == "c5":
        bench_serve(args)
        return
    if args.config == "encode":
        bench_encode(args)
        return
    if args.config == "join":
        bench_join(args)
        return

    t_gen = time.time()
    wl = make_workload(args.config, args.rows)
    query = wl["query"]
    if args.filter != "and":
        if args.config != "c2":
            raise SystemExit("--filter applies to --config c2")
        r0, r1, din = query["preds"]
        if args.filter == "not":
            query = dict(query, preds=[("r0", "not_range", 16384, 49152), r1, din])
        elif args.filter == "or":
            query = dict(query, preds=[din], **{"or": [[r0, r1]]})
        else:
            query = dict(query, preds=[r1], **{"or": [[r0, din]]})
    n0, n1 = query["window"]
    log("generated %s in %.1fs" % (wl["name"], time.time() - t_gen))

    dev = ccq.to_device(wl["columns"])
    torch.cuda.synchronize()
    log("columns resident on the GPU")
    ctx = ccq.Context(0)
    table = ccq.Table(ctx, wl["n_rows"], dev)
    plan = ccq.Plan(table, query)
    ws, res = plan.new_workspace(), plan.new_result()
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.execute(ws, res, stream)
    torch.cuda.synchronize()
    log("warmup done")

    K = args.steps
    fb = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    fe = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in fb + fe:
        e.record(stream)
    t_begin, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_begin.record(stream)
    for i in range(K):
        plan.execute(ws, res, stream, fused_events=(fb[i], fe[i]))
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_begin.elapsed_time(t_end)
    ms_step = ms_total / K
    fused_ms = [fb[i].elapsed_time(fe[i]) for i in range(K)]
    fused_avg = sum(fused_ms) / K
    gpu_result = res.to_python()
    if gpu_result["status"] != 0:
        raise SystemExit("device status %d" % gpu_result["status"])
    log("timed %d steps: %.4f ms/step, fused kernel %.4f ms" % (K, ms_step, fused_avg))

    rows = n1 - n0
    alg = algorithmic_bytes(wl, query)
    achieved = alg / (fused_avg * 1e-3) / 1e9
    traffic = traffic_from_profile("k_fused", wl["name"]) if args.filter == "and" else None

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle
        s1 = min(n1, n0 + args.cpu_sample_rows)
        sample_q = dict(query, window=(n0, s1))
        threads = os.cpu_count() or 1
        log("cpu oracle on rows [%d, %d) with %d threads" % (n0, s1, threads))
        # repeat the sample until about 10 s of CPU wall time have been spent
        t0 = time.time()
        exp = oracle.run(wl, sample_q, n_threads=threads)
        passes = 1
        while time.time() - t0 < args.cpu_seconds and passes < 1000:
            oracle.run(wl, sample_q, n_threads=threads)
            passes += 1
        dt = time.time() - t0
        if (n0, s1) == (n0, n1):
            check = gpu_result
        else:
            p2 = ccq.Plan(table, sample_q)
            check = p2.run()
        for k in ("keys", "counts", "aggs"):
            if check[k] != exp[k]:
                raise SystemExit("GPU result differs from the CPU oracle (%s)" % k)
        cpu = {"value": (s1 - n0) * passes / dt, "unit": "rows/s", "cores": threads, "kind": "oracle",
               "sample": "the same query over rows [%d, %d) of the same table, %d passes (%.1f s wall); "
                         "GPU answer equal bit for bit" % (n0, s1, passes, dt)}
        log("cpu oracle %d passes %.2f s, results equal" % (passes, dt))

    out = {
        "metric": METRIC,
        "value": rows / (ms_step * 1e-3),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "rows": rows, "groups": len(gpu_result["keys"]),
                   "compressed_bytes": alg, "query": "single-launch path, one query per ccq_execute",
                   "filter": describe_query(wl, query, args.filter)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_frac": (traffic / (fused_avg * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "kernel": "ccq::k_fused", "kernel_ms": fused_avg},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
