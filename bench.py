#!/usr/bin/env python3
"""Benchmark: one filter / group-by / aggregate query over lightweight-encoded
columns, resident in HBM, per step.

Default workload (mixed encodings, 1e9 logical rows): RLE int32 columns r0,
r1 (lognormal runs, means 64 / 200, values uniform in [0, 2^16)), an
index-encoded int64 column s (1% of rows), dictionary codes d (Zipf s=1.1
over 10k entries) packed to 14 bits;
    SELECT d, SUM(s), COUNT(*) WHERE r0 IN [0,32768) AND r1 IN [16384,65536)
    AND d IN (50 codes) GROUP BY d.
A step is one ccq_execute (clear, fused kernel, finalize) on one stream.

Prints one JSON line: logical rows/s; the fused kernel's achieved
compressed-bytes bandwidth against the 8 TB/s HBM peak (bytes = the encoded
bytes of the referenced columns inside the window); the CPU oracle timed on
the host's cores on a bounded sample, whose answer must equal the GPU's.
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
                  for f in ("ccq_kernels.hip", "ccq_plan.h", "ccq_api.cpp")]


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
           {a[1] for a in query["aggs"] if a[0] == "sum"}
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


def traffic_from_profile(workload_name):
    """HBM bytes per fused-kernel launch from the committed rocprofv3 counter
    summary, or None when it is missing or was taken on other kernel code."""
    path = os.path.join(ROOT, "profiles", "k_fused_%s_traffic.json" % workload_name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sha") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


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
    per query), over one resident table."""
    import torch
    import datagen
    from paper_2506_10092_amd import ccq

    n_rows = args.rows or 100_000_000
    t_gen = time.time()
    t = datagen.config_c2(seed=4, n_rows=n_rows, columns=("r0", "r1", "r2", "s", "d", "p"))
    qs = datagen.c4_queries(4, n_rows, n_queries=args.queries)
    log("generated table + %d queries in %.1fs" % (len(qs), time.time() - t_gen))
    ctx = ccq.Context(0)
    table = ccq.Table(ctx, n_rows, ccq.to_device(t["columns"]))
    plans = [ccq.Plan(table, q) for q in qs]
    log("plans created")
    rows = sum(q["window"][1] - q["window"][0] for q in qs)
    alg = sum(algorithmic_bytes(t, q) for q in qs)
    stream = torch.cuda.Stream()

    # single-launch path: one ccq_execute per query, each with its own buffers
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
    best, tuned_ms = batch.autotune(ws, candidates=(8, 32, 128, 512), reps=3, stream=stream)
    log("autotuned tiles_per_item=%d (%.3f ms)" % (best, tuned_ms))
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            batch.execute(ws, stream)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(args.steps):
            batch.execute(ws, stream)
        e1.record(stream)
    stream.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    if batch.to_python() != single:
        raise SystemExit("batched results differ from the single-launch path")
    log("batch %.3f ms per batch of %d queries; results equal the single-launch path" % (ms, len(qs)))
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
        "config": {"workload": "c4_batch_%d_over_%g" % (len(qs), n_rows), "rows": rows,
                   "compressed_bytes": alg, "tiles_per_item": best, "graph": True},
        "roofline": {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole batch (clear + persistent launches + finalize)", "kernel_ms": ms},
        "single_launch": {"ms": single_ms, "rows_per_s": rows / (single_ms * 1e-3),
                          "speedup_of_batch": single_ms / ms},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--queries", type=int, default=4096, help="c4: queries per batch")
    ap.add_argument("--rows", type=int, default=0, help="override the logical row count")
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
              "group tables; see the design notes). Run with --gpus 1.", file=sys.stderr)
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

    t_gen = time.time()
    wl = make_workload(args.config, args.rows)
    query = wl["query"]
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
    traffic = traffic_from_profile(wl["name"])

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
                   "compressed_bytes": alg, "query": "single-launch path, one query per ccq_execute"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "ccq::k_fused", "kernel_ms": fused_avg},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
