"""C-ABI checks that need no GPU: the library loads, exports every function
include/ccq.h declares, and its host-side validation rejects malformed
tables and queries with the documented status codes (host-only context)."""
import os
import re
import subprocess

import numpy as np
import pytest
import torch

from paper_2506_10092_amd import ccq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccq.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccq_[a-z_]+)\s*\(", text)))


def test_header_functions_are_exported():
    names = header_functions()
    assert len(names) >= 12
    out = subprocess.check_output(["nm", "-D", "--defined-only", ccq.LIB_PATH]).decode()
    exported = set(re.findall(r"\bT (ccq_[a-z_]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert sorted(ccq.SIGNATURES) == names          # the binding covers the whole header
    L = ccq.lib()
    for n in names:
        assert getattr(L, n) is not None


def test_abi_version():
    assert ccq.lib().ccq_abi_version() == 8


def _host_table(columns, n_rows):
    ctx = ccq.Context(ccq.HOST_ONLY)
    return ccq.Table(ctx, n_rows, columns)


def _cols(n=1000):
    t = lambda a, dt: torch.tensor(a, dtype=dt)
    return {
        "a": {"enc": "rle", "values": t([1, 2, 3], torch.int32), "run_ends": t([10, 500, n], torch.int64)},
        "m": {"enc": "rle", "values": t([5], torch.int64), "run_ends": t([n], torch.int64)},
        "s": {"enc": "index", "positions": t([3, 7], torch.int32), "values": t([1, 2], torch.int64)},
        "d": {"enc": "bitpacked", "packed": torch.zeros((n * 14 + 31) // 32 + 2, dtype=torch.int32), "w": 14,
              "base": 0},
        "p": {"enc": "bitpacked", "packed": torch.zeros((n * 20 + 31) // 32 + 2, dtype=torch.int32), "w": 20,
              "base": -(1 << 19)},
    }


def test_host_only_context_checks_plans():
    tb = _host_table(_cols(), 1000)
    q = {"preds": [("a", "range", 0, 3), ("d", "in", [1, 5, 9])], "keys": [("d", 0, 10000)],
         "aggs": [("sum", "s"), ("count",)], "window": (0, 1000)}
    g, ws = ccq.plan_check(tb, q)
    assert g == 3                       # dense slots over the IN-list
    assert ws >= 256 + 8 * 2 * 3
    q2 = dict(q, keys=[("a", 0, 4), ("p", 10, 1024)], preds=[])
    g, ws = ccq.plan_check(tb, q2)
    assert g == 4 * 1024
    with pytest.raises(ccq.CcqError) as e:
        ccq.Plan(tb, q)
    assert e.value.status == ccq.E_UNSUPPORTED


@pytest.mark.parametrize("bad,code", [
    ({"preds": [("zz", "range", 0, 1)]}, "unknown"),
    ({"keys": [("s", 0, 4)]}, ccq.E_UNSUPPORTED),
    ({"keys": [("a", 63, 4)]}, ccq.E_INVALID),
    ({"keys": [("a", 0, 0)]}, ccq.E_INVALID),
    ({"keys": [("m", 0, 1 << 20), ("a", 0, 1 << 10)]}, ccq.E_UNSUPPORTED),
    ({"keys": [("a", 0, 4)] * 9}, ccq.E_UNSUPPORTED),
    ({"aggs": [("count",)] * 9}, ccq.E_UNSUPPORTED),
    ({"window": (0, 1001)}, ccq.E_INVALID),
    ({"window": (10, 5)}, ccq.E_INVALID),
    ({"keys": [("a", 0, 4), ("a", 1, 4)]}, ccq.E_UNSUPPORTED),
    # two OR clauses spanning RLE and bit-packed columns; an OR over an Index
    # and a bit-packed column; two OR clauses over RLE and Index columns; one
    # of those beside an RLE x bit-packed clause
    ({"or": [[("a", "range", 0, 2), ("d", "in", [1])], [("m", "range", 0, 2), ("p", "range", 0, 5)]]},
     ccq.E_UNSUPPORTED),
    ({"or": [[("s", "range", 0, 2), ("a", "in", [1]), ("d", "in", [1])]]}, ccq.E_UNSUPPORTED),
    ({"or": [[("s", "range", 0, 2), ("d", "in", [1])]]}, ccq.E_UNSUPPORTED),
    ({"or": [[("s", "range", 0, 2), ("a", "in", [1])], [("s", "range", 5, 9), ("m", "in", [5])]]},
     ccq.E_UNSUPPORTED),
    ({"or": [[("s", "range", 0, 2), ("a", "in", [1])], [("a", "range", 0, 2), ("d", "in", [1])]]},
     ccq.E_UNSUPPORTED),
    # five two-column OR clauses need ten RLE column uses (at most eight)
    ({"or": [[("a", "range", 0, 2 + i), ("m", "range", 0, 5)] for i in range(5)]}, ccq.E_UNSUPPORTED),
    ({"or": [[]]}, ccq.E_INVALID),
    # MIN / MAX / expressions take RLE and bit-packed columns
    ({"aggs": [("min", "s")]}, ccq.E_UNSUPPORTED),
    ({"aggs": [("sum", ("a", "+", "s"))]}, ccq.E_UNSUPPORTED),
])
def test_plan_check_rejects(bad, code):
    tb = _host_table(_cols(), 1000)
    q = {"preds": [], "keys": [], "aggs": [("count",)], "window": (0, 1000)}
    q.update(bad)
    with pytest.raises(ccq.CcqError) as e:
        ccq.plan_check(tb, q)
    if code != "unknown":
        assert e.value.status == code, str(e.value)
    assert str(e.value)


def test_or_clauses_fold_or_take_rle_slots():
    """An OR clause over one column folds into that column (any encoding);
    clauses that always hold drop; clauses over RLE columns are accepted up
    to eight RLE column uses, and one clause may add a bit-packed column or
    an Index column to its RLE columns."""
    tb = _host_table(_cols(), 1000)
    base = {"preds": [], "keys": [("d", 0, 1 << 14)], "aggs": [("count",)], "window": (0, 1000)}
    ok = [
        [[("d", "in", [1, 2]), ("d", "range", 100, 200)]],
        [[("p", "range", 0, 5), ("p", "not_range", -9, 9)]],
        [[("a", "range", 0, 2), ("m", "in", [5])]] * 3 + [[("m", "range", 0, 9), ("m", "in", [7])]],
        [[("a", "not_in", []), ("d", "in", [3])]],        # holds for every row: dropped
        [[("a", "in", []), ("d", "in", [3])]],            # one live predicate: folds into d
        [[("a", "range", 0, 2), ("d", "in", [3])]],       # RLE OR bit-packed: the row clause
        [[("d", "in", [3]), ("p", "range", 0, 9)], [("a", "range", 0, 2), ("m", "in", [5])]],
        [[("s", "range", 1, 2), ("a", "in", [1])]],       # RLE OR Index: the row clause
        [[("a", "range", 0, 2), ("m", "in", [5]), ("s", "not_in", [0])], [("a", "in", [2]), ("m", "in", [5])]],
    ]
    for clauses in ok:
        ccq.plan_check(tb, dict(base, preds=[("a", "range", 1, 3)], **{"or": clauses}))


@pytest.mark.parametrize("mutate,msg", [
    (lambda c: c["a"].update(values=c["a"]["values"].to(torch.int16)), "int32 or int64"),
    (lambda c: c["d"].update(w=0), "bit_width"),
    (lambda c: c["d"].update(w=33), "bit_width"),
    (lambda c: c.update(x={"enc": "zzz"}), "encoding"),
])
def test_table_create_rejects(mutate, msg):
    cols = _cols()
    mutate(cols)
    with pytest.raises(ccq.CcqError, match=msg):
        _host_table(cols, 1000)


def test_table_create_rejects_int32_positions_past_2_31():
    cols = {"s": {"enc": "index", "positions": torch.tensor([3], dtype=torch.int32),
                  "values": torch.tensor([1], dtype=torch.int64)}}
    with pytest.raises(ccq.CcqError, match="int32 positions"):
        _host_table(cols, 3 * (1 << 31))
    cols["s"]["positions"] = torch.tensor([3], dtype=torch.int64)
    _host_table(cols, 3 * (1 << 31))


def test_last_error_is_thread_local_and_cleared():
    L = ccq.lib()
    h = ccq.ctypes.c_void_p()
    assert L.ccq_context_create(-7, ccq.ctypes.byref(h)) != 0
    assert L.ccq_last_error()
    assert L.ccq_context_create(ccq.HOST_ONLY, ccq.ctypes.byref(h)) == 0
    assert L.ccq_last_error() == b""
    L.ccq_context_destroy(h)


def test_word_owner_division_is_exact():
    """The kernel finds which lane reads packed word q as (q * ceil(2^20/w)) >> 20;
    check it equals q // w for every width and every word a tile can stage."""
    for w in range(1, 33):
        magic = ((1 << 20) + w - 1) // w
        q = np.arange(0, 64 * w + 2, dtype=np.int64)
        assert np.array_equal((q * magic) >> 20, q // w), w


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(ccq, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ccq, "_lib", None)
    with pytest.raises(ccq.CcqError, match="not built"):
        ccq.lib()


def test_work_item_size_is_capped():
    """A work item is counted by one workgroup in uint32 LDS counters, so the
    batch and the server reject items of 2^19 tiles (2^30 rows) or more
    before anything else (the check needs no device)."""
    L = ccq.lib()
    ctx = ccq.Context(ccq.HOST_ONLY)
    h = ccq.ctypes.c_void_p()
    opts = ccq.BatchOpts(1 << 20, 0)
    assert L.ccq_batch_create(ctx.h, None, 0, None, ccq.ctypes.byref(opts), ccq.ctypes.byref(h)) == ccq.E_INVALID
    assert b"tiles_per_item" in L.ccq_last_error()
    opts = ccq.BatchOpts(1 << 19, 0)      # the largest item size passes this check
    assert L.ccq_batch_create(ctx.h, None, 0, None, ccq.ctypes.byref(opts), ccq.ctypes.byref(h)) == ccq.E_INVALID
    assert b"device context" in L.ccq_last_error()
    cfg = ccq.ServerConfig(1 << 30, 8, 0, 1, 1, (1 << 19) + 1, 0)
    assert L.ccq_server_create(ctx.h, ccq.ctypes.byref(cfg), ccq.ctypes.byref(h)) == ccq.E_INVALID
    assert b"tiles_per_item" in L.ccq_last_error()


def test_avg_var_matches_the_oracle_bit_for_bit():
    """ccq_avg_var (host code of the library) against the oracle's
    post-processing: identical doubles on random exact aggregates."""
    from oracle import oracle
    rng = np.random.default_rng(11)
    n = rng.integers(0, 1 << 40, size=500)
    n[:5] = 0
    s = rng.integers(-(1 << 60), 1 << 60, size=500)
    ss = rng.integers(0, 1 << 62, size=500)
    avg, var = ccq.avg_var(n, s, ss)
    for i in range(500):
        a, v = oracle.avg_var(int(n[i]), int(s[i]), int(ss[i]))
        assert avg[i] == a and var[i] == v, i


def test_expression_plans_check_on_host():
    tb = _host_table(_cols(), 1000)
    q = {"preds": [("d", "in", [1, 2])], "keys": [("d", 0, 10000)],
         "aggs": [("min", "a"), ("max", ("a", "*", "p")), ("sum", "s"), ("count",)], "window": (0, 1000)}
    g, ws = ccq.plan_check(tb, q)
    assert g == 2 and ws >= 256 + 8 * 5 * 2
    with pytest.raises(ccq.CcqError) as e:
        ccq.plan_check(tb, dict(q, aggs=[("sum", ("a", "%", "p"))]))
    assert e.value.status == ccq.E_INVALID


def _composite_cols(n=1000):
    t = lambda a, dt: torch.tensor(a, dtype=dt)
    cols = _cols(n)
    cols["x"] = {"enc": "rle+index", "values": t([4, 9], torch.int64), "run_ends": t([600, n], torch.int64),
                 "positions": t([7, 650], torch.int32), "point_values": t([-1, 3], torch.int64)}
    cols["y"] = {"enc": "plain+index", "packed": torch.zeros((n * 6 + 31) // 32 + 2, dtype=torch.int32), "w": 6,
                 "base": -3, "positions": t([0, 999], torch.int32), "point_values": t([1 << 40, -(1 << 40)], torch.int64)}
    return cols


def test_composite_plans_check_on_host():
    """Composite columns (Section 3.2) in predicates, SUM, MIN, MAX and
    expressions; not as keys, not in an OR across columns, at most two."""
    tb = _host_table(_composite_cols(), 1000)
    q = {"preds": [("x", "range", 0, 5), ("y", "not_range", 0, 9), ("d", "in", [1, 2])], "keys": [("d", 0, 1 << 14)],
         "aggs": [("sum", "x"), ("min", "y"), ("max", ("x", "+", "y")), ("sum", "s"), ("count",)], "window": (0, 1000)}
    g, _ = ccq.plan_check(tb, q)
    assert g == 2
    ccq.plan_check(tb, dict(q, preds=[], **{"or": [[("x", "range", 0, 2), ("x", "in", [9])]]}))   # one column
    for bad in ({"keys": [("x", 0, 16)]}, {"keys": [("y", 0, 64)]},
                {"or": [[("x", "range", 0, 2), ("a", "in", [1])]]},
                {"or": [[("y", "range", 0, 2), ("d", "in", [1])]]}):
        with pytest.raises(ccq.CcqError) as e:
            ccq.plan_check(tb, dict(q, **bad))
        assert e.value.status == ccq.E_UNSUPPORTED, bad
    cols = _composite_cols()
    cols["z"] = dict(cols["x"])
    tb = _host_table(cols, 1000)
    with pytest.raises(ccq.CcqError) as e:
        ccq.plan_check(tb, dict(q, preds=[("x", "range", 0, 5), ("y", "range", 0, 5), ("z", "range", 0, 5)]))
    assert e.value.status == ccq.E_UNSUPPORTED


def test_composite_table_create_rejects():
    cols = _composite_cols()
    cols["x"]["point_values"] = cols["x"]["point_values"].to(torch.int32)     # run values are int64
    with pytest.raises(ccq.CcqError, match="share one type"):
        _host_table(cols, 1000)
    L = ccq.lib()
    d = ccq._column_desc(_composite_cols()["a"], 1000)
    d.n_points = 3                                  # points on a plain RLE column
    h = ccq.ctypes.c_void_p()
    ctx = ccq.Context(ccq.HOST_ONLY)
    assert L.ccq_table_create(ctx.h, 1000, ccq.ctypes.byref(d), 1, ccq.ctypes.byref(h)) == ccq.E_INVALID
    assert b"n_points" in L.ccq_last_error()
    d = ccq._column_desc(_composite_cols()["y"], 1000)
    d.point_values = None
    assert L.ccq_table_create(ctx.h, 1000, ccq.ctypes.byref(d), 1, ccq.ctypes.byref(h)) == ccq.E_INVALID


def test_tune_cache_file_round_trip(tmp_path):
    """The tuning cache's text file: a missing file loads nothing, a written
    file reloads the same entries, malformed files are rejected and merge
    nothing."""
    ctx = ccq.Context(ccq.HOST_ONLY)
    path = str(tmp_path / "tune.txt")
    assert ctx.tune_cache_load(path) == 0                      # no file yet
    assert ctx.tune_cache_save(path) == 0
    assert open(path).read().splitlines() == ["ccq-tune-cache 1"]
    with open(path, "a") as f:
        f.write("00000000000000ab 32 12.5\n0123456789abcdef 512 355.25\n0000000000000001 524288 1.5\n")
    assert ctx.tune_cache_load(path) == 3                      # up to 2^19 tiles per item
    out = str(tmp_path / "out.txt")
    assert ctx.tune_cache_save(out) == 3
    lines = open(out).read().splitlines()
    assert lines[0] == "ccq-tune-cache 1"
    assert sorted(lines[1:]) == sorted(["00000000000000ab 32 12.5", "0123456789abcdef 512 355.25",
                                        "0000000000000001 524288 1.5"])
    for bad in ("not a cache\n", "ccq-tune-cache 1\nzz 1 2\n", "ccq-tune-cache 1\n00ab 0 1.0\n",
                "ccq-tune-cache 1\n00ab 8 1.0 extra\n", "ccq-tune-cache 1\n00ab 524289 1.0\n"):
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        other = ccq.Context(ccq.HOST_ONLY)
        with pytest.raises(ccq.CcqError) as e:
            other.tune_cache_load(str(p))
        assert e.value.status == ccq.E_INVALID
        assert other.tune_cache_save(str(tmp_path / "empty.txt")) == 0      # nothing merged
