"""Seeded random tiny tables and queries shared by the oracle pins and the
GPU parity tests (inputs only; no query arithmetic)."""
import numpy as np

import datagen


def tiny_table(rng, n):
    cols = {}
    for i in range(3):
        R = int(rng.integers(1, max(2, n // 2)))
        cuts = np.sort(rng.choice(np.arange(1, n), size=min(R - 1, n - 1), replace=False)) if n > 1 else []
        ends = np.r_[cuts, n].astype(np.int64)
        cols["r%d" % i] = {"enc": "rle", "values": rng.integers(-5, 20, size=len(ends)).astype(np.int64),
                           "run_ends": ends}
    nnz = int(rng.integers(0, n + 1))
    pos = np.sort(rng.choice(n, size=nnz, replace=False)).astype(np.int32)
    cols["s"] = {"enc": "index", "positions": pos, "values": rng.integers(-100, 100, size=nnz).astype(np.int64)}
    w = int(rng.integers(1, 9))
    codes = rng.integers(0, 1 << w, size=n).astype(np.uint32)
    cols["d"] = {"enc": "bitpacked", "packed": datagen.pack_codes(codes, w), "w": w, "base": 0}
    wp = int(rng.integers(1, 33))
    codes = rng.integers(0, 1 << wp, size=n, dtype=np.uint64).astype(np.uint32)
    cols["p"] = {"enc": "bitpacked", "packed": datagen.pack_codes(codes, wp), "w": wp,
                 "base": -(1 << (wp - 1))}
    return {"n_rows": n, "columns": cols}, w


def tiny_query(rng, n, wd):
    preds = []
    if rng.random() < 0.7:
        lo = int(rng.integers(-6, 20))
        preds.append(("r0", "range", lo, lo + int(rng.integers(1, 20))))
    if rng.random() < 0.5:
        lo = int(rng.integers(-6, 20))
        preds.append(("r1", "range", lo, lo + int(rng.integers(1, 25))))
    if rng.random() < 0.5:
        preds.append(("d", "in", sorted(set(int(x) for x in rng.integers(0, 1 << wd, size=int(rng.integers(0, 6)))))))
    if rng.random() < 0.3:
        preds.append(("p", "range", int(rng.integers(-1000, 0)), int(rng.integers(0, 1000))))
    keys = []
    if rng.random() < 0.5:
        keys.append(("d", int(rng.integers(0, 2)), 1 << wd))
    if rng.random() < 0.4:
        keys.append(("r2", 0, 20))
        preds.append(("r2", "range", 0, 20))
    aggs = [("count",)] if rng.random() < 0.5 else []
    for c in ("r0", "s", "p", "r1"):
        if rng.random() < 0.4:
            aggs.append(("sum", c))
    a = int(rng.integers(0, n))
    b = int(rng.integers(a, n + 1))
    win = (a, b) if rng.random() < 0.3 else (0, n)
    return {"preds": preds, "keys": keys, "aggs": aggs, "window": win}


def tiny_query_with_not(rng, n, wd):
    """tiny_query with some predicates negated, plus plain and negated
    predicates stacked on one column (their conjunction is then a list of
    value intervals)."""
    q = tiny_query(rng, n, wd)
    preds = []
    for p in q["preds"]:
        if p[0] != "r2" and rng.random() < 0.5:
            p = (p[0], "not_" + p[1]) + tuple(p[2:])
        preds.append(p)
    if rng.random() < 0.6:
        lo = int(rng.integers(-3, 12))
        preds.append(("r0", "not_range", lo, lo + int(rng.integers(0, 6))))
    if rng.random() < 0.5:
        preds.append(("d", "not_in", sorted(set(int(x) for x in rng.integers(0, 1 << wd, size=int(rng.integers(1, 8)))))))
    if rng.random() < 0.4:
        lo = int(rng.integers(-500, 500))
        preds.append(("p", "not_range", lo, lo + int(rng.integers(1, 400))))
    q["preds"] = preds
    return q


def _rle_literal(rng, col):
    op = ["range", "in", "not_range", "not_in"][int(rng.integers(0, 4))]
    if op.endswith("range"):
        lo = int(rng.integers(-6, 20))
        return (col, op, lo, lo + int(rng.integers(0, 12)))
    return (col, op, sorted(set(int(x) for x in rng.integers(-5, 20, size=int(rng.integers(0, 5))))))


def tiny_query_with_or(rng, n, wd):
    """tiny_query_with_not plus OR clauses: one or two over the RLE columns
    (two or three predicates, a column possibly named twice), at times one
    over the dictionary column alone or the wide column alone, and at times
    one over RLE and bit-packed columns."""
    q = tiny_query_with_not(rng, n, wd)
    clauses = []
    for _ in range(int(rng.integers(1, 3))):
        cols = ["r%d" % int(rng.integers(0, 3)) for _ in range(int(rng.integers(2, 4)))]
        clauses.append([_rle_literal(rng, c) for c in cols])
    if rng.random() < 0.4:
        clauses.append([("d", "in", sorted(set(int(x) for x in rng.integers(0, 1 << wd, size=3)))),
                        ("d", "range", int(rng.integers(0, 1 << wd)), int(rng.integers(0, 1 << wd)) + 1)])
    if rng.random() < 0.3:
        lo = int(rng.integers(-1000, 0))
        clauses.append([("p", "range", lo, lo + 300), ("p", "not_range", -2000, 2000)])
    if rng.random() < 0.5:
        # one clause over RLE and bit-packed columns (RLE mask OR Plain mask)
        d_lit = ("d", "in", sorted(set(int(x) for x in rng.integers(0, 1 << wd, size=3))))
        lo = int(rng.integers(-1000, 500))
        p_lit = ("p", ["range", "not_range"][int(rng.integers(0, 2))], lo, lo + int(rng.integers(1, 800)))
        pick = int(rng.integers(0, 3))
        if pick == 0:
            clauses.append([_rle_literal(rng, "r%d" % int(rng.integers(0, 3))), d_lit])
        elif pick == 1:
            clauses.append([_rle_literal(rng, "r0"), _rle_literal(rng, "r1"), p_lit])
        else:
            clauses.append([d_lit, p_lit])
    q["or"] = clauses
    return q


def _index_literal(rng):
    """A predicate on the Index column s (unlisted rows hold 0): a range or
    an IN-list, with or without 0, plain or negated."""
    op = ["range", "in", "not_range", "not_in"][int(rng.integers(0, 4))]
    if op.endswith("range"):
        lo = int(rng.integers(-120, 60))
        return ("s", op, lo, lo + int(rng.integers(0, 150)))
    vals = set(int(x) for x in rng.integers(-100, 100, size=int(rng.integers(0, 6))))
    if rng.random() < 0.4:
        vals.add(0)
    return ("s", op, sorted(vals))


def tiny_query_with_rle_index_or(rng, n, wd):
    """tiny_query_with_not plus one OR clause over one or two RLE columns and
    the Index column s (RLE mask OR Index mask, Table 4), at times beside
    OR clauses over RLE columns alone and a predicate on s; about half the
    queries name no bit-packed column (run mode), the rest do (row mode)."""
    q = tiny_query_with_not(rng, n, wd)
    if rng.random() < 0.5:
        q["preds"] = [p for p in q["preds"] if p[0] not in ("d", "p")]
        q["keys"] = [k for k in q["keys"] if k[0] not in ("d", "p")]
        q["aggs"] = [a for a in q["aggs"] if a[-1] not in ("d", "p")]
    cols = ["r%d" % int(rng.integers(0, 3)) for _ in range(int(rng.integers(1, 3)))]
    clause = [_rle_literal(rng, c) for c in cols] + [_index_literal(rng)]
    clauses = [[clause[i] for i in rng.permutation(len(clause))]]
    if rng.random() < 0.4:
        clauses.append([_rle_literal(rng, "r%d" % int(rng.integers(0, 3))) for _ in range(2)])
    if rng.random() < 0.3:
        q["preds"] = q["preds"] + [_index_literal(rng)]
    q["or"] = clauses
    return q


def tiny_query_with_index_pred(rng, n, wd):
    """tiny_query_with_not plus one or two predicates on the Index column s
    (unlisted rows hold 0): ranges and IN-lists with and without 0, plain or
    negated, at times inside a one-column OR clause."""
    q = tiny_query_with_not(rng, n, wd)
    preds = []
    for _ in range(int(rng.integers(1, 3))):
        op = ["range", "in", "not_range", "not_in"][int(rng.integers(0, 4))]
        if op.endswith("range"):
            lo = int(rng.integers(-120, 60))
            preds.append(("s", op, lo, lo + int(rng.integers(0, 150))))
        else:
            vals = set(int(x) for x in rng.integers(-100, 100, size=int(rng.integers(0, 6))))
            if rng.random() < 0.4:
                vals.add(0)
            preds.append(("s", op, sorted(vals)))
    if rng.random() < 0.3:
        q["or"] = [preds]
    else:
        q["preds"] = q["preds"] + preds
    return q


def tiny_query_with_exprs(rng, n, wd):
    """tiny_query whose aggregates include MIN, MAX and SUM / MIN / MAX of
    the row-wise sum, difference or product of two RLE or bit-packed
    columns."""
    q = tiny_query(rng, n, wd)
    cols = ["r0", "r1", "r2", "d", "p"]
    aggs = [a for a in q["aggs"] if a[0] == "count" or a[1] != "s"]
    for _ in range(int(rng.integers(1, 4))):
        f = ["sum", "min", "max"][int(rng.integers(0, 3))]
        a = cols[int(rng.integers(0, len(cols)))]
        if rng.random() < 0.5:
            aggs.append((f, a))
        else:
            b = cols[int(rng.integers(0, len(cols)))]
            aggs.append((f, (a, "+-*"[int(rng.integers(0, 3))], b)))
    q["aggs"] = aggs
    return q


def composite_columns(rng, n, p_single=None):
    """Two composite columns over n rows (Section 3.2): x as RLE + Index
    (pure runs of two or more rows, single rows as points) and y as Plain +
    Index (values outside [base, base + 2^w) as points; the
    codes at those rows are random, since they are never read)."""
    # segments: pure runs of 2-6 rows and single rows (points), in random order
    p_single = float(rng.choice([0.0, 0.3, 0.9])) if p_single is None else p_single
    rv, rs, re_, pp, pv = [], [], [], [], []
    r = 0
    while r < n:
        v = int(rng.integers(-5, 20))
        if rng.random() < p_single or r + 2 > n:
            pp.append(r)
            pv.append(v)
            r += 1
        else:
            e = min(n, r + int(rng.integers(2, 7)))
            rv.append(v)
            rs.append(r)
            re_.append(e)
            r = e
    xs = np.zeros(n, dtype=np.int64)
    for v, a, b in zip(rv, rs, re_):
        xs[a:b] = v
    xs[np.asarray(pp, dtype=np.int64)] = pv
    x = {"enc": "rle+index", "values": np.asarray(rv, dtype=np.int64), "run_starts": np.asarray(rs, dtype=np.int64),
         "run_ends": np.asarray(re_, dtype=np.int64), "positions": np.asarray(pp, dtype=np.int32),
         "point_values": np.asarray(pv, dtype=np.int64)}
    w = int(rng.integers(1, 12))
    base = int(rng.integers(-50, 50))
    ys = base + rng.integers(0, 1 << w, size=n)
    out = rng.random(n) < rng.choice([0.0, 0.05, 0.3])
    ys = np.where(out, rng.choice([-1, 1], size=n) * rng.integers(1 << 20, 1 << 40, size=n), ys).astype(np.int64)
    inside = (ys >= base) & (ys < base + (1 << w))
    codes = np.where(inside, ys - base, rng.integers(0, 1 << w, size=n)).astype(np.uint32)
    pos = np.flatnonzero(~inside).astype(np.int32)
    y = {"enc": "plain+index", "packed": datagen.pack_codes(codes, w), "w": w, "base": base,
         "positions": pos, "point_values": ys[pos].copy()}
    return x, y, xs, ys


def abi_column(col, n_rows):
    """The library's form of a column.  RLE + Index takes the RLE part as
    run ends only: run i covers the rows from the previous end to its own
    that no point lists, and the last run ends at n_rows (a column of points
    only gets one run, whose value is never read)."""
    if col["enc"] != "rle+index":
        return col
    v, e = col["values"], np.asarray(col["run_ends"], dtype=np.int64).copy()
    if len(e) == 0:
        v, e = np.zeros(1, dtype=np.asarray(v).dtype), np.array([n_rows], dtype=np.int64)
    e[-1] = n_rows
    return {"enc": "rle+index", "values": v, "run_ends": e, "positions": col["positions"],
            "point_values": col["point_values"]}


def composite_table(rng, n):
    """tiny_table's columns plus the composites x and y."""
    t, wd = tiny_table(rng, n)
    x, y, _, _ = composite_columns(rng, n)
    t["columns"]["x"] = x
    t["columns"]["y"] = y
    return t, wd


def tiny_query_with_composites(rng, n, wd):
    """Predicates, SUM, MIN, MAX and expressions over the composite columns
    x and y beside the plain columns; keys on the other columns."""
    preds = []
    lo = int(rng.integers(-6, 20))
    kind = rng.choice(["range", "not_range", "in"])
    if rng.random() < 0.7:
        if kind == "in":
            preds.append(("x", "in", sorted(set(int(v) for v in rng.integers(-5, 20, size=int(rng.integers(0, 6)))))))
        else:
            preds.append(("x", str(kind), lo, lo + int(rng.integers(1, 15))))
    if rng.random() < 0.5:
        a = int(rng.integers(-100, 100))
        preds.append(("y", str(rng.choice(["range", "not_range"])), a, a + int(rng.integers(1, 400))))
    if rng.random() < 0.4:
        lo = int(rng.integers(-6, 20))
        preds.append(("r0", "range", lo, lo + int(rng.integers(1, 20))))
    if rng.random() < 0.3:
        preds.append(("d", "in", sorted(set(int(v) for v in rng.integers(0, 1 << wd, size=int(rng.integers(0, 6)))))))
    keys = []
    if rng.random() < 0.4:
        keys.append(("d", 0, 1 << wd))
    if rng.random() < 0.3:
        keys.append(("r2", 0, 20))
        preds.append(("r2", "range", 0, 20))
    aggs = [("count",)]
    pool = [("sum", "x"), ("sum", "y"), ("min", "x"), ("max", "y"), ("max", "x"), ("min", "y"), ("sum", "s"),
            ("sum", ("x", "+", "y")), ("sum", ("x", "*", "r0")), ("min", ("y", "-", "x")), ("sum", "r1")]
    for i in rng.permutation(len(pool))[:int(rng.integers(1, 5))]:
        aggs.append(pool[i])
    a = int(rng.integers(0, n))
    b = int(rng.integers(a, n + 1))
    win = (a, b) if rng.random() < 0.3 else (0, n)
    return {"preds": preds, "keys": keys, "aggs": aggs, "window": win}
