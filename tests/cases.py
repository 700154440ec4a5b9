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
