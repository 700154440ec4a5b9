"""Pure-Python brute force for tiny tables (test helper, no C, no numpy math).

Decodes every column row by row with its own decoder (the packed stream is
read as one Python big integer, a different route from the oracle's two-word
read), evaluates the query one row at a time and groups with a dict.  A
second route loads the decoded rows into sqlite3 and lets SQL do the work.
"""
from __future__ import annotations

import sqlite3


def decode_rows(col, n_rows):
    enc = col["enc"]
    if enc == "rle":
        out = []
        start = 0
        for v, e in zip(col["values"], col["run_ends"]):
            out.extend([int(v)] * (int(e) - start))
            start = int(e)
        assert len(out) == n_rows
        return out
    if enc == "index":
        out = [0] * n_rows
        for p, v in zip(col["positions"], col["values"]):
            out[int(p)] = int(v)
        return out
    if enc in ("bitpacked", "plain+index"):
        w = int(col["w"])
        big = 0
        for i, word in enumerate(col["packed"]):
            big |= int(word) << (32 * i)
        mask = (1 << w) - 1
        out = [int(col.get("base", 0)) + ((big >> (r * w)) & mask) for r in range(n_rows)]
        if enc == "plain+index":
            for p, v in zip(col["positions"], col["point_values"]):
                out[int(p)] = int(v)
        return out
    if enc == "rle+index":
        out = [None] * n_rows
        for v, s, e in zip(col["values"], col["run_starts"], col["run_ends"]):
            for r in range(int(s), int(e)):
                out[r] = int(v)
        for p, v in zip(col["positions"], col["point_values"]):
            assert out[int(p)] is None
            out[int(p)] = int(v)
        assert None not in out
        return out
    raise ValueError(enc)


def agg_value(rows, a, r):
    """Row r's argument of aggregate a: a column, or (col, op, col2) row-wise."""
    if a[0] == "count":
        return 1
    if isinstance(a[1], tuple):
        x, op, y = rows[a[1][0]][r], a[1][1], rows[a[1][2]][r]
        return x + y if op == "+" else x - y if op == "-" else x * y
    return rows[a[1]][r]


def run(table, query):
    n = int(table["n_rows"])
    rows = {name: decode_rows(c, n) for name, c in table["columns"].items()}
    r0, r1 = query.get("window", (0, n))
    groups = {}

    def holds(p, r):
        v = rows[p[0]][r]
        if p[1] in ("range", "not_range"):
            ok = p[2] <= v < p[3]
        else:
            ok = v in set(p[2])
        return not ok if p[1].startswith("not_") else ok

    for r in range(r0, r1):
        ok = all(holds(p, r) for p in query["preds"])
        ok = ok and all(any(holds(p, r) for p in clause) for clause in query.get("or", ()))
        if not ok:
            continue
        key = []
        for (c, shift, card) in query["keys"]:
            k = rows[c][r] >> shift
            if not (0 <= k < card):
                raise ValueError("key outside domain")
            key.append(k)
        key = tuple(key)
        acc = groups.setdefault(key, [0] + [None] * len(query["aggs"]))
        acc[0] += 1
        for i, a in enumerate(query["aggs"]):
            v = agg_value(rows, a, r)
            old = acc[1 + i]
            if a[0] == "min":
                acc[1 + i] = v if old is None else min(old, v)
            elif a[0] == "max":
                acc[1 + i] = v if old is None else max(old, v)
            else:
                acc[1 + i] = v if old is None else old + v
    if not query["keys"]:
        acc = groups.get((), [0] + [0] * len(query["aggs"]))
        return {"keys": [()], "counts": [acc[0]], "aggs": [tuple(acc[1:])]}
    ks = sorted(groups)
    return {"keys": ks, "counts": [groups[k][0] for k in ks], "aggs": [tuple(groups[k][1:]) for k in ks]}


def run_sqlite(table, query):
    """Same query through sqlite3 over the decoded rows."""
    n = int(table["n_rows"])
    names = list(table["columns"])
    rows = {name: decode_rows(table["columns"][name], n) for name in names}
    db = sqlite3.connect(":memory:")
    cols = ", ".join('"%s" INTEGER' % c for c in names)
    db.execute("CREATE TABLE t (rid INTEGER, %s)" % cols)
    db.executemany("INSERT INTO t VALUES (%s)" % ", ".join("?" * (len(names) + 1)),
                   [(r,) + tuple(rows[c][r] for c in names) for r in range(n)])
    r0, r1 = query.get("window", (0, n))
    where = ["rid >= %d" % r0, "rid < %d" % r1]

    def sql_pred(p):
        if p[1] in ("range", "not_range"):
            cond = '"%s" >= %d AND "%s" < %d' % (p[0], p[2], p[0], p[3])
        else:
            # an empty IN list is false (not NULL, which NOT would keep unknown)
            cond = ('"%s" IN (%s)' % (p[0], ", ".join(str(int(x)) for x in p[2]))) if len(p[2]) else "0"
        return "NOT (%s)" % cond if p[1].startswith("not_") else "(%s)" % cond

    where += [sql_pred(p) for p in query["preds"]]
    where += ["(%s)" % " OR ".join(sql_pred(p) for p in clause) for clause in query.get("or", ())]
    keys = ['("%s" >> %d)' % (c, s) for (c, s, _) in query["keys"]]
    def sql_arg(a):
        if isinstance(a[1], tuple):
            return '("%s" %s "%s")' % (a[1][0], a[1][1], a[1][2])
        return '"%s"' % a[1]

    aggs = ["COUNT(*)"] + ["COUNT(*)" if a[0] == "count" else "COALESCE(%s(%s), 0)" % (a[0].upper(), sql_arg(a))
                           for a in query["aggs"]]
    sql = "SELECT %s FROM t WHERE %s" % (", ".join(keys + aggs), " AND ".join(where))
    if keys:
        sql += " GROUP BY %s ORDER BY %s" % (", ".join(keys), ", ".join(keys))
    out = db.execute(sql).fetchall()
    nk = len(keys)
    return {"keys": [tuple(r[:nk]) for r in out], "counts": [r[nk] for r in out],
            "aggs": [tuple(r[nk + 1:]) for r in out]}
