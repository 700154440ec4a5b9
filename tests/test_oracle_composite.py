"""Pins of the oracle's composite encodings (Section 3.2: RLE + Index,
Plain + Index), CPU only: the paper's two examples, round trips through the
oracle's encoders, predicates as the OR of the parts' masks (Section 5.4:
a composite mask is the disjunction of its RLE and Index parts), and brute
force plus sqlite3 on tiny tables."""
import json
import os

import numpy as np
import pytest

import datagen
from oracle import encode as E
from oracle import oracle
from tests import brute
from tests.cases import composite_columns, composite_table, tiny_query_with_composites

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "composite.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("garbage", [0, 77, 255])
def test_paper_plain_index_example(garbage):
    """The Plain slots at outlier positions hold anything and are never read."""
    g = _golden()["plain_index"]
    n = g["n_rows"]
    codes = np.full(n, garbage, dtype=np.uint32)
    codes[:len(g["plain"])] = g["plain"]
    col = {"enc": "plain+index", "packed": datagen.pack_codes(codes, 8), "w": 8, "base": 0,
           "positions": np.array(g["outlier_positions"], dtype=np.int32),
           "point_values": np.array(g["outlier_values"], dtype=np.int64)}
    assert oracle.decode(col, n).tolist() == g["expect_rows"]


def test_paper_rle_index_example():
    g = _golden()["rle_index"]
    col = {"enc": "rle+index", "values": np.array(g["rle_values"], dtype=np.int64),
           "run_starts": np.array(g["rle_starts"], dtype=np.int64),
           "run_ends": np.array(g["rle_ends_inclusive"], dtype=np.int64) + 1,
           "positions": np.array(g["index_positions"], dtype=np.int32),
           "point_values": np.array(g["index_values"], dtype=np.int64)}
    assert oracle.decode(col, g["n_rows"]).tolist() == g["expect_rows"]
    # the oracle's encoder gives the same parts
    (v, s, e), (p, pv) = E.plain_to_rle_index(np.array(g["expect_rows"]))
    assert v.tolist() == g["rle_values"] and s.tolist() == g["rle_starts"]
    assert (e - 1).tolist() == g["rle_ends_inclusive"]
    assert p.tolist() == g["index_positions"] and pv.tolist() == g["index_values"]


@pytest.mark.parametrize("seed", range(20))
def test_round_trip_through_the_encoders(seed):
    rng = np.random.default_rng([seed, 41])
    n = int(rng.integers(1, 3000))
    x = np.repeat(rng.integers(-1000, 1000, size=n), rng.integers(1, 5, size=n))[:n].astype(np.int64)
    (v, s, e), (p, pv) = E.plain_to_rle_index(x)
    col = {"enc": "rle+index", "values": v, "run_starts": s, "run_ends": e, "positions": p.astype(np.int32),
           "point_values": pv}
    assert np.array_equal(oracle.decode(col, n), x)
    w = int(rng.integers(1, 16))
    base = int(rng.integers(-(1 << 20), 1 << 20))
    y = np.where(rng.random(n) < 0.1, rng.integers(-(1 << 40), 1 << 40, size=n), base + rng.integers(0, 1 << w, size=n))
    packed, (p, pv) = E.plain_to_plain_index(y, w, base)
    col = {"enc": "plain+index", "packed": packed, "w": w, "base": base, "positions": p.astype(np.int32),
           "point_values": pv}
    assert np.array_equal(oracle.decode(col, n), y)
    assert np.array_equal(oracle.decode(col, n, n // 3, n - n // 4), y[n // 3:n - n // 4])


def _part_rows(col, n, test):
    """Rows passing `test` by the parts: the pure runs (or the Plain codes of
    unlisted rows) whose value passes, united with the passing points."""
    rows = set()
    if col["enc"] == "rle+index":
        for v, s, e in zip(col["values"], col["run_starts"], col["run_ends"]):
            if test(int(v)):
                rows.update(range(int(s), int(e)))
    else:
        listed = set(int(p) for p in col["positions"])
        plain = brute.decode_rows(dict(col, enc="bitpacked"), n)
        rows.update(r for r in range(n) if r not in listed and test(plain[r]))
    rows.update(int(p) for p, v in zip(col["positions"], col["point_values"]) if test(int(v)))
    return rows


@pytest.mark.parametrize("seed", range(30))
def test_predicates_select_the_union_of_the_parts(seed):
    rng = np.random.default_rng([seed, 42])
    n = int(rng.integers(1, 400))
    x, y, _, _ = composite_columns(rng, n)
    r = rng.integers(0, 1000, size=n).astype(np.int64)
    table = {"n_rows": n, "columns": {"x": x, "y": y,
                                      "r": {"enc": "index", "positions": np.arange(n, dtype=np.int32), "values": r}}}
    for name, col, lo, hi in (("x", x, -2, 9), ("y", y, -40, 60)):
        rows = _part_rows(col, n, lambda v: lo <= v < hi)
        q = {"preds": [(name, "range", lo, hi)], "keys": [], "aggs": [("count",), ("sum", "r")], "window": (0, n)}
        got = oracle.run(table, q)
        assert got["counts"] == [len(rows)]
        assert got["aggs"][0][1] == sum(int(r[i]) for i in rows)
        # NOT: the complement within the window (Section 5.4: NOT of a composite mask)
        q["preds"] = [(name, "not_range", lo, hi)]
        got = oracle.run(table, q)
        assert got["counts"] == [n - len(rows)]


@pytest.mark.parametrize("seed", range(40))
def test_composite_queries_match_brute_force_and_sqlite(seed):
    rng = np.random.default_rng([seed, 43])
    n = int(rng.integers(1, 200))
    table, wd = composite_table(rng, n)
    for _ in range(3):
        q = tiny_query_with_composites(rng, n, wd)
        got = oracle.run(table, q)
        assert got == brute.run(table, q), q
        assert got == brute.run_sqlite(table, q), q


def test_composite_validation():
    n = 10
    ok = {"enc": "rle+index", "values": np.array([1, 2], dtype=np.int64), "run_starts": np.array([0, 5]),
          "run_ends": np.array([4, 10]), "positions": np.array([4], dtype=np.int32),
          "point_values": np.array([7], dtype=np.int64)}
    assert oracle.decode(ok, n).tolist() == [1] * 4 + [7] + [2] * 5
    bad = [
        dict(ok, positions=np.array([3], dtype=np.int32)),                       # inside a run, row 4 uncovered
        dict(ok, positions=np.zeros(0, dtype=np.int32), point_values=np.zeros(0, dtype=np.int64)),   # a gap
        dict(ok, run_starts=np.array([0, 3])),                                   # runs overlap
        dict(ok, run_ends=np.array([4, 11])),                                    # past the rows
        dict(ok, positions=np.array([4, 4], dtype=np.int32), point_values=np.array([7, 7], dtype=np.int64)),
    ]
    for b in bad:
        with pytest.raises(oracle.OracleError):
            oracle.decode(b, n)
    pk = {"enc": "plain+index", "packed": datagen.pack_codes(np.zeros(n, dtype=np.uint32), 4), "w": 4, "base": 0,
          "positions": np.array([2, 1], dtype=np.int32), "point_values": np.array([5, 6], dtype=np.int64)}
    with pytest.raises(oracle.OracleError):
        oracle.decode(pk, n)
