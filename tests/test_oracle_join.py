"""Pins of the join oracle (oracle/join.py), CPU only: the paper's two join
examples, brute force over every row pair on seeded tables of every
encoding pair, the closed form COUNT = sum over values of
count_left(v) * count_right(v), and sqlite3's inner join."""
import json
import os
import sqlite3
from collections import Counter

import numpy as np
import pytest

import datagen
from oracle import join as J
from oracle import oracle
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "joins.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _packed(vals, w=8):
    return {"enc": "bitpacked", "packed": datagen.pack_codes(np.asarray(vals, dtype=np.uint32), w), "w": w, "base": 0}


def test_paper_select_example():
    g = _golden()["select_example"]
    ra, sb, sc = _packed(g["R_A"]), _packed(g["S_B"]), _packed(g["S_C"])
    blocks = J.join_blocks(J.entries(ra, 3, 0, 3), J.entries(sb, 3, 0, 3))
    pr = J.pairs(blocks)
    assert [p[0] for p in pr] == g["left_index"] and [p[1] for p in pr] == g["right_index"]
    assert J.apply(blocks, sc, 3, "right").tolist() == g["apply_S_C"]


def test_paper_plain_rle_example():
    g = _golden()["plain_rle_example"]
    plain = _packed(g["plain"])
    rle = {"enc": "rle", "values": np.array(g["rle_values"], dtype=np.int64),
           "run_ends": np.array(g["rle_ends_inclusive"], dtype=np.int64) + 1}
    blocks = J.join_blocks(J.entries(plain, 3, 0, 3), J.entries(rle, 3, 0, 3))
    # the plain side expands by the matching run's length; the RLE side keeps run ranges
    assert Counter(a for a0, al, b0, bl in blocks for a in [a0] * bl) == Counter(g["plain_index"])
    runs = Counter((b0, b0 + bl - 1) for a0, al, b0, bl in blocks)
    ends = np.array(g["rle_ends_inclusive"])
    starts = np.concatenate([[0], ends[:-1] + 1])
    assert runs == Counter((int(starts[r]), int(ends[r])) for r in g["rle_runs"])
    assert runs == Counter(zip(g["rle_starts"], g["rle_ends_inclusive_out"]))


def _column(rng, kind, n):
    if kind == "rle":
        cuts = np.sort(rng.choice(np.arange(1, n), size=min(n - 1, int(rng.integers(0, n))), replace=False)) if n > 1 else []
        ends = np.r_[cuts, n].astype(np.int64)
        return {"enc": "rle", "values": rng.integers(0, 6, size=len(ends)).astype(np.int64), "run_ends": ends}
    if kind == "index":
        pos = np.sort(rng.choice(n, size=int(rng.integers(0, n + 1)), replace=False)).astype(np.int32)
        return {"enc": "index", "positions": pos, "values": rng.integers(0, 6, size=len(pos)).astype(np.int64)}
    return _packed(rng.integers(0, 6, size=n), 3)


def _rows(col, n):
    """Rows present in the joined relation with their values."""
    if col["enc"] == "index":
        return [(int(p), int(v)) for p, v in zip(col["positions"], col["values"])]
    return list(enumerate(brute.decode_rows(col, n)))


@pytest.mark.parametrize("seed", range(45))
def test_join_matches_brute_force_and_sqlite(seed):
    rng = np.random.default_rng([seed, 600])
    kinds = ["rle", "index", "bitpacked"]
    lk, rk = kinds[seed % 3], kinds[(seed // 3) % 3]
    nl, nr = int(rng.integers(1, 120)), int(rng.integers(1, 120))
    L, R = _column(rng, lk, nl), _column(rng, rk, nr)
    lb, le = sorted(int(x) for x in rng.integers(0, nl + 1, size=2))
    rb, re_ = sorted(int(x) for x in rng.integers(0, nr + 1, size=2))
    blocks = J.join_blocks(J.entries(L, nl, lb, le), J.entries(R, nr, rb, re_))
    got = sorted(J.pairs(blocks))
    lrows = [(a, v) for a, v in _rows(L, nl) if lb <= a < le]
    rrows = [(b, v) for b, v in _rows(R, nr) if rb <= b < re_]
    assert got == sorted((a, b) for a, va in lrows for b, vb in rrows if va == vb)
    cl, cr = Counter(v for _, v in lrows), Counter(v for _, v in rrows)
    assert len(got) == sum(cl[v] * cr[v] for v in cl)
    db = sqlite3.connect(":memory:")
    db.execute("CREATE TABLE l (a INTEGER, v INTEGER)")
    db.execute("CREATE TABLE r (b INTEGER, v INTEGER)")
    db.executemany("INSERT INTO l VALUES (?, ?)", lrows)
    db.executemany("INSERT INTO r VALUES (?, ?)", rrows)
    assert sorted(db.execute("SELECT a, b FROM l JOIN r ON l.v = r.v").fetchall()) == got
    # Apply Join Index: a right-side column read at the pairs' right rows
    C = _column(rng, "rle", nr)
    ap = J.apply(blocks, C, nr, "right")
    crow = brute.decode_rows(C, nr)
    assert ap.tolist() == [crow[b] for _, b in J.pairs(blocks)]
    # blocks of RLE entries stay ranges (Table 6): a block's length is its run's clipped length
    if lk == "rle":
        assert all(al >= 1 for _, al, _, _ in blocks)
