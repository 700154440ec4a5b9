"""Pins of the encoding oracle (oracle/encode.py), CPU only: the paper's
worked examples of Section 3, round trips, the invariants that define each
encoding, the order statistics against a full sort, and each branch of the
encoding choice on inputs built to take it."""
import json
import os

import numpy as np
import pytest

from oracle import encode as E

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "encodings.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_paper_plain_to_rle_example():
    g = _golden()["plain_to_rle"]
    vals, ends = E.plain_to_rle(np.array(g["input"], dtype=np.int32))
    assert vals.tolist() == g["values"]
    assert (ends - 1).tolist() == g["ends_inclusive"]
    assert [0] + ends[:-1].tolist() == g["starts"]


def test_paper_plain_to_plain_index_example():
    g = _golden()["plain_to_plain_index"]
    x = np.array(g["input"], dtype=np.int64)
    # the narrow part 1..3 needs 2 bits above base 1
    packed, (pos, pv) = E.plain_to_plain_index(x, 2, 1)
    assert pos.tolist() == g["outlier_positions"] and pv.tolist() == g["outlier_values"]
    dec = E.decode_plain_index(packed, 2, 1, (pos, pv), len(x), np.int64)
    assert dec.tolist() == g["input"]
    assert dec[:3].tolist() == g["plain"]
    # the outliers' slots hold code 0
    assert int(packed[0]) >> 6 & 15 == 0


def test_paper_plain_to_rle_index_example():
    g = _golden()["plain_to_rle_index"]
    (rv, rs, re_), (ip, iv) = E.plain_to_rle_index(np.array(g["input"], dtype=np.int32))
    assert rv.tolist() == g["rle_values"] and rs.tolist() == g["rle_starts"]
    assert (re_ - 1).tolist() == g["rle_ends_inclusive"]
    assert iv.tolist() == g["index_values"] and ip.tolist() == g["index_positions"]


def _columns(seed):
    rng = np.random.default_rng([seed, 8080])
    n = int(rng.integers(1, 3000))
    kind = seed % 5
    if kind == 0:          # long runs
        x = np.repeat(rng.integers(-5, 5, size=n), rng.integers(1, 50, size=n))[:n]
    elif kind == 1:        # every row its own value
        x = rng.permutation(n) - n // 2
    elif kind == 2:        # runs and singles mixed
        x = np.where(rng.random(n) < 0.3, rng.integers(0, 1000, size=n), np.arange(n) // 40)
    elif kind == 3:        # extremes of int64
        x = rng.choice(np.array([np.iinfo(np.int64).min, -1, 0, 1, np.iinfo(np.int64).max]), size=n)
    else:                  # one value
        x = np.full(n, 7)
    dt = np.int64 if kind == 3 or seed % 2 else np.int32
    return np.asarray(x).astype(dt)


@pytest.mark.parametrize("seed", range(40))
def test_round_trips_and_invariants(seed):
    x = _columns(seed)
    n = len(x)
    vals, ends = E.plain_to_rle(x)
    assert np.array_equal(E.decode_rle(vals, ends), x)
    assert ends[-1] == n and np.all(np.diff(ends) > 0)
    assert np.all(vals[1:] != vals[:-1])                 # maximal runs
    runs, points = E.plain_to_rle_index(x)
    rv, rs, re_ = runs
    assert np.all(re_ - rs >= 2)                          # the RLE part holds runs of two or more rows
    covered = np.zeros(n, dtype=int)
    for s_, e_ in zip(rs, re_):
        covered[s_:e_] += 1
    covered[points[0]] += 1
    assert np.all(covered == 1)                           # disjoint, covering
    assert len(rv) + len(points[0]) == len(vals)
    assert np.array_equal(E.decode_rle_index(runs, points, n, x.dtype), x)
    for w in (1, 3, 8, 17, 32):
        base = int(np.sort(x.astype(np.int64))[n // 3])
        packed, pts = E.plain_to_plain_index(x, w, base)
        assert len(packed) == (n * w + 31) // 32 + 2
        inside = [(base <= int(v) < base + (1 << w)) for v in x]
        assert pts[0].tolist() == [i for i, ok in enumerate(inside) if not ok]
        if n <= 600:
            assert np.array_equal(E.decode_plain_index(packed, w, base, pts, n, x.dtype), x)


def test_pack_bits_by_hand():
    # codes 5 (101), 2 (010), 7 (111) at 3 bits: bits 0-2, 3-5, 6-8 -> 0b111_010_101
    assert int(E.pack_bits([5, 2, 7], 3)[0]) == 0b111010101
    # a 20-bit code straddling two words
    p = E.pack_bits([0, (1 << 20) - 1], 20)
    assert int(p[0]) == 0xFFF00000 and int(p[1]) == 0xFF


@pytest.mark.parametrize("seed", range(20))
def test_choose_order_statistics(seed):
    x = _columns(seed)
    c = E.choose(x)
    xs = sorted(int(v) for v in x)
    n = len(xs)
    assert (c["min_value"], c["max_value"]) == (xs[0], xs[-1])
    assert (c["lo_cut"], c["hi_cut"]) == (xs[n // 20], xs[n - 1 - n // 20])
    assert c["runs"] == len(E.plain_to_rle(x)[0])


def test_choose_branches():
    rng = np.random.default_rng(3)
    n = 1_200_000
    small = E.choose(np.arange(1000, dtype=np.int32))
    assert small["choice"] == "plain" and small["bit_width"] == 10 and small["base"] == 0
    long_runs = np.repeat(rng.integers(0, 100, size=n // 100), 100).astype(np.int32)
    assert E.choose(long_runs)["choice"] == "rle"
    # blocks of 4000 constant rows and 200 rows of distinct values: the
    # single-row runs bring RLE under the ratio, the long runs alone stay above
    blocks = n // 4200
    mixed = np.concatenate([np.concatenate([np.full(4000, b), -1 - np.arange(200) - 200 * b])
                            for b in range(blocks)]).astype(np.int32)
    c = E.choose(mixed)
    assert c["choice"] == "rle+index", c
    assert c["index_points"] == c["single_runs"] > 0
    # 16-bit values with 2% of rows far out: the cut range is narrower
    narrow = rng.integers(0, 1 << 16, size=n).astype(np.int64)
    far = rng.choice(n, size=n // 50, replace=False)
    narrow[far] = 1 << 40
    c = E.choose(narrow)
    assert c["choice"] == "plain+index" and c["bit_width"] == 16
    # centered on the cut range, which lies inside the kept codes
    assert c["base"] <= c["lo_cut"] and c["hi_cut"] < c["base"] + (1 << 16)
    assert c["index_points"] == len(far) + int(((narrow < c["base"]) & (narrow < (1 << 40))).sum())
    uniform = rng.integers(0, 1 << 20, size=n).astype(np.int32)
    c = E.choose(uniform)
    assert c["choice"] == "plain" and c["bit_width"] == 20
    wide = rng.integers(-(1 << 62), 1 << 62, size=n).astype(np.int64)
    assert E.choose(wide)["choice"] == "rle"
