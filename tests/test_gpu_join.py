"""GPU parity of the joins (ccq_join_index, ccq_join_apply) against the CPU
oracle (oracle/join.py).  Get Join Index lists its blocks of one left entry
in an unspecified order, so blocks are compared as sorted lists (and checked
to come in left-entry order); Apply Join Index is fed the oracle's blocks
and compared value by value."""
import sys

import numpy as np
import pytest

import datagen
from oracle import join as J

pytestmark = pytest.mark.gpu

KINDS = ["rle", "index", "bitpacked"]
I64 = np.iinfo(np.int64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_10092_amd import ccq
    assert torch.cuda.is_available()
    return ccq.Context(0)


def column(rng, kind, n, domain, vtype=np.int64, values=None):
    """A column of n rows whose values lie in [0, domain) (or are drawn from
    `values`), runs of 1-40 rows for RLE, about half the rows listed for
    Index."""
    draw = (lambda k: rng.choice(np.asarray(values, dtype=np.int64), size=k)) if values is not None else \
        (lambda k: rng.integers(0, domain, size=k))
    if kind == "rle":
        lens = rng.integers(1, 41, size=n // 20 + 2)
        ends = np.cumsum(lens)
        ends = np.r_[ends[ends < n], n].astype(np.int64)
        return {"enc": "rle", "values": draw(len(ends)).astype(vtype), "run_ends": ends}
    if kind == "index":
        pos = np.flatnonzero(rng.random(n) < 0.5)
        ptype = np.int32 if n < (1 << 31) else np.int64
        return {"enc": "index", "positions": pos.astype(ptype), "values": draw(len(pos)).astype(vtype)}
    w = max(1, int(domain - 1).bit_length())
    return {"enc": "bitpacked", "packed": datagen.pack_codes(draw(n).astype(np.uint32), w), "w": w, "base": 0}


def table(ctx, col, n):
    from paper_2506_10092_amd import ccq
    return ccq.Table(ctx, n, ccq.to_device({"c": col}))


def block_list(t):
    return [tuple(int(x) for x in row) for row in t.cpu().numpy().tolist()]


def check_join(ctx, L, nl, R, nr, lw=None, rw=None):
    from paper_2506_10092_amd import ccq
    lw = lw or (0, nl)
    rw = rw or (0, nr)
    want = J.join_blocks(J.entries(L, nl, *lw), J.entries(R, nr, *rw))
    tl, tr = table(ctx, L, nl), table(ctx, R, nr)
    got, n_pairs = ccq.join_index(tl, "c", tr, "c", lw, rw)
    got = block_list(got)
    assert sorted(got) == sorted(want)
    assert n_pairs == sum(a[1] * a[3] for a in want)
    # blocks of one left entry are adjacent, left entries in row order
    starts = [b[0] for b in got]
    assert starts == sorted(starts)
    return tl, tr, want


@pytest.mark.parametrize("lk", KINDS)
@pytest.mark.parametrize("rk", KINDS)
def test_join_index_matches_oracle(ctx, lk, rk):
    for seed, (nl, nr, domain) in enumerate([(37, 29, 4), (2047, 3001, 50), (20_011, 9_001, 3000),
                                             (50_000, 700, 40)]):
        say("join", lk, rk, seed, nl, nr, domain)
        rng = np.random.default_rng([seed, KINDS.index(lk), KINDS.index(rk), 31])
        L, R = column(rng, lk, nl, domain), column(rng, rk, nr, domain)
        lb, le = sorted(int(x) for x in rng.integers(0, nl + 1, size=2))
        rb, re_ = sorted(int(x) for x in rng.integers(0, nr + 1, size=2))
        check_join(ctx, L, nl, R, nr)
        check_join(ctx, L, nl, R, nr, (lb, le), (rb, re_))


@pytest.mark.parametrize("lk", KINDS)
@pytest.mark.parametrize("rk", KINDS)
def test_join_apply_matches_oracle(ctx, lk, rk):
    """Apply Join Index over the oracle's blocks, each side and each
    encoding of the applied column (an Index column reads 0 off its points)."""
    import torch
    from paper_2506_10092_amd import ccq
    rng = np.random.default_rng([KINDS.index(lk), KINDS.index(rk), 77])
    nl, nr = 6001, 4099
    L, R = column(rng, lk, nl, 60), column(rng, rk, nr, 60)
    blocks = J.join_blocks(J.entries(L, nl, 0, nl), J.entries(R, nr, 0, nr))
    dev = torch.tensor(blocks, dtype=torch.int64, device="cuda").reshape(-1, 4)
    for side, col, n in (("left", L, nl), ("right", R, nr)):
        for k in KINDS:
            other = column(rng, k, n, 1 << 12)
            for name, c in (("joined", col), ("other", other)):
                say("apply", lk, rk, side, k, name, len(blocks))
                t = table(ctx, c, n)
                got = ccq.join_apply(t, "c", dev, side).cpu().numpy()
                want = J.apply(blocks, c, n, side)
                assert np.array_equal(got, want), (side, k, name)


def test_paper_select_example(ctx):
    """Section 8's select example (R.A = [A, B, B], S.B = [B, B, A], S.C =
    [D, E, F] as integers) through both entry points."""
    import json
    import os
    from paper_2506_10092_amd import ccq
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "joins.json")))["select_example"]
    pk = lambda v: {"enc": "bitpacked", "packed": datagen.pack_codes(np.asarray(v, dtype=np.uint32), 8), "w": 8,
                    "base": 0}
    ra, sb, sc = table(ctx, pk(g["R_A"]), 3), table(ctx, pk(g["S_B"]), 3), table(ctx, pk(g["S_C"]), 3)
    blocks, n_pairs = ccq.join_index(ra, "c", sb, "c")
    assert n_pairs == 5
    pr = sorted(J.pairs(block_list(blocks)))
    assert pr == sorted(zip(g["left_index"], g["right_index"]))
    # apply over the blocks in the paper's order
    want_blocks = J.join_blocks(J.entries(pk(g["R_A"]), 3, 0, 3), J.entries(pk(g["S_B"]), 3, 0, 3))
    import torch
    dev = torch.tensor(want_blocks, dtype=torch.int64, device="cuda").reshape(-1, 4)
    assert ccq.join_apply(sc, "c", dev, "right").cpu().tolist() == g["apply_S_C"]


def test_join_edge_cases(ctx):
    from paper_2506_10092_amd import ccq
    rng = np.random.default_rng(5)
    # extreme values, INT64_MIN included (the hash table's empty marker has a slot of its own)
    ext = [I64.min, I64.min + 1, -1, 0, 1, I64.max]
    for lk, rk in (("rle", "index"), ("index", "rle"), ("rle", "rle"), ("index", "index")):
        say("extremes", lk, rk)
        L, R = column(rng, lk, 3000, 0, values=ext), column(rng, rk, 2000, 0, values=ext)
        check_join(ctx, L, 3000, R, 2000)
    # int32 values joined with int64 values
    L = column(rng, "rle", 5000, 30, vtype=np.int32)
    R = column(rng, "index", 4000, 30, vtype=np.int64)
    check_join(ctx, L, 5000, R, 4000)
    # no common value; empty windows; an Index column that lists nothing
    check_join(ctx, column(rng, "rle", 900, 5), 900,
               {"enc": "rle", "values": np.array([7, 8], dtype=np.int64), "run_ends": np.array([10, 50])}, 50)
    L, R = column(rng, "bitpacked", 1000, 8), column(rng, "rle", 1000, 8)
    check_join(ctx, L, 1000, R, 1000, (500, 500), (0, 1000))
    check_join(ctx, L, 1000, R, 1000, (0, 1000), (1000, 1000))
    empty = {"enc": "index", "positions": np.zeros(0, dtype=np.int32), "values": np.zeros(0, dtype=np.int64)}
    check_join(ctx, L, 1000, empty, 1000)
    check_join(ctx, empty, 1000, L, 1000)
    # one value on both sides: every left entry matches every right entry (long chains)
    one = lambda k, n: column(rng, k, n, 1)
    check_join(ctx, one("bitpacked", 700), 700, one("rle", 9000), 9000)
    check_join(ctx, one("index", 1500), 1500, one("index", 800), 800)
    # a bit-packed column of 32-bit codes and a negative base
    codes = rng.integers(0, 1 << 32, size=4000, dtype=np.uint64).astype(np.uint32)
    R = {"enc": "bitpacked", "packed": datagen.pack_codes(codes, 32), "w": 32, "base": -(1 << 31)}
    Lv = codes.astype(np.int64) - (1 << 31)
    L = {"enc": "index", "positions": np.arange(0, 4000, 3, dtype=np.int32), "values": Lv[::3].copy()}
    check_join(ctx, L, 4000, R, 4000)


def test_join_errors(ctx):
    import torch
    from paper_2506_10092_amd import ccq
    rng = np.random.default_rng(9)
    L, R = column(rng, "rle", 1000, 3), column(rng, "bitpacked", 1000, 3)
    tl, tr = table(ctx, L, 1000), table(ctx, R, 1000)
    with pytest.raises(ccq.CcqError) as e:
        ccq.join_index(tl, "c", tr, "c", (0, 1001))
    assert e.value.status == ccq.E_INVALID
    with pytest.raises(ccq.CcqError) as e:
        ccq.join_index(tl, 3, tr, "c")
    assert e.value.status == ccq.E_INVALID
    # too small a block buffer: CCQ_E_CAPACITY with the counts still returned
    L_ = ccq.lib()
    wsb = L_.ccq_join_workspace_bytes(tl.h, 0, 0, 1000, tr.h, 0, 0, 1000)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    buf = torch.empty((1, 4), dtype=torch.int64, device="cuda")
    nb, npairs = ccq.ctypes.c_int64(), ccq.ctypes.c_int64()
    st = L_.ccq_join_index(tl.h, 0, 0, 1000, tr.h, 0, 0, 1000, ccq.ctypes.c_void_p(ws.data_ptr()), wsb,
                           ccq._stream_ptr(None), ccq.ctypes.c_void_p(buf.data_ptr()), 1, ccq.ctypes.byref(nb),
                           ccq.ctypes.byref(npairs))
    want = J.join_blocks(J.entries(L, 1000, 0, 1000), J.entries(R, 1000, 0, 1000))
    assert st == ccq.E_CAPACITY and nb.value == len(want) and npairs.value == sum(a[1] * a[3] for a in want)
    st = L_.ccq_join_index(tl.h, 0, 0, 1000, tr.h, 0, 0, 1000, ccq.ctypes.c_void_p(ws.data_ptr()), wsb - 256,
                           ccq._stream_ptr(None), None, 0, ccq.ctypes.byref(nb), ccq.ctypes.byref(npairs))
    assert st == ccq.E_CAPACITY
    # blocks whose rows leave the table are rejected before anything is written
    for bad in ([[990, 20, 0, 1]], [[-1, 1, 0, 1]], [[0, -2, 0, 1]], [[0, 1, 5, -1]]):
        b = torch.tensor(bad, dtype=torch.int64, device="cuda")
        with pytest.raises(ccq.CcqError) as e:
            ccq.join_apply(tl, "c", b, "left")
        assert e.value.status == ccq.E_INVALID
    with pytest.raises(ccq.CcqError):
        ccq.join_apply(tl, "c", torch.tensor([[0, 1, 0, 1]], dtype=torch.int64, device="cuda"), 2)
    # no blocks: nothing out
    assert ccq.join_apply(tl, "c", torch.zeros((0, 4), dtype=torch.int64, device="cuda"), "left").numel() == 0


def test_join_large(ctx):
    """A million-row bit-packed column joined with a 100k-run RLE column:
    per-left-row block counts and the pair count against numpy's
    value counts, and the applied right values equal the left values."""
    from paper_2506_10092_amd import ccq
    rng = np.random.default_rng(123)
    n, domain = 1 << 20, 1 << 17
    lv = rng.integers(0, domain, size=n)
    L = {"enc": "bitpacked", "packed": datagen.pack_codes(lv.astype(np.uint32), 17), "w": 17, "base": 0}
    R = column(rng, "rle", 2_000_000, domain)
    nr = 2_000_000
    say("join large", n, len(R["values"]))
    tl, tr = table(ctx, L, n), table(ctx, R, nr)
    blocks, n_pairs = ccq.join_index(tl, "c", tr, "c")
    b = blocks.cpu().numpy()
    rv = R["values"].astype(np.int64)
    rlen = np.diff(np.r_[0, R["run_ends"]])
    runs_of = np.bincount(rv, minlength=domain)
    rows_of = np.bincount(rv, weights=rlen, minlength=domain).astype(np.int64)
    assert len(b) == int(runs_of[lv].sum())
    assert n_pairs == int(rows_of[lv].sum())
    assert np.array_equal(np.bincount(b[:, 0], minlength=n), runs_of[lv])
    assert (b[:, 1] == 1).all()
    # the right side's rows of every block hold the left row's value
    got = ccq.join_apply(tr, "c", blocks, "right").cpu().numpy()
    left_rows = np.repeat(b[:, 0], b[:, 3])
    assert np.array_equal(got, lv[left_rows])
