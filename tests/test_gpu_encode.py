"""GPU parity of the encoders (ccq_plain_to_rle, ccq_plain_to_rle_index,
ccq_plain_to_plain_index) and of the encoding choice (ccq_encode_choose)
against the CPU oracle (oracle/encode.py), array by array, bit for bit."""
import sys

import numpy as np
import pytest

import datagen
from oracle import encode as E
from oracle import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_10092_amd import ccq
    assert torch.cuda.is_available()
    return ccq.Context(0)


def column(kind, n, dtype, seed=1):
    rng = np.random.default_rng([seed, n, KINDS.index(kind)])
    if kind == "runs":
        x = np.repeat(rng.integers(-1000, 1000, size=n // 7 + 1), rng.integers(1, 14, size=n // 7 + 1))[:n]
        if len(x) < n:
            x = np.concatenate([x, np.full(n - len(x), 5)])
    elif kind == "distinct":
        x = rng.permutation(n) - n // 3
    elif kind == "mixed":
        x = np.where(rng.random(n) < 0.2, rng.integers(0, 1 << 16, size=n), np.arange(n) // 300)
    elif kind == "extremes":
        x = rng.choice(np.array([np.iinfo(np.int64).min, -3, 0, 9, np.iinfo(np.int64).max]), size=n)
    else:
        x = np.full(n, -17)
    if dtype == np.int32 and kind == "extremes":
        x = np.clip(x, np.iinfo(np.int32).min, np.iinfo(np.int32).max)
    return np.asarray(x).astype(dtype)


def to_np(t):
    return t.cpu().numpy()


SIZES = [1, 2, 31, 4095, 4096, 4097, 100_017, 3_000_011]
KINDS = ["runs", "distinct", "mixed", "extremes", "constant"]


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("kind", KINDS)
def test_encoders_match_oracle(ctx, kind, dtype):
    import torch
    from paper_2506_10092_amd import ccq
    for n in SIZES:
        x = column(kind, n, dtype)
        say("encode case:", kind, np.dtype(dtype).name, n)
        d = torch.from_numpy(x).cuda()
        rle = ccq.plain_to_rle(ctx, d)
        vals, ends = E.plain_to_rle(x)
        assert np.array_equal(to_np(rle["values"]), vals) and np.array_equal(to_np(rle["run_ends"]), ends)
        ri = ccq.plain_to_rle_index(ctx, d)
        (rv, rs, re_), (ip, iv) = E.plain_to_rle_index(x)
        assert np.array_equal(to_np(ri["runs"]["values"]), rv)
        assert np.array_equal(to_np(ri["runs"]["starts"]), rs)
        assert np.array_equal(to_np(ri["runs"]["ends"]), re_)
        assert np.array_equal(to_np(ri["points"]["positions"]), ip)
        assert np.array_equal(to_np(ri["points"]["values"]), iv)
        c = ccq.encode_choose(ctx, d)
        assert c == E.choose(x), (c, E.choose(x))
        xs = np.sort(x.astype(np.int64))
        for w, base in ((1, int(xs[0])), (7, int(xs[n // 2]) - 3), (20, int(xs[n // 20])), (32, int(xs[0]))):
            pi = ccq.plain_to_plain_index(ctx, d, w, base)
            packed, (pos, pv) = E.plain_to_plain_index(x, w, base)
            got = to_np(pi["column"]["packed"]).view(np.uint32)
            assert np.array_equal(got, packed), (w, base)
            assert np.array_equal(to_np(pi["points"]["positions"]), pos)
            assert np.array_equal(to_np(pi["points"]["values"]), pv)


def test_choose_branches_on_gpu(ctx):
    """Inputs built to take each branch of the choice (as in the oracle's
    pins), chosen identically on the GPU."""
    import torch
    from paper_2506_10092_amd import ccq
    rng = np.random.default_rng(3)
    n = 1_200_000
    narrow = rng.integers(0, 1 << 16, size=n).astype(np.int64)
    narrow[rng.choice(n, size=n // 50, replace=False)] = 1 << 40
    blocks = n // 4200
    mixed = np.concatenate([np.concatenate([np.full(4000, b), -1 - np.arange(200) - 200 * b])
                            for b in range(blocks)]).astype(np.int32)
    cols = {"plain": np.arange(1000, dtype=np.int32),
            "rle": np.repeat(rng.integers(0, 100, size=n // 100), 100).astype(np.int32),
            "rle+index": mixed, "plain+index": narrow,
            "plain20": rng.integers(0, 1 << 20, size=n).astype(np.int32),
            "wide": rng.integers(-(1 << 62), 1 << 62, size=n).astype(np.int64)}
    for name, x in cols.items():
        say("choose case:", name)
        got = ccq.encode_choose(ctx, torch.from_numpy(x).cuda())
        exp = E.choose(x)
        assert got == exp
        assert got["choice"] == {"plain20": "plain", "wide": "rle"}.get(name, name)


def test_rle_encoder_at_1e8_rows_and_query(ctx):
    """A 1e8-row column of lognormal runs (mean 64) encoded on the GPU equals
    the oracle's runs; a query over the GPU-encoded column equals the
    oracle's answer over the oracle-encoded one."""
    import torch
    from paper_2506_10092_amd import ccq
    n = 100_000_000
    src = datagen.rle_column(9, 7000, n, "lognormal", 64, 0, 1 << 16)
    x = E.decode_rle(src["values"], src["run_ends"])
    say("encode 1e8: runs in the source", len(src["values"]))
    d = torch.from_numpy(x).cuda()
    rle = ccq.plain_to_rle(ctx, d)
    vals, ends = E.plain_to_rle(x)
    assert np.array_equal(to_np(rle["run_ends"]), ends) and np.array_equal(to_np(rle["values"]), vals)
    del d
    host = {"n_rows": n, "columns": {"a": {"enc": "rle", "values": vals, "run_ends": ends}}}
    q = {"preds": [("a", "range", 1000, 40000)], "keys": [("a", 12, 16)], "aggs": [("sum", "a"), ("count",)],
         "window": (17, n - 5)}
    tb = ccq.Table(ctx, n, {"a": rle})
    got = ccq.Plan(tb, q).run()
    exp = oracle.run(host, q)
    assert got["status"] == 0
    for k in ("keys", "counts", "aggs"):
        assert got[k] == exp[k], k


def test_empty_and_capacity(ctx):
    import torch
    from paper_2506_10092_amd import ccq
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    assert to_np(ccq.plain_to_rle(ctx, e)["run_ends"]).size == 0
    assert ccq.encode_choose(ctx, e)["n_rows"] == 0
    x = torch.arange(10, dtype=torch.int64, device="cuda")
    ws = torch.empty(int(ccq.lib().ccq_encode_workspace_bytes(10)), dtype=torch.uint8, device="cuda")
    import ctypes
    n = ctypes.c_int64()
    st = ccq.lib().ccq_plain_to_rle(ctx.h, ctypes.c_void_p(x.data_ptr()), ccq.I64, 10,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), None, None, None, 3,
                                    ctypes.byref(n))
    assert st == ccq.E_CAPACITY and n.value == 10
