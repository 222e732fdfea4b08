"""Precomputed Huffman tables on the GPU (Sec. 4): the table set derived
from a sample and the streams coded with it, bit for bit against the
oracle."""

import bz2
import sys

import numpy as np
import pytest

from oracle import cref
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bz():
    import torch
    import paper_1109_2348_amd as bz
    assert torch.cuda.is_available()
    return bz


@pytest.fixture(scope="module")
def ctx(bz):
    c = bz.Context()
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).cuda()


def _data(total, block, seed):
    b = W.config2(total=total, block=block, seed=seed)
    return b.data, [int(o) for o in b.offsets]


def _hand_tables():
    t0 = [1, 2] + [10] * 256
    t1 = [8] * 254 + [9] * 4
    return np.array([t0, t1], np.uint8)


def test_sample_tables_equal_oracle(bz, ctx):
    sample, so = _data(300_000, 50_000, seed=61)
    _say(f"tables from a {sample.size}-byte sample in {len(so) - 1} blocks")
    ctx.set_fixed_tables(None)
    got = bz.fixed_tables_from_sample(_dev(sample), so, ctx=ctx)
    want = cref.tables_from_sample([sample[so[k]:so[k + 1]] for k in range(len(so) - 1)])
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_sample_cut_to_one_block_of_symbols(bz, ctx):
    sample, so = _data(1_200_000, 300_000, seed=62)
    _say("tables from a sample above 900000 symbols")
    ctx.set_fixed_tables(None)
    got = bz.fixed_tables_from_sample(_dev(sample), so, ctx=ctx)
    want = cref.tables_from_sample([sample[so[k]:so[k + 1]] for k in range(len(so) - 1)])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("level", [1, 9])
def test_compress_with_sample_tables_equals_oracle(bz, ctx, level):
    sample, so = _data(200_000, 40_000, seed=63)
    fixed = cref.tables_from_sample([sample[so[k]:so[k + 1]] for k in range(len(so) - 1)])
    data, offs = _data(2_500_000, 250_000, seed=64)
    offs = [0, 5, 5, 1000, 70_000] + [o for o in offs if o > 70_000]  # tiny and empty blocks too
    _say(f"compress with sample tables, level {level}, {len(offs) - 1} blocks")
    ctx.set_fixed_tables(fixed)
    try:
        z = bz.Compressor(ctx=ctx)(_dev(data), offs, level=level).cpu().numpy().tobytes()
    finally:
        ctx.set_fixed_tables(None)
    assert z == cref.compress(data, offs, level, fixed=fixed)
    assert bz2.decompress(z) == data.tobytes()


def test_hand_tables_and_return_to_built_tables(bz, ctx):
    data, offs = _data(600_000, 100_000, seed=65)
    f = _hand_tables()
    _say("compress with two hand-made tables, then without")
    ctx.set_fixed_tables(f)
    z = bz.Compressor(ctx=ctx)(_dev(data), offs, level=1).cpu().numpy().tobytes()
    ctx.set_fixed_tables(None)
    assert z == cref.compress(data, offs, 1, fixed=f)
    z2 = bz.Compressor(ctx=ctx)(_dev(data), offs, level=1).cpu().numpy().tobytes()
    assert z2 == cref.compress(data, offs, 1)


def test_batch_with_fixed_tables(bz, ctx):
    data, offs = _data(900_000, 90_000, seed=66)
    f = _hand_tables()
    req = [0, 3, 3, 7, 10]
    _say("compress_batch with hand-made tables, 4 requests")
    ctx.set_fixed_tables(f)
    try:
        outs = bz.native.BatchCompressor(ctx=ctx)(_dev(data), offs, req, 9)
        outs = [o.cpu().numpy().tobytes() for o in outs]
    finally:
        ctx.set_fixed_tables(None)
    for r in range(len(req) - 1):
        a, e = offs[req[r]], offs[req[r + 1]]
        sub = [o - a for o in offs[req[r]:req[r + 1] + 1]]
        assert outs[r] == cref.compress(data[a:e], sub, 9, fixed=f), f"request {r}"


def test_bad_tables_rejected(bz, ctx):
    f = _hand_tables()
    bad = [f[:1],                                            # one table
           np.concatenate([f] * 4)[:7],                      # seven tables
           np.where(np.arange(258) == 3, 0, f).astype(np.uint8),   # a zero length
           np.where(np.arange(258) == 3, 18, f).astype(np.uint8),  # longer than 17
           np.array([[1] * 258, [8] * 258], np.uint8)]       # Kraft sum above 1
    for b in bad:
        with pytest.raises(bz.BzgError) as ei:
            ctx.set_fixed_tables(b)
        assert ei.value.code == bz.native.BZG_EINVAL
