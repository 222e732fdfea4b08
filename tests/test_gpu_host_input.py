"""compress_host: input in host memory, uploads, kernels and downloads
overlapped chunk by chunk; each chunk one bzip2 stream.  Parity: the output
is the oracle's stream of every chunk, one after another."""

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


def _expected(data: np.ndarray, level: int, block: int, per_chunk: int) -> bytes:
    cb = block * per_chunk
    if data.size == 0:
        return cref.compress(data, [0], level)
    out = []
    for lo in range(0, data.size, cb):
        chunk = data[lo:lo + cb]
        offs = list(range(0, chunk.size, block)) + [chunk.size]
        out.append(cref.compress(chunk, offs, level))
    return b"".join(out)


def _mixed(total: int, seed: int) -> np.ndarray:
    b = W.config2(total=total, block=150_000, seed=seed)
    return b.data


@pytest.mark.parametrize("level,per_chunk", [(1, 2), (2, 3)])
def test_pageable_input_chunks_equal_oracle_streams(bz, level, per_chunk):
    data = _mixed(1_234_567, seed=21 + level)
    block = 100_000 * level
    _say(f"compress_host pageable: {data.size} B, level {level}, {per_chunk} blocks per chunk")
    got = bz.compress_host(data, level=level, chunk_bytes=per_chunk * block)
    want = _expected(data, level, block, per_chunk)
    assert got.tobytes() == want
    assert bz2.decompress(got.tobytes()) == data.tobytes()


def test_pinned_input_and_output(bz):
    import torch
    data = _mixed(2_000_003, seed=31)
    pin = torch.empty(data.size, dtype=torch.uint8, pin_memory=True)
    pin.numpy()[:] = data
    out = torch.empty(data.size + (1 << 20), dtype=torch.uint8, pin_memory=True)
    _say(f"compress_host pinned: {data.size} B, level 9, 1 block per chunk")
    got = bz.compress_host(pin, level=9, block_bytes=300_000, chunk_bytes=300_000, out=out)
    want = _expected(data, 9, 300_000, 1)
    assert got.tobytes() == want
    assert bz2.decompress(got.tobytes()) == data.tobytes()


def test_empty_and_single_short_chunk(bz):
    _say("compress_host empty and 777-byte inputs")
    got = bz.compress_host(np.zeros(0, np.uint8), level=9)
    assert got.tobytes() == cref.compress(np.zeros(0, np.uint8), [0], 9)
    small = _mixed(777, seed=41)
    got = bz.compress_host(small.tobytes(), level=3)
    assert got.tobytes() == _expected(small, 3, 300_000, 128)


def test_output_too_small_is_reported(bz):
    import torch
    data = _mixed(400_000, seed=51)
    out = torch.empty(100, dtype=torch.uint8)
    _say("compress_host capacity error")
    with pytest.raises(bz.BzgError) as ei:
        bz.compress_host(data, level=1, chunk_bytes=100_000, out=out)
    assert ei.value.code == bz.native.BZG_ECAPACITY
    # the context stays usable
    got = bz.compress_host(data, level=1, chunk_bytes=100_000)
    assert got.tobytes() == _expected(data, 1, 100_000, 1)
