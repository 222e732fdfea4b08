"""GPU decompression: streams from the oracle's encoder and from stock
bzip2 decode to the bytes they were made from (the plain definition of a
decoder's result; the oracle's own decoder is pinned to it on the CPU)."""

import bz2
import random
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


def _dev(b):
    import torch
    return torch.from_numpy(np.frombuffer(bytes(b), np.uint8).copy()).cuda()


def _roundtrip(bz, stream: bytes, want: bytes, name: str):
    _say(f"decompress {name}: {len(stream)} B -> {len(want)} B")
    got = bz.decompress(_dev(stream)).cpu().numpy().tobytes()
    assert len(got) == len(want), f"{name}: {len(got)} bytes, want {len(want)}"
    if got != want:
        first = next(i for i in range(len(want)) if got[i] != want[i])
        raise AssertionError(f"{name}: output differs at byte {first}")


def test_small_cases_from_the_oracle(bz):
    rnd = random.Random(7)
    cases = [b"a", b"ab", b"banana", b"aaaa", b"aaaaa", b"a" * 300, b"abab" * 100, bytes(range(256)) * 5,
             b"\x05" * 1000 + b"\x05\x05\x05\x05\x05x" * 77, bytes(rnd.randrange(256) for _ in range(5000)),
             bytes(rnd.randrange(3) for _ in range(20000))]
    for i, x in enumerate(cases):
        for level in (1, 9):
            _roundtrip(bz, cref.compress(np.frombuffer(x, np.uint8), None, level), x, f"case {i} level {level}")


def test_mixed_blocks_from_the_oracle(bz):
    b = W.config2(total=3 * 900_000 + 12_345, block=450_000, seed=71)
    z = cref.compress(b.data, [int(o) for o in b.offsets], 9, threads=16)
    _roundtrip(bz, z, b.data.tobytes(), "uniform/text/sparse blocks, level 9")
    z = cref.compress(b.data, None, 1, threads=16)
    _roundtrip(bz, z, b.data.tobytes(), "same bytes, level 1 (many blocks)")


def test_periodic_and_all_same_blocks(bz):
    b = W.config3(nb=6, block=200_000, seed=72, n_same=2)
    z = cref.compress(b.data, [int(o) for o in b.offsets], 9, threads=16)
    _roundtrip(bz, z, b.data.tobytes(), "periodic and all-same blocks")


def test_stock_bzip2_streams(bz):
    b = W.config2(total=1_500_000, block=300_000, seed=73)
    data = b.data.tobytes()
    for level in (1, 5, 9):
        _roundtrip(bz, bz2.compress(data, level), data, f"stock bzip2 level {level}")
    _roundtrip(bz, bz2.compress(b"", 9), b"", "stock empty stream")
    _roundtrip(bz, bz2.compress(b"x", 9), b"x", "stock one byte")


def test_several_streams_and_own_streams(bz):
    import torch
    a = W.config2(total=700_000, block=100_000, seed=74).data
    c = W.config4(nb=30, lo=100, hi=200_000, seed=75)
    za = bz.compress_host(a, level=2, chunk_bytes=200_000).tobytes()  # four streams
    zc = bz.compress(torch.from_numpy(c.data).cuda(), c.offsets, level=9).cpu().numpy().tobytes()
    _roundtrip(bz, za + zc + bz2.compress(b"tail", 1), a.tobytes() + c.data.tobytes() + b"tail",
               "GPU streams and a stock one, concatenated")


def test_capacity_retry_and_bad_input(bz):
    import torch
    data = W.config2(total=400_000, block=100_000, seed=76).data.tobytes()
    z = cref.compress(np.frombuffer(data, np.uint8), None, 1)
    _say("decompress with a small first output buffer")
    got = bz.decompress(_dev(z), out_cap=1000).cpu().numpy().tobytes()
    assert got == data
    _say("decompress input with no bzip2 header")
    with pytest.raises(bz.BzgError) as ei:
        bz.decompress(_dev(b"not a bzip2 stream at all" * 4))
    assert ei.value.code == bz.native.BZG_EDATA
    # a block CRC changed: the data decode normally, the check fails
    bad = bytearray(z)
    bad[10] ^= 0x40  # inside the first block's stored CRC (bytes 10..13)
    _say("decompress with a wrong block CRC")
    with pytest.raises(bz.BzgError) as ei:
        bz.decompress(_dev(bytes(bad)))
    assert ei.value.code == bz.native.BZG_EDATA
    # the context still works
    assert bz.decompress(_dev(z)).cpu().numpy().tobytes() == data


def _straddles(syms, step):
    """Whether some run of RUNA/RUNB digits (symbols 0 and 1) crosses a
    multiple of `step` in the symbol sequence."""
    d = np.asarray(syms) <= 1
    k = np.arange(step, d.size, step)
    return bool(np.any(d[k] & d[k - 1]))


def test_runs_across_chunk_and_step_boundaries(bz):
    # large sparse blocks: thousands of zero runs among the symbols, so runs
    # cross the decoder's 4096-symbol chunks and its 64-symbol steps (pinned
    # below on the oracle's own symbol sequence of each block)
    data = np.concatenate(W.source_blocks("sparse", [900_000, 700_001], 91)).astype(np.uint8)
    offs = [0, 900_000, data.size]
    for lo, hi in zip(offs[:-1], offs[1:]):
        _, last, _ = cref.bwt(cref.rle1(data[lo:hi]))
        syms = cref.mtf_zrle(last)[0]
        assert _straddles(syms, 4096) and _straddles(syms, 64), "the block should exercise run carries"
    z = cref.compress(data, offs, 9, threads=16)
    _roundtrip(bz, z, data.tobytes(), "sparse 900 KB blocks with runs across chunks")


def test_long_and_short_blocks_decoded_as_two_classes(bz):
    # 96 blocks of log-uniform length 2 KB .. 300 KB: the long ones (a
    # quarter of the longest block's bits or more) are decoded on a second
    # stream, the rest on the call's, and every block's bytes land at its
    # place in the output
    b = W.config4(nb=96, lo=2000, hi=300_000, seed=91)
    z = cref.compress(b.data, [int(o) for o in b.offsets], 9, threads=16)
    _roundtrip(bz, z, b.data.tobytes(), "96 blocks of 2 KB .. 300 KB in two length classes")
    # the same blocks as 96 streams of one block each, concatenated
    parts = [cref.compress(b.data[int(b.offsets[k]):int(b.offsets[k + 1])], None, 9) for k in range(96)]
    _roundtrip(bz, b"".join(bytes(p) for p in parts), b.data.tobytes(), "96 one-block streams")
