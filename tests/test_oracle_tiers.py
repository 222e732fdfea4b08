"""The C oracle (full-size blocks) against the Python oracle (literal
definitions) and against the stock decoder at full size."""

import bz2
import itertools
import random

import numpy as np
import pytest

from oracle import cref, ref
import workloads as W


def _small_inputs():
    rnd = random.Random(21)
    out = [b"a", b"ab", b"abab", b"aaaa", b"a" * 300, bytes(range(256))]
    for n in [1, 2, 3, 7, 64, 500, 1500]:
        for alpha in [b"ab", b"abc", bytes(range(256))]:
            out.append(bytes(rnd.choice(alpha) for _ in range(n)))
    return out


@pytest.mark.parametrize("x", _small_inputs())
def test_stages_agree(x):
    assert cref.crc32(x) == ref.crc32_bzip2(x)
    r1 = ref.rle1_encode(x)
    assert cref.rle1(x).tobytes() == r1
    sa, last, optr = cref.bwt(r1)
    assert list(sa) == ref.bwt_sa(r1)
    assert (last.tobytes(), optr) == ref.bwt_encode(r1)
    syms, used, nu, mtf = cref.mtf_zrle(last)
    m, u = ref.mtf_encode(last.tobytes())
    assert list(mtf) == m and [i for i in range(256) if used[i]] == u
    assert list(syms) == ref.zrle_encode(m, len(u))
    lens, sel = cref.tables(syms, nu + 2)
    plens, psel = ref.choose_tables(list(syms), nu + 2)
    assert lens.tolist() == plens and sel.tolist() == psel


def test_bwt_agree_brute_force_family():
    for n in range(1, 11):
        for t in itertools.product(b"ab", repeat=n):
            s = bytes(t)
            sa, last, optr = cref.bwt(s)
            assert list(sa) == ref.bwt_sa(s)


def test_huffman_agree():
    rnd = random.Random(31)
    for _ in range(300):
        a = rnd.randrange(3, 259)
        f = [rnd.choice([0, 1, 2, 3, rnd.randrange(10**6)]) for _ in range(a)]
        assert cref.huffman_lengths(f).tolist() == ref.huffman_lengths(f)


@pytest.mark.parametrize("seed", range(6))
def test_streams_agree(seed):
    rnd = random.Random(seed)
    x = bytes(rnd.choice(b"abc ") if rnd.random() < 0.7 else rnd.randrange(256)
              for _ in range(rnd.randrange(1, 2500)))
    offs = sorted(set([0, len(x)] + [rnd.randrange(len(x) + 1) for _ in range(2)]))
    assert cref.compress(x, offs, level=1) == ref.compress(x, level=1, offsets=offs)


def test_check_sa_detects_errors():
    x = np.frombuffer(b"mississippi", np.uint8)
    sa, _, _ = cref.bwt(x)
    assert cref.check_sa(x, sa) == -1
    bad = sa.copy()
    bad[3], bad[4] = bad[4], bad[3]
    assert cref.check_sa(x, bad) == 3
    dup = sa.copy()
    dup[0] = dup[1]
    assert cref.check_sa(x, dup) == x.size
    per = np.frombuffer(b"abcabcabcabc", np.uint8)
    sa, _, _ = cref.bwt(per)
    assert cref.check_sa(per, sa) == -1
    bad = sa.copy()
    bad[0], bad[1] = bad[1], bad[0]  # equal rotations in ascending order
    assert cref.check_sa(per, bad) == 0


@pytest.mark.slow
def test_full_size_blocks_stock_decodes():
    b = W.config2(total=900000 * 3)  # one block of each source, full size
    z = cref.compress(b.data, b.offsets, level=9, threads=3)
    assert bz2.decompress(z) == b.data.tobytes()
    offs = cref.split_blocks(b.data, b.offsets, 900000)
    for k in range(offs.size - 1):
        n1 = cref.rle1(b.data[int(offs[k]):int(offs[k + 1])]).size
        assert n1 <= 900000


@pytest.mark.slow
def test_full_size_sa_property():
    b = W.config2(total=900000 * 3)
    for k in range(3):
        r1 = cref.rle1(b.block(k))
        sa, last, optr = cref.bwt(r1)
        assert cref.check_sa(r1, sa) == -1
        assert sa[optr] == 0
    c = W.config3(nb=3, n_same=1, block=200000)
    for k in range(3):
        blk = c.block(k)
        sa, last, optr = cref.bwt(blk)
        assert cref.check_sa(blk, sa) == -1


def test_stock_limit_is_inclusive():
    """The stock decoder takes a post-RLE1 block of exactly 100000*digit bytes
    and rejects one byte more; this is why the oracle cuts blocks at that
    limit."""
    g = np.random.default_rng(5)
    base = g.integers(0, 256, 100000, dtype=np.uint8)
    for i in range(3, base.size):
        if base[i] == base[i - 1] == base[i - 2] == base[i - 3]:
            base[i] ^= 1
    assert cref.rle1(base).size == 100000
    z = cref.compress(base, level=1)
    assert bz2.decompress(z) == base.tobytes()
    # the same block plus one byte: 100001 post-RLE1 bytes in a "BZh1" stream,
    # written by hand from the oracle's stages (no split)
    x = base.tobytes() + b"\x07"
    r1 = cref.rle1(x)
    assert r1.size == 100001
    sa, last, optr = cref.bwt(r1)
    syms, used, nu, _ = cref.mtf_zrle(last)
    body, nbits, _, _ = cref.body(syms, used)
    w = ref.BitWriter()
    for c in b"BZh1":
        w.put(c, 8)
    crc = cref.crc32(x)
    w.put(ref.BLOCK_MAGIC, 48)
    w.put(crc, 32)
    w.put(0, 1)
    w.put(optr, 24)
    for i in range(nbits):
        w.bits.append((body[i >> 3] >> (7 - (i & 7))) & 1)
    w.put(ref.EOS_MAGIC, 48)
    w.put(ref.combine_stream_crc([crc]), 32)
    z = w.tobytes()
    with pytest.raises(OSError):
        bz2.decompress(z)  # well-formed, but over the stock limit
    assert bz2.decompress(cref.compress(x, level=1)) == x  # the split stream decodes
    # and the same hand assembly at exactly the limit is accepted
    r1 = cref.rle1(base)
    sa, last, optr = cref.bwt(r1)
    syms, used, nu, _ = cref.mtf_zrle(last)
    body, nbits, _, _ = cref.body(syms, used)
    w = ref.BitWriter()
    for c in b"BZh1":
        w.put(c, 8)
    crc = cref.crc32(base)
    w.put(ref.BLOCK_MAGIC, 48)
    w.put(crc, 32)
    w.put(0, 1)
    w.put(optr, 24)
    for i in range(nbits):
        w.bits.append((body[i >> 3] >> (7 - (i & 7))) & 1)
    w.put(ref.EOS_MAGIC, 48)
    w.put(ref.combine_stream_crc([crc]), 32)
    assert w.tobytes() == cref.compress(base, level=1)
