"""Parity of the HIP path (through the C ABI) with the CPU oracle: every
output is integer and must match bit for bit."""

import bz2
import itertools
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).cuda()


def _concat(blocks):
    offs = np.zeros(len(blocks) + 1, np.uint64)
    offs[1:] = np.cumsum([len(b) for b in blocks])
    data = np.concatenate([np.frombuffer(bytes(b), np.uint8) if not isinstance(b, np.ndarray) else b
                           for b in blocks]) if blocks else np.zeros(0, np.uint8)
    return data.astype(np.uint8), offs


def _check_bwt(bz, blocks, name, full_oracle=True):
    data, offs = _concat(blocks)
    _say(f"bwt {name}: {len(blocks)} blocks, {data.size} bytes")
    L, prim, sa = bz.bwt(_dev(data), offs, want_sa=True)
    L = L.cpu().numpy()
    prim = prim.cpu().numpy()
    sa = sa.cpu().numpy().view(np.uint32)
    for k, blk in enumerate(blocks):
        a, b = int(offs[k]), int(offs[k + 1])
        if full_oracle:
            rsa, rL, ro = cref.bwt(blk)
            assert np.array_equal(sa[a:b], rsa), f"{name} block {k}: SA differs"
            assert np.array_equal(L[a:b], rL), f"{name} block {k}: L differs"
            assert int(prim[k]) == ro, f"{name} block {k}: primary {prim[k]} != {ro}"
        else:
            blk = np.asarray(blk, np.uint8)
            assert cref.check_sa(blk, sa[a:b]) == -1, f"{name} block {k}: SA not sorted"
            n = b - a
            assert np.array_equal(L[a:b], blk[(sa[a:b].astype(np.int64) - 1) % n])
            assert int(sa[a + int(prim[k])]) == 0


def test_bwt_brute_force_families(bz):
    blocks = []
    for n in range(1, 9):
        blocks += [bytes(t) for t in itertools.product(b"ab", repeat=n)]
    for n in range(1, 6):
        blocks += [bytes(t) for t in itertools.product(b"abc", repeat=n)]
    _check_bwt(bz, blocks, "all strings over {a,b} <= 8 and {a,b,c} <= 5")


def test_bwt_random_sizes(bz):
    rnd = random.Random(1)
    blocks = []
    for n in [1, 2, 3, 4, 5, 63, 64, 65, 4095, 4096, 4097, 2047, 2048, 2049, 10000, 33333]:
        alpha = rnd.choice([b"ab", b"abcd", bytes(range(256))])
        blocks.append(bytes(rnd.choice(alpha) for _ in range(n)))
    _check_bwt(bz, blocks, "random sizes across tile edges")


def test_bwt_periodic_and_same(bz):
    blocks = [b"a" * 5000, b"ab" * 3000, b"abc" * 2000 + b"ab", b"xyzxa" * 1400, b"\x00" * 70000,
              (b"q" * 300 + b"r") * 40]
    c = W.config3(nb=6, n_same=2, block=20000, seed=31)
    blocks += [c.block(k) for k in range(c.n_blocks)]
    _check_bwt(bz, blocks, "periodic / all-same / flipped-periodic")


def test_bwt_text_blocks(bz):
    b = W.config2(total=3 * 150000, block=150000, seed=7)
    _check_bwt(bz, [b.block(k) for k in range(b.n_blocks)], "uniform/text/sparse 150000-byte blocks")


def test_bwt_max_block(bz):
    g = np.random.default_rng(3)
    blk = g.integers(0, 4, size=1 << 21, dtype=np.uint8)
    _check_bwt(bz, [blk], "one block of 2^21 bytes", full_oracle=False)


def test_bwt_rejects_bad_blocks(bz):
    x = _dev(np.zeros(10, np.uint8))
    with pytest.raises(bz.BzgError):
        bz.bwt(x, [0, 5, 5, 10])  # empty block
    with pytest.raises(bz.BzgError):
        bz.bwt(_dev(np.zeros((1 << 21) + 1, np.uint8)), [0, (1 << 21) + 1])


def _check_mtf(bz, Ls, name):
    data, offs = _concat(Ls)
    _say(f"mtf {name}: {len(Ls)} blocks, {data.size} bytes")
    syms, nsyms, inuse = bz.mtf(_dev(data), offs)
    syms = syms.cpu().numpy().view(np.uint16)
    nsyms = nsyms.cpu().numpy()
    inuse = inuse.cpu().numpy()
    for k, Lk in enumerate(Ls):
        rs, used, nu, _ = cref.mtf_zrle(Lk)
        base = int(offs[k]) + k
        assert int(nsyms[k]) == rs.size, f"{name} block {k}: nsyms {nsyms[k]} != {rs.size}"
        assert np.array_equal(syms[base:base + rs.size], rs), f"{name} block {k}: symbols differ"
        bits = np.unpackbits(inuse[32 * k:32 * k + 32], bitorder="little")
        assert np.array_equal(bits, used), f"{name} block {k}: in-use map differs"


def test_mtf_random(bz):
    rnd = random.Random(2)
    Ls = []
    for n in [1, 2, 3, 64, 100, 8191, 8192, 8193, 20000, 50001]:
        alpha = rnd.choice([b"a", b"ab", b"abc", bytes(range(256)), bytes(range(0, 256, 3))])
        p0 = rnd.random()
        s = bytearray()
        for _ in range(n):
            s.append(s[-1] if s and rnd.random() < p0 else rnd.choice(alpha))
        Ls.append(bytes(s))
    _check_mtf(bz, Ls, "random blocks with runs")


def test_mtf_bwt_columns(bz):
    b = W.config2(total=4 * 100000, block=100000, seed=11)
    Ls = []
    for k in range(b.n_blocks):
        _, L, _ = cref.bwt(cref.rle1(b.block(k)))
        Ls.append(L)
    Ls.append(np.zeros(30000, np.uint8))  # one long zero run across chunks
    _check_mtf(bz, Ls, "BWT columns of uniform/text/sparse")


def test_mtf_many_blocks_full_alphabet(bz):
    # enough blocks and rows for 4096-row chunks; every byte in use in the
    # first block (the symbol counts of all blocks are written by the stage)
    g = np.random.default_rng(41)
    Ls = []
    for k in range(24):
        n = int(g.integers(20_000, 200_000))
        runs = g.geometric(0.3 if k % 3 else 0.02, size=n)
        vals = g.integers(0, 256 if k % 2 == 0 else 27, size=n).astype(np.uint8)
        Ls.append(np.repeat(vals, runs)[:n])
    _check_mtf(bz, Ls, "24 blocks with runs, 4096-row chunks")


def _check_huff(bz, sym_lists, used_list, name):
    import torch
    _say(f"huffman {name}: {len(sym_lists)} blocks")
    nb = len(sym_lists)
    so = np.zeros(nb + 1, np.uint64)
    so[1:] = np.cumsum([s.size for s in sym_lists])
    syms = torch.from_numpy(np.concatenate(sym_lists).astype(np.uint16).view(np.int16)).cuda()
    nsyms = torch.tensor([s.size for s in sym_lists], dtype=torch.int32).cuda()
    inuse = torch.from_numpy(np.concatenate([np.packbits(u.astype(np.uint8), bitorder="little")
                                             for u in used_list])).cuda()
    out, oo, nbits, tabs = bz.huffman(syms, nsyms, inuse, so, want_tables=True)
    out = out.cpu().numpy()
    nbits = nbits.cpu().numpy()
    tabs = tabs.cpu().numpy()
    for k in range(nb):
        ref, rbits, rlens, rsel = cref.body(sym_lists[k], used_list[k])
        assert int(nbits[k]) == rbits, f"{name} block {k}: {nbits[k]} bits != {rbits}"
        g = int(tabs[1568 * k])
        assert g == rlens.shape[0]
        a = rlens.shape[1]
        for t in range(g):
            got = tabs[1568 * k + 16 + 258 * t:1568 * k + 16 + 258 * t + a]
            assert np.array_equal(got, rlens[t]), f"{name} block {k}: table {t} lengths differ"
        body = out[int(oo[k]):int(oo[k]) + (rbits + 7) // 8].tobytes()
        assert body == ref, f"{name} block {k}: body bits differ"


def test_huffman_from_oracle_symbols(bz):
    b = W.config2(total=6 * 60000, block=60000, seed=13)
    sl, ul = [], []
    for k in range(b.n_blocks):
        _, L, _ = cref.bwt(cref.rle1(b.block(k)))
        s, used, _, _ = cref.mtf_zrle(L)
        sl.append(s)
        ul.append(used)
    for n in [1, 2, 3, 49, 50, 51, 199, 200, 599, 600, 1199, 2399, 2400]:  # table-count edges
        rnd = np.random.default_rng(n)
        nu = int(rnd.integers(1, 40))
        s = rnd.integers(0, nu + 1, size=n - 1).astype(np.uint16)
        sl.append(np.concatenate([s, [nu + 1]]).astype(np.uint16))
        used = np.zeros(256, np.uint8)
        used[rnd.choice(256, size=nu, replace=False)] = 1
        ul.append(used)
    _check_huff(bz, sl, ul, "oracle symbol streams + table-count edges")


def _spaced_stream(counts):
    """Symbols 1..k with the given counts, each symbol's occurrences evenly
    spaced over the stream (so every 50-symbol group sees the same mix and
    the refinement keeps one table for almost all of them), then EOB."""
    n = sum(counts)
    keys = np.concatenate([(np.arange(c) + 0.5) * n / c + v * 1e-6 for v, c in enumerate(counts)])
    vals = np.concatenate([np.full(c, v + 1, np.uint16) for v, c in enumerate(counts)])
    s = vals[np.argsort(keys, kind="stable")]
    return np.concatenate([s, [len(counts) + 1]]).astype(np.uint16)


def _halvings(counts):
    """Rescale steps the length limit takes for these table counts."""
    from oracle import ref
    w = [max(int(x), 1) for x in counts]
    k = 0
    while max(ref.huffman_lengths(w, max_len=1 << 30)) > 17:
        w = [1 + x // 2 for x in w]
        k += 1
    return k


def test_huffman_length_limit_rescale(bz):
    """Streams whose final tables need the 17-bit rescale once, twice and
    three times (Sec. 3.4): the GPU's tables, bit counts and bodies equal
    the oracle's."""
    fib = [1, 1]
    while len(fib) < 26:
        fib.append(fib[-1] + fib[-2])
    cases = [("fibonacci", fib[1:24], 1), ("powers of 2 to 2^18", [2 ** k for k in range(18, -1, -1)], 2),
             ("powers of 2 to 2^19", [2 ** k for k in range(19, -1, -1)], 3)]
    sl, ul = [], []
    for name, counts, want in cases:
        s = _spaced_stream(counts)
        nu = len(counts)
        used = np.zeros(256, np.uint8)
        used[10:10 + nu] = 1
        _, _, rlens, rsel = cref.body(s, used)
        got = max(_halvings(np.bincount(s[np.repeat(rsel == t, 50)[:s.size]], minlength=nu + 2))
                  for t in range(rlens.shape[0]))
        assert got >= want, f"{name}: final tables need {got} rescale steps, wanted {want}"
        sl.append(s)
        ul.append(used)
    _check_huff(bz, sl, ul, "length-limit rescale (1, 2, 3 halvings)")


def _check_compress(bz, data, offs, level, name):
    _say(f"compress {name}: {data.size} bytes, level {level}")
    z = bz.compress(_dev(data), offs, level=level).cpu().numpy().tobytes()
    ref = cref.compress(data, offs, level=level, threads=16)
    if z != ref:
        n = min(len(z), len(ref))
        first = next((i for i in range(n) if z[i] != ref[i]), n)
        raise AssertionError(f"{name}: stream differs at byte {first} (gpu {len(z)} B, oracle {len(ref)} B)")
    return z


def test_compress_small_cases(bz):
    rnd = random.Random(5)
    cases = [b"", b"a", b"ab", b"banana", b"aaaa", b"aaaaa", b"a" * 300, b"abab" * 100,
             bytes(range(256)) * 5, bytes(rnd.randrange(256) for _ in range(5000))]
    for i, x in enumerate(cases):
        data = np.frombuffer(x, np.uint8)
        offs = [0, len(x)] if x else [0]
        z = _check_compress(bz, data, offs, 9, f"small case {i}")
        assert bz2.decompress(z) == x


def test_compress_runs_across_tiles(bz):
    """RLE1 runs that open, close or cross a piece boundary (every 255 bytes
    of a run) at the edge of a 4096-byte input tile, including pieces whose
    count byte belongs to the previous tile's output."""
    rnd = np.random.default_rng(23)
    parts, offs = [], [0]
    for s in list(range(0, 9)) + list(range(249, 262)):
        for L in (1, 4, 5, 7, 255, 256, 259, 260, 510, 4099):
            fill = rnd.integers(0, 255, 4096 - s, dtype=np.uint8)  # never 255
            tail = rnd.integers(0, 255, 97, dtype=np.uint8)
            blk = np.concatenate([fill, np.full(L, 255, np.uint8), tail])
            parts.append(blk)
            offs.append(offs[-1] + blk.size)
    data = np.concatenate(parts)
    z = _check_compress(bz, data, offs, 9, f"{len(parts)} blocks with runs at tile edges")
    assert bz2.decompress(z) == data.tobytes()


def test_compress_config1(bz):
    b = W.config1()
    z = _check_compress(bz, b.data, b.offsets, 1, "single 100000-byte block, order-2 Markov")
    assert bz2.decompress(z) == b.data.tobytes()


def test_compress_mixed_blocks(bz):
    b = W.config2(total=9 * 100000 + 12345, block=100000, seed=17)
    z = _check_compress(bz, b.data, b.offsets, 1, "10 blocks uniform/text/sparse, level 1 (cuts)")
    assert bz2.decompress(z) == b.data.tobytes()


def test_compress_uneven_blocks(bz):
    b = W.config4(nb=40, lo=10, hi=150000, seed=19)
    z = _check_compress(bz, b.data, b.offsets, 2, "40 uneven blocks")
    assert bz2.decompress(z) == b.data.tobytes()


def test_compress_one_block_of_many_pieces(bz):
    # one caller block cut by the RLE1 limit into over 80 pieces (level 1:
    # 100000 bytes after RLE1 each), uniform bytes then runs, against the
    # oracle's unbounded cut
    d = np.concatenate(W.source_blocks("uniform", [7_600_000], 31) + W.source_blocks("sparse", [1_400_001], 32))
    d = d.astype(np.uint8)
    z = _check_compress(bz, d, [0, d.size], 1, "one 9 MB caller block, level 1")
    assert bz2.decompress(z) == d.tobytes()


@pytest.mark.parametrize("level", [9, 5])
def test_compress_empty_blocks_without_cuts(bz, level):
    # no block needs cutting at these levels, and empty blocks sit at the
    # front, in the middle and at the end: every non-empty block must stay
    b = W.config2(total=6 * 80000 + 777, block=80000, seed=23)
    o = [int(x) for x in b.offsets]
    offs = [0, 0] + o[1:4] + [o[3]] + o[4:] + [o[-1], o[-1]]
    z = _check_compress(bz, b.data, offs, level, f"empty blocks among {len(o) - 1} uncut blocks, level {level}")
    assert bz2.decompress(z) == b.data.tobytes()


def test_compress_rejects_bad_args(bz):
    x = _dev(np.zeros(10, np.uint8))
    with pytest.raises(bz.BzgError):
        bz.compress(x, [0, 10], level=0)
    with pytest.raises(bz.BzgError):
        bz.compress(x, [0, 7, 3, 10], level=9)


def _batch_inputs(reqs, block):
    """All requests' bytes, block offsets (each request cut into `block`-byte
    blocks) and the request -> block ranges."""
    datas, offs, rq = [], [0], [0]
    pos = 0
    for r in reqs:
        n = len(r)
        for a in range(0, n, block):
            offs.append(pos + min(a + block, n))
        pos += n
        datas.append(np.frombuffer(bytes(r), np.uint8) if not isinstance(r, np.ndarray) else r)
        rq.append(len(offs) - 1)
    data = np.concatenate(datas) if datas else np.zeros(0, np.uint8)
    return data, np.array(offs, np.uint64), np.array(rq, np.uint32)


def _check_batch(bz, reqs, level, block, name):
    from paper_1109_2348_amd import native
    data, offs, rq = _batch_inputs(reqs, block)
    _say(f"compress_batch {name}: {len(reqs)} requests, {data.size} bytes, {offs.size - 1} blocks, level {level}")
    zs = native.compress_batch(_dev(data), offs, rq, level=level)
    assert len(zs) == len(reqs)
    for i, r in enumerate(reqs):
        a, e = int(rq[i]), int(rq[i + 1])
        ro = offs[a:e + 1] - offs[a]
        rd = data[int(offs[a]):int(offs[e])]
        z = zs[i].cpu().numpy().tobytes()
        ref = cref.compress(rd, ro if e > a else [0], level=level, threads=16)
        assert z == ref, f"{name}: request {i} ({rd.size} B) differs from the oracle run on it alone"
        assert bz2.decompress(z) == rd.tobytes()
    return zs


def test_compress_batch_each_stream_alone(bz):
    rnd = random.Random(23)
    b = W.config4(nb=12, lo=1, hi=120000, seed=29)
    reqs = [b"", b"banana", b.block(0), b"", bytes(rnd.randrange(4) for _ in range(70000))]
    reqs += [b.block(k) for k in range(1, 12)] + [b"a" * 250000, b""]
    _check_batch(bz, reqs, 1, 100000, "mixed sizes, empty requests, level-1 cuts")


def test_compress_batch_same_as_compress_blocks(bz):
    b = W.config2(total=3 * 900000 + 4321, block=900000, seed=31)
    data, offs, rq = _batch_inputs([b.data[: 2 * 900000], b.data[2 * 900000:]], 900000)
    from paper_1109_2348_amd import native
    _say("compress_batch vs compress_blocks: 2 requests of 900000-byte blocks")
    zs = native.compress_batch(_dev(data), offs, rq, level=9)
    for i in range(2):
        a, e = int(rq[i]), int(rq[i + 1])
        alone = bz.compress(_dev(data[int(offs[a]):int(offs[e])]), offs[a:e + 1] - offs[a], level=9)
        assert zs[i].cpu().numpy().tobytes() == alone.cpu().numpy().tobytes()


def test_compress_batch_all_empty_and_capacity(bz):
    import ctypes as C
    import torch
    from paper_1109_2348_amd import native
    _say("compress_batch: all-empty requests; one range too small")
    zs = native.compress_batch(_dev(np.zeros(0, np.uint8)), [0, 0, 0], [0, 0, 1, 2], level=3)
    for z in zs:
        assert bz2.decompress(z.cpu().numpy().tobytes()) == b""
    data, offs, rq = _batch_inputs([bytes(range(256)) * 40, b"xyz" * 999], 100000)
    x = _dev(data)
    out = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    oo = np.array([0, 64, 1 << 16], np.uint64)  # request 0 gets 64 bytes: too few
    ctx = native.context()
    bc = native.BatchCompressor(ctx=ctx)
    bc.out = out
    _, ob = bc.enqueue(x, offs, rq, 9, out_offsets=oo)
    with pytest.raises(bz.BzgError) as ei:
        ctx.sync_check(native._stream(x.device))
    assert ei.value.code == native.BZG_ECAPACITY
    ob = ob.cpu().numpy()
    assert ob[0] > 64 and ob[1] > 0
    oo = np.array([0, 4 * ((int(ob[0]) + 3) // 4), 1 << 16], np.uint64)  # exactly enough
    _, ob = bc.enqueue(x, offs, rq, 9, out_offsets=oo)
    ctx.sync_check(native._stream(x.device))
    ob = ob.cpu().numpy()
    o = out.cpu().numpy()
    for i in range(2):
        z = o[int(oo[i]): int(oo[i]) + int(ob[i])].tobytes()
        a, e = int(rq[i]), int(rq[i + 1])
        assert bz2.decompress(z) == data[int(offs[a]):int(offs[e])].tobytes()


def test_compress_batch_rejects_bad_args(bz):
    from paper_1109_2348_amd import native
    x = _dev(np.zeros(10, np.uint8))
    with pytest.raises(bz.BzgError):
        native.compress_batch(x, [0, 5, 10], [0, 1], level=9)  # ranges end before n_blocks
    with pytest.raises(bz.BzgError):
        native.compress_batch(x, [0, 5, 10], [0, 2, 1, 2], level=9)  # ranges decrease
    with pytest.raises(bz.BzgError):
        native.compress_batch(x, [0, 5, 10], [0, 2], level=10)


def test_compress_batch_many_small_requests(bz):
    rnd = random.Random(37)
    reqs = []
    for i in range(600):
        k = rnd.choice([0, 0, 1, 2, 3, 4, 5, 17, 64, 255, 256, 1000, 5000])
        reqs.append(bytes(rnd.randrange(256) for _ in range(k)) if i % 3 else bytes([i & 255]) * k)
    _check_batch(bz, reqs, 9, 900000, "600 requests of 0..5000 bytes")


@pytest.mark.slow
def test_compress_config4_full(bz):
    """8192 uneven blocks in one call: the stock decoder recovers the input;
    sampled blocks, compressed in one launch as separate streams, equal the
    oracle's streams of those blocks."""
    from paper_1109_2348_amd import native
    b = W.config4()
    _say(f"compress 8192 uneven blocks ({b.data.size} B), level 9")
    z = bz.compress(_dev(b.data), b.offsets, level=9).cpu().numpy().tobytes()
    assert bz2.decompress(z) == b.data.tobytes()
    rnd = random.Random(41)
    pick = sorted(rnd.sample(range(b.n_blocks), 24))
    blocks = [b.block(k) for k in pick]
    data, offs, rq = _batch_inputs(blocks, 900000)
    _say(f"compress_batch of {len(pick)} sampled blocks vs the oracle")
    zs = native.compress_batch(_dev(data), offs, rq, level=9)
    for k, blk, zk in zip(pick, blocks, zs):
        assert zk.cpu().numpy().tobytes() == cref.compress(blk, [0, blk.size], level=9), f"block {k}"


@pytest.mark.slow
def test_compress_config2_full(bz):
    b = W.config2()
    z = _check_compress(bz, b.data, b.offsets, 9, "64 MiB in 900000-byte blocks")
    assert bz2.decompress(z) == b.data.tobytes()


@pytest.mark.slow
def test_bwt_config3_all_blocks(bz):
    """Sort worst case, every block validated: the oracle's property check
    (a permutation whose adjacent rotations are in order, equal ones by
    descending start) fixes the suffix order uniquely, so with it L and the
    primary index follow.  Threaded over the host cores."""
    import concurrent.futures as cf
    import time
    b = W.config3()
    _say("bwt 256 x 900000 periodic / all-same (all blocks, property check)")
    L, prim, sa = bz.bwt(_dev(b.data), b.offsets, want_sa=True)
    sa = sa.cpu().numpy().view(np.uint32)
    L = L.cpu().numpy()
    prim = prim.cpu().numpy()
    t0 = time.time()

    def one(k):
        a, e = int(b.offsets[k]), int(b.offsets[k + 1])
        blk = b.block(k)
        s = sa[a:e]
        if cref.check_sa(blk, s) != -1:
            return f"block {k} ({b.kinds[k]}): SA not sorted"
        if not np.array_equal(L[a:e], blk[(s.astype(np.int64) - 1) % (e - a)]):
            return f"block {k}: L is not the byte before each sorted rotation"
        if int(s[int(prim[k])]) != 0:
            return f"block {k}: primary {prim[k]} is not the row of rotation 0"
        return None

    with cf.ThreadPoolExecutor(16) as ex:
        errs = [m for m in ex.map(one, range(b.n_blocks)) if m]
    _say(f"checked {b.n_blocks} blocks in {time.time() - t0:.1f} s")
    assert not errs, errs[:5]
