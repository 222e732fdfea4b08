"""Tier-0 oracle: plain, slow, obviously-correct Python for every stage of the
bzip2 compression path (test infrastructure only; never used by the product).

Paper passages followed (Eirola, "Lossless data compression on GPGPU
architectures"):

* Sec. 2.1   -- splitting the input into blocks that are compressed
                independently.
* Sec. 3.1   -- the Burrows-Wheeler transform is the sort of the rotations of
                the input; the inverse can start from any row.
* Sec. 3.2   -- run-length encoding in four steps (Figure 1: boundary flags,
                prefix sum, scatter, differences) and decoding (Figure 2).
* Sec. 3.3   -- move-to-front over a stack of recently used symbols.
* Sec. 3.4   -- variable-length encoding: code lengths, prefix sum of the
                lengths gives the bit offsets (Figure 3); Huffman codes.
* Sec. 4     -- the stages combined into a bzip2-compatible compressor; code
                tables chosen by analysing the data.

The paper does not give the bzip2 container syntax (RLE1, RUNA/RUNB, the table
heuristic, the bit layout); those follow the public bzip2 format description
and the readings listed in the design notes.  Every reading is marked
"Reading:" below.
"""

from __future__ import annotations

import heapq
from typing import List, Sequence, Tuple

# ---------------------------------------------------------------------------
# Figures 1-3 of the paper, as written (generic primitives).
# ---------------------------------------------------------------------------


def exclusive_scan(xs: Sequence[int]) -> List[int]:
    """Exclusive prefix sum (Sec. 2.1: the parallel prefix-sum primitive)."""
    out, acc = [], 0
    for x in xs:
        out.append(acc)
        acc += x
    return out


def inclusive_scan(xs: Sequence[int]) -> List[int]:
    out, acc = [], 0
    for x in xs:
        acc += x
        out.append(acc)
    return out


def rle_encode_fig1(data: Sequence) -> dict:
    """Run-length encoding in the four steps of Figure 1 (Sec. 3.2).

    Step 1 marks the last element of every run; step 2 takes the exclusive
    prefix sum of the marks as output positions; step 3 copies the character
    and its end index (last index + 1) to that position; step 4 differences
    the end indices to get the run lengths.
    """
    n = len(data)
    flags = [1 if (i == n - 1 or data[i] != data[i + 1]) else 0 for i in range(n)]
    pos = exclusive_scan(flags)
    nruns = sum(flags)
    chars = [None] * nruns
    ends = [0] * nruns
    for i in range(n):
        if flags[i]:
            chars[pos[i]] = data[i]
            ends[pos[i]] = i + 1
    lengths = [ends[k] - (ends[k - 1] if k else 0) for k in range(nruns)]
    return {"flags": flags, "positions": pos, "chars": chars, "ends": ends,
            "lengths": lengths}


def rle_decode_fig2(chars: Sequence, lengths: Sequence[int]) -> dict:
    """Run-length decoding in the four steps of Figure 2 (Sec. 3.2).

    Step 1: inclusive prefix sum of the lengths gives each run's end; step 2
    sets a 1 at index end-1; step 3: exclusive prefix sum of those flags gives
    every output element the index of its run; step 4 gathers the characters.
    """
    ends = inclusive_scan(lengths)
    n = ends[-1] if ends else 0
    flags = [0] * n
    for e in ends:
        if e:
            flags[e - 1] = 1
    idx = exclusive_scan(flags)
    out = [chars[idx[i]] for i in range(n)]
    return {"ends": ends, "flags": flags, "indices": idx, "output": out}


def vle_offsets_fig3(code_lengths: Sequence[int]) -> List[int]:
    """Figure 3 (Sec. 3.4): the bit offset of every codeword is the exclusive
    prefix sum of the codeword lengths."""
    return exclusive_scan(code_lengths)


# ---------------------------------------------------------------------------
# Block CRC (bzip2 container; not in the paper).
# ---------------------------------------------------------------------------

CRC_POLY = 0x04C11DB7


def crc32_bzip2(data: bytes) -> int:
    """CRC-32/BZIP2 written bit by bit from its definition: polynomial
    0x04C11DB7, bits taken most-significant first, register preset to all
    ones, result complemented."""
    reg = 0xFFFFFFFF
    for byte in data:
        for bit in range(7, -1, -1):
            inbit = (byte >> bit) & 1
            top = (reg >> 31) & 1
            reg = (reg << 1) & 0xFFFFFFFF
            if top ^ inbit:
                reg ^= CRC_POLY
    return reg ^ 0xFFFFFFFF


def combine_stream_crc(block_crcs: Sequence[int]) -> int:
    """Stream CRC: rotate the running value left by one bit, then XOR in the
    next block's CRC."""
    c = 0
    for k in block_crcs:
        c = (((c << 1) | (c >> 31)) & 0xFFFFFFFF) ^ k
    return c


# ---------------------------------------------------------------------------
# RLE1 (bzip2's first run-length stage).  Reading: the paper's generic RLE of
# Sec. 3.2 stands for bzip2's RLE1, applied before the BWT.
# ---------------------------------------------------------------------------


def rle1_encode(block: bytes) -> bytes:
    out = bytearray()
    i, n = 0, len(block)
    while i < n:
        b = block[i]
        r = 1
        while i + r < n and block[i + r] == b:
            r += 1
        i += r
        while r > 0:  # cut the run into pieces of at most 255
            c = min(r, 255)
            if c >= 4:
                out += bytes([b, b, b, b, c - 4])
            else:
                out += bytes([b] * c)
            r -= c
    return bytes(out)


def rle1_decode(data: bytes) -> bytes:
    out = bytearray()
    i, n = 0, len(data)
    while i < n:
        b = data[i]
        r = 1
        while r < 4 and i + r < n and data[i + r] == b:
            r += 1
        out += bytes([b] * r)
        i += r
        if r == 4:
            if i >= n:
                raise ValueError("RLE1: run of four without a count byte")
            out += bytes([b] * data[i])
            i += 1
    return bytes(out)


# ---------------------------------------------------------------------------
# BWT (Sec. 3.1).
# ---------------------------------------------------------------------------


def bwt_sa(s: bytes) -> List[int]:
    """Sorted rotation start indices.  The rotations are compared as unsigned
    byte strings; equal rotations (only in cyclically periodic blocks) are
    ordered by descending start index (Reading: the paper does not fix a
    tie-break; this one is the stock bzip2 encoder's observed order)."""
    n = len(s)
    ss = s + s
    return sorted(range(n), key=lambda i: (ss[i:i + n], -i))


def bwt_encode(s: bytes) -> Tuple[bytes, int]:
    """L[k] = the byte before rotation SA[k]; origPtr = the row holding
    rotation 0."""
    if not s:
        raise ValueError("empty block")
    sa = bwt_sa(s)
    n = len(s)
    last = bytes(s[(i - 1) % n] for i in sa)
    return last, sa.index(0)


def bwt_decode(last: bytes, orig_ptr: int) -> bytes:
    """Inverse BWT by the LF mapping, walking from row origPtr (Sec. 3.1)."""
    n = len(last)
    order = sorted(range(n), key=lambda k: (last[k], k))  # stable by byte
    # order[j] = the row of L whose byte is the j-th byte of F (first column)
    out = bytearray(n)
    row = orig_ptr
    for i in range(n):
        j = order[row]
        out[i] = last[j]
        row = j
    return bytes(out)


# ---------------------------------------------------------------------------
# MTF (Sec. 3.3).  Reading: the stack holds the block's in-use byte values,
# initially ascending; the output is the stack position.
# ---------------------------------------------------------------------------


def in_use(data: bytes) -> List[int]:
    return sorted(set(data))


def mtf_encode(last: bytes) -> Tuple[List[int], List[int]]:
    stack = in_use(last)
    used = list(stack)
    out = []
    for b in last:
        v = stack.index(b)
        out.append(v)
        stack.pop(v)
        stack.insert(0, b)
    return out, used


def mtf_decode(idx: Sequence[int], used: Sequence[int]) -> bytes:
    stack = list(used)
    out = bytearray()
    for v in idx:
        b = stack.pop(v)
        out.append(b)
        stack.insert(0, b)
    return bytes(out)


# ---------------------------------------------------------------------------
# RUNA/RUNB zero-run coding (bzip2 container; the run detection is the
# primitive of Figure 1).
# ---------------------------------------------------------------------------

RUNA, RUNB = 0, 1


def zero_run_digits(r: int) -> List[int]:
    """A run of r zeros as bijective base-2 digits, least significant first:
    digit 1 -> RUNA, digit 2 -> RUNB."""
    out = []
    while r > 0:
        if r & 1:
            out.append(RUNA)
            r = (r - 1) >> 1
        else:
            out.append(RUNB)
            r = (r - 2) >> 1
    return out


def zero_run_value(digits: Sequence[int]) -> int:
    r, w = 0, 1
    for d in digits:
        r += w * (1 if d == RUNA else 2)
        w <<= 1
    return r


def zrle_encode(mtf: Sequence[int], n_inuse: int) -> List[int]:
    out: List[int] = []
    run = 0
    for v in mtf:
        if v == 0:
            run += 1
            continue
        out += zero_run_digits(run)
        run = 0
        out.append(v + 1)
    out += zero_run_digits(run)
    out.append(n_inuse + 1)  # end of block
    return out


def zrle_decode(syms: Sequence[int], n_inuse: int) -> List[int]:
    out: List[int] = []
    digits: List[int] = []
    for s in syms:
        if s in (RUNA, RUNB):
            digits.append(s)
            continue
        out += [0] * zero_run_value(digits)
        digits = []
        if s == n_inuse + 1:
            return out
        out.append(s - 1)
    raise ValueError("no end-of-block symbol")


# ---------------------------------------------------------------------------
# Huffman tables (Sec. 3.4 Huffman coding; Sec. 4 tables chosen from the data).
# Reading: every constant below (table count by symbol count, the initial
# partition, four refinement passes, 50-symbol groups, maximum length 17,
# weight floor 1, the (weight, id) tie-break and the halving rescale) is a
# project constant; the paper gives no construction.
# ---------------------------------------------------------------------------

GROUP = 50
MAX_LEN = 17
N_ITERS = 4


def huffman_lengths(freq: Sequence[int], max_len: int = MAX_LEN) -> List[int]:
    """Textbook Huffman: repeatedly merge the two lightest nodes, ordered by
    (weight, id) with leaves numbered by symbol and internal nodes numbered
    from len(freq) upward in creation order; the code length is the leaf
    depth.  While the longest code exceeds max_len every weight w becomes
    1 + w // 2 and the tree is rebuilt."""
    a = len(freq)
    w = [max(f, 1) for f in freq]
    while True:
        heap = [(w[i], i) for i in range(a)]
        heapq.heapify(heap)
        parent = {}
        nxt = a
        while len(heap) > 1:
            w1, x = heapq.heappop(heap)
            w2, y = heapq.heappop(heap)
            parent[x] = nxt
            parent[y] = nxt
            heapq.heappush(heap, (w1 + w2, nxt))
            nxt += 1
        lengths = []
        for i in range(a):
            d, node = 0, i
            while node in parent:
                node = parent[node]
                d += 1
            lengths.append(d)
        if max(lengths) <= max_len:
            return lengths
        w = [1 + x // 2 for x in w]


def canonical_codes(lengths: Sequence[int]) -> List[int]:
    """Codes assigned in order of (length, symbol), counting up and shifting
    left by one between lengths."""
    codes = [0] * len(lengths)
    code = 0
    for ln in range(min(lengths), max(lengths) + 1):
        for s, l in enumerate(lengths):
            if l == ln:
                codes[s] = code
                code += 1
        code <<= 1
    return codes


def n_tables(n_syms: int, alpha_size: int) -> int:
    if n_syms < 200:
        g = 2
    elif n_syms < 600:
        g = 3
    elif n_syms < 1200:
        g = 4
    elif n_syms < 2400:
        g = 5
    else:
        g = 6
    return min(g, alpha_size)


def initial_tables(freq: Sequence[int], n_groups: int) -> List[List[int]]:
    """Cut the alphabet into n_groups contiguous ranges of about equal total
    frequency; table t costs 0 inside its range and 15 outside."""
    a = len(freq)
    rem = sum(freq)
    gs = 0
    tables = []
    for t in range(n_groups):
        left = n_groups - t
        if left == 1:
            ge = a - 1
        else:
            ge = gs
            acc = freq[gs]
            while ge + 1 <= a - left and acc * left < rem:
                ge += 1
                acc += freq[ge]
        tables.append([0 if gs <= v <= ge else 15 for v in range(a)])
        rem -= sum(freq[gs:ge + 1])
        gs = ge + 1
    return tables


def choose_tables(syms: Sequence[int], alpha_size: int, n_iters: int = N_ITERS):
    """Returns (lengths per table, selectors) after n_iters refinement passes
    (the tests pin single passes with n_iters=1)."""
    n = len(syms)
    freq = [0] * alpha_size
    for s in syms:
        freq[s] += 1
    g = n_tables(n, alpha_size)
    n_sel = (n + GROUP - 1) // GROUP
    lens = initial_tables(freq, g)
    sel = [0] * n_sel
    for _ in range(n_iters):
        tf = [[0] * alpha_size for _ in range(g)]
        for j in range(n_sel):
            grp = syms[j * GROUP:(j + 1) * GROUP]
            costs = [sum(lens[t][s] for s in grp) for t in range(g)]
            best = min(range(g), key=lambda t: (costs[t], t))
            sel[j] = best
            for s in grp:
                tf[best][s] += 1
        lens = [huffman_lengths(tf[t]) for t in range(g)]
    return lens, sel


# ---------------------------------------------------------------------------
# Bit writer / reader (MSB first) and the bzip2 container.
# ---------------------------------------------------------------------------

BLOCK_MAGIC = 0x314159265359
EOS_MAGIC = 0x177245385090


class BitWriter:
    def __init__(self):
        self.bits: List[int] = []

    def put(self, value: int, nbits: int):
        for k in range(nbits - 1, -1, -1):
            self.bits.append((value >> k) & 1)

    def tobytes(self) -> bytes:
        bits = self.bits + [0] * (-len(self.bits) % 8)
        out = bytearray()
        for i in range(0, len(bits), 8):
            v = 0
            for b in bits[i:i + 8]:
                v = (v << 1) | b
            out.append(v)
        return bytes(out)


class BitReader:
    def __init__(self, data: bytes):
        self.data = data
        self.pos = 0

    def get(self, nbits: int) -> int:
        v = 0
        for _ in range(nbits):
            byte = self.data[self.pos >> 3]
            v = (v << 1) | ((byte >> (7 - (self.pos & 7))) & 1)
            self.pos += 1
        return v


def write_block_body(w: BitWriter, used: Sequence[int], lens, sel, syms):
    """Everything after origPtr: symbol map, table count, selectors (MTF then
    unary), delta-coded code lengths, then the codes (Figure 3: the codes are
    laid end to end, each at the prefix sum of the earlier lengths)."""
    used_set = set(used)
    ranges = [any((16 * i + j) in used_set for j in range(16)) for i in range(16)]
    for i in range(16):
        w.put(1 if ranges[i] else 0, 1)
    for i in range(16):
        if ranges[i]:
            for j in range(16):
                w.put(1 if (16 * i + j) in used_set else 0, 1)
    g = len(lens)
    w.put(g, 3)
    w.put(len(sel), 15)
    stack = list(range(g))
    for s in sel:
        v = stack.index(s)
        w.put((1 << (v + 1)) - 2, v + 1)  # v ones then a zero
        stack.pop(v)
        stack.insert(0, s)
    for t in range(g):
        cur = lens[t][0]
        w.put(cur, 5)
        for ln in lens[t]:
            while cur < ln:
                w.put(0b10, 2)
                cur += 1
            while cur > ln:
                w.put(0b11, 2)
                cur -= 1
            w.put(0, 1)
    codes = [canonical_codes(l) for l in lens]
    for j, s in enumerate(syms):
        t = sel[j // GROUP]
        w.put(codes[t][s], lens[t][s])


# ---------------------------------------------------------------------------
# Precomputed tables (Sec. 4: tables computed beforehand by analysing data,
# so that no Huffman tree is built per block).
# ---------------------------------------------------------------------------

FULL_ALPHA = 258  # RUNA, RUNB, MTF values 1..255, EOB for 256 bytes in use


def to_full_alphabet(syms: Sequence[int], alpha_size: int) -> List[int]:
    """A block's symbols in the alphabet of a block with every byte in use:
    RUNA, RUNB and MTF values keep their numbers, EOB becomes 257.
    Reading: precomputed tables are indexed this way."""
    return [FULL_ALPHA - 1 if s == alpha_size - 1 else s for s in syms]


SAMPLE_SYMS = 900000  # symbols a sample contributes at most (about one block's worth)


def sample_symbols(block: bytes) -> Tuple[List[int], int]:
    """A sample block's symbols: BWT, MTF and RUNA/RUNB of the block as
    given (Reading: no RLE1 in the analysis), with its alphabet size."""
    last, _ = bwt_encode(block)
    mtf, used = mtf_encode(last)
    return zrle_encode(mtf, len(used)), len(used) + 2


def tables_from_sample(block_syms: Sequence[Tuple[Sequence[int], int]]):
    """Reading of "chosen by analysing the data": the blocks' symbol streams
    (each with its alphabet size), in the full alphabet and one after another,
    cut to the first SAMPLE_SYMS symbols, get the same table heuristic as one
    block (choose_tables).  Returns the tables' code lengths over the 258
    symbols."""
    pooled: List[int] = []
    for syms, a in block_syms:
        pooled += to_full_alphabet(syms, a)
    lens, _ = choose_tables(pooled[:SAMPLE_SYMS], FULL_ALPHA)
    return lens


def restrict_tables(fixed, alpha_size: int):
    """The fixed tables as a block of alphabet alpha_size uses them: symbols
    0..alpha_size-2 keep their lengths, EOB takes the length of symbol 257.
    A subset of a prefix code's lengths still satisfies Kraft's inequality,
    so canonical codes of the restriction form a prefix code."""
    return [[t[v] for v in range(alpha_size - 1)] + [t[FULL_ALPHA - 1]] for t in fixed]


def select_fixed(syms: Sequence[int], lens) -> List[int]:
    """Each 50-symbol group takes the table that codes it in the fewest bits,
    the lowest index on ties (the selector step of choose_tables, once)."""
    n_sel = (len(syms) + GROUP - 1) // GROUP
    sel = []
    for j in range(n_sel):
        grp = syms[j * GROUP:(j + 1) * GROUP]
        costs = [sum(t[s] for s in grp) for t in lens]
        sel.append(min(range(len(lens)), key=lambda t: (costs[t], t)))
    return sel


def encode_block(raw: bytes, fixed=None) -> dict:
    """All stages for one block; returns every intermediate for tests.  With
    `fixed` (precomputed tables over 258 symbols) the tables are not built:
    the block uses their restriction and only chooses selectors."""
    crc = crc32_bzip2(raw)
    r1 = rle1_encode(raw)
    last, optr = bwt_encode(r1)
    mtf, used = mtf_encode(last)
    syms = zrle_encode(mtf, len(used))
    if fixed is None:
        lens, sel = choose_tables(syms, len(used) + 2)
    else:
        lens = restrict_tables(fixed, len(used) + 2)
        sel = select_fixed(syms, lens)
    return {"crc": crc, "rle1": r1, "bwt": last, "orig_ptr": optr, "mtf": mtf,
            "used": used, "syms": syms, "lens": lens, "sel": sel}


def cut_blocks(n: int, block_bytes: int) -> List[int]:
    """Offsets of consecutive blocks of block_bytes input bytes, the last one
    shorter (Sec. 2.1).  Reading: blocks are cut by input bytes."""
    offs = list(range(0, n, block_bytes)) + [n]
    return offs if n else [0]


def rle1_limit(level: int) -> int:
    """Largest RLE1 output a decoder for header digit `level` accepts."""
    return 100000 * level


def split_for_limit(data: bytes, offsets: Sequence[int], limit: int) -> List[int]:
    """Reading: a caller's block whose RLE1 output exceeds the limit is cut
    after the longest input prefix whose own RLE1 output fits; the rest is
    treated as the next block (and cut again if needed).  The RLE1 length of a
    prefix never decreases as the prefix grows, so the cut is found by
    bisection.  Empty blocks are dropped."""
    out = [0] if not offsets else [offsets[0]]
    for k in range(len(offsets) - 1):
        lo_off, hi_off = offsets[k], offsets[k + 1]
        while hi_off > lo_off:
            raw = data[lo_off:hi_off]
            if len(rle1_encode(raw)) <= limit:
                out.append(hi_off)
                break
            lo, hi = 0, len(raw)  # largest j with |rle1(raw[:j])| <= limit
            while lo < hi:
                mid = (lo + hi + 1) // 2
                if len(rle1_encode(raw[:mid])) <= limit:
                    lo = mid
                else:
                    hi = mid - 1
            lo_off += lo
            out.append(lo_off)
    return out


def compress(data: bytes, level: int = 9, offsets: Sequence[int] | None = None, fixed=None) -> bytes:
    """Reading: the header digit is the level; blocks are first cut so that no
    RLE1 output exceeds 100000 * level (split_for_limit).  fixed: optional
    precomputed tables (lengths over 258 symbols, 2..6 tables)."""
    if offsets is None:
        offsets = cut_blocks(len(data), 100000 * level)
    offsets = split_for_limit(data, offsets, rle1_limit(level))
    blocks = [encode_block(data[offsets[k]:offsets[k + 1]], fixed)
              for k in range(len(offsets) - 1) if offsets[k + 1] > offsets[k]]
    w = BitWriter()
    w.put(ord("B"), 8)
    w.put(ord("Z"), 8)
    w.put(ord("h"), 8)
    w.put(ord("0") + level, 8)
    for b in blocks:
        w.put(BLOCK_MAGIC, 48)
        w.put(b["crc"], 32)
        w.put(0, 1)
        w.put(b["orig_ptr"], 24)
        write_block_body(w, b["used"], b["lens"], b["sel"], b["syms"])
    w.put(EOS_MAGIC, 48)
    w.put(combine_stream_crc([b["crc"] for b in blocks]), 32)
    return w.tobytes()


# ---------------------------------------------------------------------------
# Decoder (inverts every stage; used to round-trip the oracle's own output and
# to recover the stage outputs of other encoders' streams).
# ---------------------------------------------------------------------------


def decode_block_body(r: BitReader):
    ranges = [r.get(1) for _ in range(16)]
    used = []
    for i in range(16):
        if ranges[i]:
            for j in range(16):
                if r.get(1):
                    used.append(16 * i + j)
    alpha = len(used) + 2
    g = r.get(3)
    n_sel = r.get(15)
    stack = list(range(g))
    sel = []
    for _ in range(n_sel):
        v = 0
        while r.get(1):
            v += 1
        s = stack.pop(v)
        stack.insert(0, s)
        sel.append(s)
    lens = []
    for _ in range(g):
        cur = r.get(5)
        ln = []
        for _ in range(alpha):
            while r.get(1):
                cur += -1 if r.get(1) else 1
            ln.append(cur)
        lens.append(ln)
    tables = []
    for t in range(g):
        codes = canonical_codes(lens[t])
        tables.append({(lens[t][s], codes[s]): s for s in range(alpha)})
    syms = []
    eob = alpha - 1
    j = 0
    while True:
        t = sel[j // GROUP]
        code, ln = 0, 0
        while (ln, code) not in tables[t]:
            code = (code << 1) | r.get(1)
            ln += 1
            if ln > 20:
                raise ValueError("bad code")
        s = tables[t][(ln, code)]
        syms.append(s)
        j += 1
        if s == eob:
            break
    return used, lens, sel, syms


def decompress(stream: bytes, want_stages: bool = False):
    r = BitReader(stream)
    if stream[:3] != b"BZh":
        raise ValueError("bad magic")
    r.pos = 32
    out = bytearray()
    stages = []
    crcs = []
    while True:
        magic = r.get(48)
        if magic == EOS_MAGIC:
            stored = r.get(32)
            if stored != combine_stream_crc(crcs):
                raise ValueError("stream CRC mismatch")
            break
        if magic != BLOCK_MAGIC:
            raise ValueError("bad block magic")
        crc = r.get(32)
        if r.get(1):
            raise ValueError("randomised blocks not supported")
        optr = r.get(24)
        used, lens, sel, syms = decode_block_body(r)
        mtf = zrle_decode(syms, len(used))
        last = mtf_decode(mtf, used)
        r1 = bwt_decode(last, optr)
        raw = rle1_decode(r1)
        if crc32_bzip2(raw) != crc:
            raise ValueError("block CRC mismatch")
        crcs.append(crc)
        out += raw
        stages.append({"crc": crc, "orig_ptr": optr, "used": used, "lens": lens,
                       "sel": sel, "syms": syms, "mtf": mtf, "bwt": last,
                       "rle1": r1})
    return (bytes(out), stages) if want_stages else bytes(out)
