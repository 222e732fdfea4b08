"""Oracle for the light-weight field codecs (test infrastructure only; the
product never imports it).

The paper points at compressors that code each field of a record with a
cheap code instead of a general-purpose one (Sec. 2.1: null suppression and
Elias delta coding), and at a GPU floating-point compressor that subtracts a
prediction and drops leading zero bytes (Sec. 3.5, GFC).  Each codec below is
written from its definition, one value at a time, with the same stream
layout the GPU path produces (the layout is this project's; the paper gives
none -- see the readings in the design notes):

* null suppression, 32-bit integers: per value a 2-bit code (bytes - 1, the
  bytes needed for the value, at least one), four codes per byte, low bits
  first; then each value's bytes, least significant first, back to back;
* Elias delta, 32-bit integers v (coded as x = v + 1 >= 1): N = floor(log2 x),
  M = floor(log2(N + 1)); M zero bits, then N + 1 in M + 1 bits, then the N
  low bits of x; codes back to back in a bit stream whose bit k is bit
  31 - k % 32 of 32-bit word k / 32; an index of the bit offset of every
  1024th value;
* GFC-style delta, 64-bit floats: the residual r = bits(x_i) - bits(x_{i-1})
  modulo 2^64 (x_{-1} = 0); when r's top bit is set the code keeps -r and a
  sign flag; per value a 4-bit code (sign << 3 | leading zero bytes, at most
  7), two codes per byte, low nibble first; then each value's 8 - lzb low
  bytes, least significant first.

Every stream starts with the value count as a little-endian uint64.
"""

from __future__ import annotations

import struct
from typing import List, Sequence

EDELTA_INDEX_EVERY = 1024


# ------------------------------------------------------------ null suppression

def ns_bytes(v: int) -> int:
    n = 1
    while v >= 1 << (8 * n):
        n += 1
    return n


def ns_encode(values: Sequence[int]) -> bytes:
    n = len(values)
    out = bytearray(struct.pack("<Q", n))
    codes = bytearray((n + 3) // 4)
    for i, v in enumerate(values):
        codes[i // 4] |= (ns_bytes(v) - 1) << (2 * (i % 4))
    out += codes
    for v in values:
        out += int(v).to_bytes(ns_bytes(v), "little")
    return bytes(out)


def ns_decode(stream: bytes) -> List[int]:
    (n,) = struct.unpack_from("<Q", stream, 0)
    pos = 8 + (n + 3) // 4
    out = []
    for i in range(n):
        k = ((stream[8 + i // 4] >> (2 * (i % 4))) & 3) + 1
        out.append(int.from_bytes(stream[pos:pos + k], "little"))
        pos += k
    return out


# ---------------------------------------------------------------- Elias delta

def edelta_code(x: int) -> str:
    """Elias delta code of x >= 1 as a bit string."""
    assert x >= 1
    n = x.bit_length() - 1
    m = (n + 1).bit_length() - 1
    return "0" * m + format(n + 1, "b") + (format(x, "b")[1:] if n else "")


def edelta_encode(values: Sequence[int]) -> bytes:
    bits = []
    index = []
    pos = 0
    for i, v in enumerate(values):
        if i % EDELTA_INDEX_EVERY == 0:
            index.append(pos)
        c = edelta_code(int(v) + 1)
        bits.append(c)
        pos += len(c)
    s = "".join(bits)
    words = (len(s) + 31) // 32
    s += "0" * (32 * words - len(s))
    out = bytearray(struct.pack("<QQ", len(values), pos))
    for p in index:
        out += struct.pack("<Q", p)
    for w in range(words):
        out += struct.pack("<I", int(s[32 * w:32 * w + 32], 2))
    return bytes(out)


def edelta_decode(stream: bytes) -> List[int]:
    n, total = struct.unpack_from("<QQ", stream, 0)
    ni = (n + EDELTA_INDEX_EVERY - 1) // EDELTA_INDEX_EVERY
    base = 16 + 8 * ni
    nw = (total + 31) // 32
    s = "".join(format(struct.unpack_from("<I", stream, base + 4 * w)[0], "032b") for w in range(nw))
    out, p = [], 0
    for _ in range(n):
        m = 0
        while s[p] == "0":
            m += 1
            p += 1
        n1 = int(s[p:p + m + 1], 2)
        p += m + 1
        nb = n1 - 1
        x = int("1" + s[p:p + nb], 2) if nb else 1
        p += nb
        out.append(x - 1)
    return out


# ------------------------------------------------------- GFC-style float delta

def _bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def gfc_encode_bits(words: Sequence[int]) -> bytes:
    """Codes 64-bit patterns (the bits of the doubles)."""
    n = len(words)
    out = bytearray(struct.pack("<Q", n))
    codes = bytearray((n + 1) // 2)
    data = bytearray()
    prev = 0
    for i, w in enumerate(words):
        r = (int(w) - prev) % (1 << 64)
        prev = int(w)
        sign = r >> 63
        if sign:
            r = (-r) % (1 << 64)
        lzb = 0
        while lzb < 7 and (r >> (8 * (7 - lzb))) & 0xFF == 0:
            lzb += 1
        codes[i // 2] |= ((sign << 3) | lzb) << (4 * (i % 2))
        data += r.to_bytes(8, "little")[:8 - lzb]
    return bytes(out + codes + data)


def gfc_decode_bits(stream: bytes) -> List[int]:
    (n,) = struct.unpack_from("<Q", stream, 0)
    pos = 8 + (n + 1) // 2
    out, prev = [], 0
    for i in range(n):
        c = (stream[8 + i // 2] >> (4 * (i % 2))) & 15
        k = 8 - (c & 7)
        r = int.from_bytes(stream[pos:pos + k], "little")
        pos += k
        if c >> 3:
            r = (-r) % (1 << 64)
        prev = (prev + r) % (1 << 64)
        out.append(prev)
    return out


def gfc_encode(values: Sequence[float]) -> bytes:
    return gfc_encode_bits([_bits(v) for v in values])
