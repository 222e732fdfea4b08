"""Pins of the field-codec oracle (Sec. 2.1 null suppression and Elias
delta, Sec. 3.5 GFC-style float delta), on the CPU."""

import math
import os
import random
import struct

from oracle import fields as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "elias_delta.txt")


def _golden():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        x, code = line.split()
        out.append((int(x), code))
    return out


def test_elias_delta_textbook_codewords():
    for x, code in _golden():
        assert F.edelta_code(x) == code, x


def test_elias_delta_stream_layout_by_hand():
    # values 0, 1, 7 are coded as x = 1, 2, 8: "1" "0100" "00100000" = 13
    # bits, MSB first in word 0: 1010 0001 0000 0000 ... = 0xA1000000
    z = F.edelta_encode([0, 1, 7])
    assert z[:16] == struct.pack("<QQ", 3, 13)
    assert z[16:24] == struct.pack("<Q", 0)  # index: value 0 starts at bit 0
    assert z[24:] == struct.pack("<I", 0xA1000000)
    assert F.edelta_decode(z) == [0, 1, 7]


def test_null_suppression_by_hand():
    vals = [0, 255, 256, 65535, 65536, 1 << 24, (1 << 32) - 1]
    # bytes needed 1 1 2 2 3 4 4 -> codes 0 0 1 1 2 3 3, four per byte, low
    # bits first: 0 | 0<<2 | 1<<4 | 1<<6 = 0x50, 2 | 3<<2 | 3<<4 = 0x3E
    want = struct.pack("<Q", 7) + bytes([0x50, 0x3E]) + bytes.fromhex(
        "00" "ff" "0001" "ffff" "000001" "00000001" "ffffffff")
    assert F.ns_encode(vals) == want
    assert F.ns_decode(want) == vals


def test_gfc_by_hand():
    # 1.0 = 0x3FF0000000000000: residual itself, no leading zero byte -> code 0, 8 bytes
    # 1.0 again: residual 0 -> 7 leading zero bytes (at most 7) -> code 7, one byte 00
    # 2.0 = 0x4000000000000000: residual 0x0010000000000000 -> code 1, 7 bytes
    # 1.0: residual -0x0010000000000000 -> sign, code 8 | 1 = 9, 7 bytes
    z = F.gfc_encode([1.0, 1.0, 2.0, 1.0])
    codes = bytes([0x70, 0x91])
    data = (0x3FF0000000000000).to_bytes(8, "little") + b"\x00" + \
        (0x0010000000000000).to_bytes(8, "little")[:7] * 2
    assert z == struct.pack("<Q", 4) + codes + data
    assert F.gfc_decode_bits(z) == [0x3FF0000000000000, 0x3FF0000000000000, 0x4000000000000000,
                                    0x3FF0000000000000]


def test_round_trips_random():
    rnd = random.Random(3)
    ints = [rnd.choice([0, 1, 2, 255, 256, 70000, (1 << 32) - 1, rnd.getrandbits(32), rnd.getrandbits(9)])
            for _ in range(3000)]
    assert F.ns_decode(F.ns_encode(ints)) == ints
    assert F.edelta_decode(F.edelta_encode(ints)) == ints
    specials = [0.0, -0.0, math.inf, -math.inf, float("nan"), 5e-324, 1.7976931348623157e308]
    vals = [rnd.choice(specials) if rnd.random() < 0.05 else rnd.gauss(0, 1e3) for _ in range(3000)]
    bits = [struct.unpack("<Q", struct.pack("<d", v))[0] for v in vals]
    assert F.gfc_decode_bits(F.gfc_encode(vals)) == bits


def test_lengths_are_the_definitions():
    for x in range(1, 5000):
        n = int(math.log2(x))
        m = int(math.log2(n + 1))
        assert len(F.edelta_code(x)) == n + 2 * m + 1
    for v in [0, 1, 255, 256, 65535, 65536, (1 << 24) - 1, 1 << 24]:
        assert F.ns_bytes(v) == max(1, (v.bit_length() + 7) // 8)
