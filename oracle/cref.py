"""ctypes loader for the tier-1 C oracle (``ref.c``).  Test infrastructure
only: the tests, the smoke check and the benchmark's CPU-baseline leg load
it; the product package never does."""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ref.c")
LIB = os.path.join(HERE, "libbzref.so")

MAXA, MAXG = 258, 6


def build(force: bool = True) -> str:
    """Compile ref.c with gcc (plain -O2, pthreads)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        u8p, u16p, u32p, u64p = (C.POINTER(C.c_uint8), C.POINTER(C.c_uint16),
                                 C.POINTER(C.c_uint32), C.POINTER(C.c_uint64))
        L.ref_crc32.restype = C.c_uint32
        L.ref_crc32.argtypes = [u8p, C.c_uint64]
        L.ref_rle1.restype = C.c_uint64
        L.ref_rle1.argtypes = [u8p, C.c_uint64, u8p]
        L.ref_bwt.restype = C.c_int64
        L.ref_bwt.argtypes = [u8p, C.c_uint32, u32p, u8p]
        L.ref_check_sa.restype = C.c_int64
        L.ref_check_sa.argtypes = [u8p, C.c_uint32, u32p]
        L.ref_cyclic_period.restype = C.c_uint32
        L.ref_cyclic_period.argtypes = [u8p, C.c_uint32]
        L.ref_mtf_zrle.restype = C.c_uint32
        L.ref_mtf_zrle.argtypes = [u8p, C.c_uint32, u16p, u8p, u32p, u8p]
        L.ref_huffman_lengths.restype = None
        L.ref_huffman_lengths.argtypes = [u32p, C.c_int, u8p]
        L.ref_tables.restype = C.c_int
        L.ref_tables.argtypes = [u16p, C.c_uint32, C.c_int, u8p, u8p]
        L.ref_rle1_len.restype = C.c_uint64
        L.ref_rle1_len.argtypes = [u8p, C.c_uint64]
        L.ref_split_blocks.restype = C.c_int64
        L.ref_split_blocks.argtypes = [u8p, u64p, C.c_uint32, C.c_uint64, u64p, C.c_uint64]
        L.ref_compress.restype = C.c_int64
        L.ref_compress.argtypes = [u8p, u64p, C.c_uint32, C.c_int, u8p, C.c_uint64, u64p, C.c_int]
        L.ref_compress_fixed.restype = C.c_int64
        L.ref_compress_fixed.argtypes = [u8p, u64p, C.c_uint32, C.c_int, u8p, C.c_int, u8p, C.c_uint64, u64p,
                                         C.c_int]
        L.ref_body.restype = C.c_int64
        L.ref_body.argtypes = [u16p, C.c_uint32, u8p, u8p, C.c_uint64, u8p, u8p,
                               C.POINTER(C.c_int)]
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(C.POINTER(t))


def _u8(x) -> np.ndarray:
    return np.ascontiguousarray(np.frombuffer(bytes(x), dtype=np.uint8)) if not isinstance(
        x, np.ndarray) else np.ascontiguousarray(x, dtype=np.uint8)


def crc32(data) -> int:
    a = _u8(data)
    return int(lib().ref_crc32(_p(a, C.c_uint8), a.size))


def rle1(data) -> np.ndarray:
    a = _u8(data)
    out = np.zeros(5 * ((a.size + 3) // 4) + 1, np.uint8)
    m = lib().ref_rle1(_p(a, C.c_uint8), a.size, _p(out, C.c_uint8))
    return out[:m].copy()


def bwt(data):
    """Returns (sa uint32[n], last uint8[n], orig_ptr)."""
    a = _u8(data)
    sa = np.zeros(a.size, np.uint32)
    last = np.zeros(a.size, np.uint8)
    optr = lib().ref_bwt(_p(a, C.c_uint8), a.size, _p(sa, C.c_uint32), _p(last, C.c_uint8))
    if optr < 0:
        raise ValueError("bwt failed")
    return sa, last, int(optr)


def check_sa(data, sa) -> int:
    """-1 when sa is the sorted rotation order, else the first bad row."""
    a = _u8(data)
    s = np.ascontiguousarray(sa, dtype=np.uint32)
    return int(lib().ref_check_sa(_p(a, C.c_uint8), a.size, _p(s, C.c_uint32)))


def cyclic_period(data) -> int:
    a = _u8(data)
    return int(lib().ref_cyclic_period(_p(a, C.c_uint8), a.size))


def mtf_zrle(last):
    """Returns (syms uint16[], used uint8[256] flags, n_inuse, mtf uint8[n])."""
    a = _u8(last)
    out = np.zeros(a.size + 1, np.uint16)
    used = np.zeros(256, np.uint8)
    mtf = np.zeros(max(a.size, 1), np.uint8)
    nu = C.c_uint32(0)
    ns = lib().ref_mtf_zrle(_p(a, C.c_uint8), a.size, _p(out, C.c_uint16), _p(used, C.c_uint8),
                            C.byref(nu), _p(mtf, C.c_uint8))
    return out[:ns].copy(), used, int(nu.value), mtf[:a.size].copy()


def huffman_lengths(freq) -> np.ndarray:
    f = np.ascontiguousarray(freq, dtype=np.uint32)
    out = np.zeros(f.size, np.uint8)
    lib().ref_huffman_lengths(_p(f, C.c_uint32), f.size, _p(out, C.c_uint8))
    return out


def tables(syms, alpha_size: int):
    """Returns (lens[G][alpha], sel[nsel])."""
    s = np.ascontiguousarray(syms, dtype=np.uint16)
    lens = np.zeros(MAXG * MAXA, np.uint8)
    nsel = (s.size + 49) // 50
    sel = np.zeros(max(nsel, 1), np.uint8)
    g = lib().ref_tables(_p(s, C.c_uint16), s.size, alpha_size, _p(lens, C.c_uint8),
                         _p(sel, C.c_uint8))
    return lens.reshape(MAXG, MAXA)[:g, :alpha_size].copy(), sel[:nsel].copy()


def body(syms, used):
    """Block body (symbol map .. last code) as (bytes, nbits, lens, sel)."""
    s = np.ascontiguousarray(syms, dtype=np.uint16)
    u = np.ascontiguousarray(used, dtype=np.uint8)
    cap = 4096 + 3 * s.size
    out = np.zeros(cap, np.uint8)
    lens = np.zeros(MAXG * MAXA, np.uint8)
    nsel = (s.size + 49) // 50
    sel = np.zeros(max(nsel, 1), np.uint8)
    g = C.c_int(0)
    bits = lib().ref_body(_p(s, C.c_uint16), s.size, _p(u, C.c_uint8), _p(out, C.c_uint8), cap,
                          _p(lens, C.c_uint8), _p(sel, C.c_uint8), C.byref(g))
    if bits < 0:
        raise ValueError("body capacity")
    a = int(u.astype(bool).sum()) + 2
    return (out[:(bits + 7) // 8].tobytes(), int(bits),
            lens.reshape(MAXG, MAXA)[:g.value, :a].copy(), sel[:nsel].copy())


def split_blocks(data, offsets, limit: int) -> np.ndarray:
    a = _u8(data)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    nb = offs.size - 1
    max_out = nb + a.size // 50000 + 2
    out = np.zeros(max_out + 1, np.uint64)
    m = lib().ref_split_blocks(_p(a, C.c_uint8), _p(offs, C.c_uint64), nb, limit,
                               _p(out, C.c_uint64), max_out)
    if m < 0:
        raise ValueError("split")
    return out[:m + 1].copy()


SAMPLE_SYMS = 900000


def tables_from_sample(blocks):
    """Precomputed tables from sample blocks (see ref.tables_from_sample):
    every block's symbols through BWT and MTF + RUNA/RUNB (no RLE1), mapped
    to the 258-symbol alphabet (EOB -> 257), pooled, cut to the first
    SAMPLE_SYMS, and given the table heuristic as one block.  Returns lens
    uint8[G][258]."""
    pooled = []
    for blk in blocks:
        if len(blk) == 0:
            continue
        _, last, _ = bwt(blk)
        syms, _, nu, _ = mtf_zrle(last)
        syms = syms.astype(np.uint16)
        syms[-1] = MAXA - 1  # EOB
        pooled.append(syms)
    allsyms = np.concatenate(pooled)[:SAMPLE_SYMS] if pooled else np.zeros(0, np.uint16)
    lens, _ = tables(allsyms, MAXA)
    return lens


def compress(data, offsets=None, level: int = 9, threads: int = 1, fixed=None) -> bytes:
    """One bzip2 stream; fixed: optional precomputed tables uint8[G][258]."""
    a = _u8(data)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8).reshape(-1, MAXA)
    if offsets is None:
        bb = 100000 * level
        offsets = list(range(0, a.size, bb)) + [a.size] if a.size else [0]
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    nb = offs.size - 1
    cap = 64 + a.size + a.size // 4 + 4096 * max(nb, 1)
    out = np.zeros(cap, np.uint8)
    need = C.c_uint64(0)
    while True:
        if fx is None:
            r = lib().ref_compress(_p(a, C.c_uint8) if a.size else None, _p(offs, C.c_uint64), nb,
                                   level, _p(out, C.c_uint8), cap, C.byref(need), threads)
        else:
            r = lib().ref_compress_fixed(_p(a, C.c_uint8) if a.size else None, _p(offs, C.c_uint64), nb,
                                         level, _p(fx, C.c_uint8), fx.shape[0], _p(out, C.c_uint8), cap,
                                         C.byref(need), threads)
        if r < 0:
            raise ValueError("oracle compress failed")
        if r > 0:
            return out[:r].tobytes()
        cap = int(need.value)
        out = np.zeros(cap, np.uint8)
