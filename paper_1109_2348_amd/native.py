"""Python binding of the bzgpu C ABI (include/bzgpu.h): argument marshalling
only.  Device memory and streams come from PyTorch; every stage runs in the
HIP kernels of libbzgpu.so.  There is no fallback: without the built library
(or without a GPU) these functions raise."""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbzgpu.so")

BZG_OK, BZG_EINVAL, BZG_ECAPACITY, BZG_EHIP, BZG_ENOMEM, BZG_EDATA = 0, -1, -3, -4, -5, -6
MAX_BLOCK = 1 << 21
TABLE_STRIDE = 1568


class BzgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bzgpu error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1109_2348_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, u64p, u32p = C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)
        L.bzg_create.restype = C.c_int
        L.bzg_create.argtypes = [C.POINTER(C.c_void_p), C.c_int]
        L.bzg_destroy.restype = None
        L.bzg_destroy.argtypes = [vp]
        L.bzg_last_error.restype = C.c_char_p
        L.bzg_last_error.argtypes = [vp]
        L.bzg_compress_bound.restype = C.c_uint64
        L.bzg_compress_bound.argtypes = [C.c_uint64, C.c_uint32]
        L.bwt_forward_batch.restype = C.c_int
        L.bwt_forward_batch.argtypes = [vp, vp, u64p, C.c_uint32, vp, vp, vp, vp]
        L.mtf_encode_batch.restype = C.c_int
        L.mtf_encode_batch.argtypes = [vp, vp, u64p, C.c_uint32, vp, vp, vp, vp]
        L.huffman_encode_batch.restype = C.c_int
        L.huffman_encode_batch.argtypes = [vp, vp, vp, vp, u64p, C.c_uint32, vp, u64p, vp, vp, vp]
        L.compress_blocks.restype = C.c_int
        L.compress_blocks.argtypes = [vp, vp, u64p, C.c_uint32, C.c_int, vp, C.c_uint64, u64p, u32p, vp]
        L.compress_batch.restype = C.c_int
        L.compress_batch.argtypes = [vp, vp, u64p, C.c_uint32, u32p, C.c_uint32, C.c_int, vp, u64p, u64p, vp]
        L.bzg_profile.restype = C.c_int
        L.bzg_profile.argtypes = [vp, C.c_int]
        L.bzg_profile_read.restype = C.c_int
        L.bzg_profile_read.argtypes = [vp, C.c_char_p, C.c_size_t]
        _lib = L
    return _lib


EXPORTS = ("bzg_create", "bzg_destroy", "bzg_last_error", "bzg_compress_bound", "bwt_forward_batch",
           "mtf_encode_batch", "huffman_encode_batch", "compress_blocks", "compress_batch", "bzg_profile",
           "bzg_profile_read")


class Profile:
    """Per-kernel HIP-event timing inside the library (diagnostics)."""

    def enable(self, ctx: "Context"):
        ctx.check(lib().bzg_profile(ctx.h, 1))

    def disable(self, ctx: "Context"):
        ctx.check(lib().bzg_profile(ctx.h, 0))

    def read(self, ctx: "Context") -> dict:
        buf = C.create_string_buffer(1 << 16)
        ctx.check(lib().bzg_profile_read(ctx.h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, launches, ms, nbytes = line.split()
            out[name] = {"launches": int(launches), "ms": float(ms), "bytes": float(nbytes)}
        return out


class Context:
    """A bzgpu context on one HIP device (owns the library's scratch memory)."""

    def __init__(self, device: Optional[int] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("bzgpu needs a HIP device")
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        rc = lib().bzg_create(C.byref(h), self.device)
        if rc != 0:
            raise BzgError(rc, "bzg_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().bzg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int):
        if rc != 0:
            raise BzgError(rc, lib().bzg_last_error(self.h).decode())


_contexts = {}


def context(device: Optional[int] = None) -> Context:
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _contexts:
        _contexts[d] = Context(d)
    return _contexts[d]


def _stream(dev: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _offs(offsets) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    if a.ndim != 1 or a.size < 1:
        raise ValueError("offsets must be a 1-D sequence with at least one entry")
    return a


def _u64p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _dev_u8(x: torch.Tensor) -> torch.Tensor:
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.uint8):
        raise TypeError("expected a uint8 tensor on the GPU")
    return x.contiguous()


def uniform_offsets(n: int, block_bytes: int) -> np.ndarray:
    if n == 0:
        return np.zeros(1, np.uint64)
    return np.array(list(range(0, n, block_bytes)) + [n], dtype=np.uint64)


def bwt(x: torch.Tensor, offsets, want_sa: bool = False,
        ctx: Optional[Context] = None) -> Tuple[torch.Tensor, torch.Tensor, Optional[torch.Tensor]]:
    """BWT of every block -> (last column uint8, primary int32[nb], sa int32 or None)."""
    x = _dev_u8(x)
    o = _offs(offsets)
    nb = o.size - 1
    ctx = ctx or context(x.device.index)
    L = torch.empty_like(x)
    prim = torch.empty(max(nb, 1), dtype=torch.int32, device=x.device)
    sa = torch.empty(x.numel(), dtype=torch.int32, device=x.device) if want_sa else None
    rc = lib().bwt_forward_batch(ctx.h, C.c_void_p(x.data_ptr()), _u64p(o), nb, C.c_void_p(L.data_ptr()),
                                 C.c_void_p(prim.data_ptr()), C.c_void_p(sa.data_ptr()) if sa is not None else None,
                                 _stream(x.device))
    ctx.check(rc)
    return L, prim[:nb], sa


def mtf(L: torch.Tensor, offsets, ctx: Optional[Context] = None):
    """MTF + RUNA/RUNB -> (syms int16 [n + nb] (uint16 values; block k at
    offsets[k] + k), nsyms int32[nb], inuse uint8[32 nb])."""
    L = _dev_u8(L)
    o = _offs(offsets)
    nb = o.size - 1
    ctx = ctx or context(L.device.index)
    syms = torch.zeros(L.numel() + nb + 1, dtype=torch.int16, device=L.device)
    nsyms = torch.zeros(max(nb, 1), dtype=torch.int32, device=L.device)
    inuse = torch.zeros(32 * max(nb, 1), dtype=torch.uint8, device=L.device)
    rc = lib().mtf_encode_batch(ctx.h, C.c_void_p(L.data_ptr()), _u64p(o), nb, C.c_void_p(syms.data_ptr()),
                                C.c_void_p(nsyms.data_ptr()), C.c_void_p(inuse.data_ptr()), _stream(L.device))
    ctx.check(rc)
    return syms, nsyms[:nb], inuse[:32 * nb]


def body_capacity(n_syms_cap: int) -> int:
    """Bytes that always hold a block body of at most n_syms_cap symbols."""
    groups = (n_syms_cap + 49) // 50
    bits = 16 + 256 + 18 + groups * 6 + 6 * (5 + 258 * 33) + n_syms_cap * 17
    return ((bits + 7) // 8 + 3) // 4 * 4


def huffman(syms: torch.Tensor, nsyms: torch.Tensor, inuse: torch.Tensor, sym_offsets,
            out_offsets=None, want_tables: bool = False, ctx: Optional[Context] = None):
    """Tables + packing -> (out uint8, out_offsets uint64, nbits int64[nb], tables uint8 or None)."""
    so = _offs(sym_offsets)
    nb = so.size - 1
    if out_offsets is None:
        caps = [body_capacity(int(so[k + 1] - so[k])) for k in range(nb)]
        out_offsets = np.zeros(nb + 1, np.uint64)
        out_offsets[1:] = np.cumsum(caps)
    oo = _offs(out_offsets)
    dev = syms.device
    ctx = ctx or context(dev.index)
    out = torch.zeros(max(int(oo[-1]), 4), dtype=torch.uint8, device=dev)
    nbits = torch.zeros(max(nb, 1), dtype=torch.int64, device=dev)
    tabs = torch.zeros(TABLE_STRIDE * max(nb, 1), dtype=torch.uint8, device=dev) if want_tables else None
    rc = lib().huffman_encode_batch(ctx.h, C.c_void_p(syms.data_ptr()), C.c_void_p(nsyms.data_ptr()),
                                    C.c_void_p(inuse.data_ptr()), _u64p(so), nb, C.c_void_p(out.data_ptr()),
                                    _u64p(oo), C.c_void_p(nbits.data_ptr()),
                                    C.c_void_p(tabs.data_ptr()) if tabs is not None else None, _stream(dev))
    ctx.check(rc)
    return out, oo, nbits[:nb], tabs


def compress_bound(n_bytes: int, n_blocks: int) -> int:
    return int(lib().bzg_compress_bound(n_bytes, n_blocks))


class Compressor:
    """Reusable compress_blocks caller: keeps the output buffer between calls.
    ctx: the library context (default: the device's shared one; give each
    host thread that should overlap with others a Context of its own)."""

    def __init__(self, device: Optional[int] = None, ctx: Optional[Context] = None):
        self.ctx = ctx or context(device)
        self.out = None
        self.out_bytes = C.c_uint64(0)
        self.n_blocks = C.c_uint32(0)

    def __call__(self, x: torch.Tensor, offsets=None, level: int = 9, block_bytes: Optional[int] = None):
        x = _dev_u8(x)
        if offsets is None:
            offsets = uniform_offsets(x.numel(), block_bytes or 100000 * level)
        o = _offs(offsets)
        nb = o.size - 1
        need = compress_bound(int(o[-1] - o[0]) if nb else 0, nb)
        if self.out is None or self.out.numel() < need or self.out.device != x.device:
            self.out = torch.empty(need, dtype=torch.uint8, device=x.device)
        rc = lib().compress_blocks(self.ctx.h, C.c_void_p(x.data_ptr()), _u64p(o), nb, level,
                                   C.c_void_p(self.out.data_ptr()), self.out.numel(), C.byref(self.out_bytes),
                                   C.byref(self.n_blocks), _stream(x.device))
        self.ctx.check(rc)
        return self.out[: self.out_bytes.value]


def compress(x: torch.Tensor, offsets=None, level: int = 9, block_bytes: Optional[int] = None) -> torch.Tensor:
    """Whole-pipeline compression of the blocks of x into one bzip2 stream
    (a uint8 tensor on x's device)."""
    return Compressor(x.device.index)(x, offsets, level, block_bytes).clone()


class BatchCompressor:
    """Reusable compress_batch caller: many requests, one stream each, all
    blocks through every stage together.  Keeps its output buffer.  ctx as
    for Compressor."""

    def __init__(self, device: Optional[int] = None, ctx: Optional[Context] = None):
        self.ctx = ctx or context(device)
        self.out = None

    def __call__(self, x: torch.Tensor, offsets, req_blocks, level: int = 9):
        """x: all requests' bytes on the GPU; offsets: block boundaries in x;
        req_blocks: n_req+1 block indices (request r = blocks
        [req_blocks[r], req_blocks[r+1])).  Returns one uint8 tensor view per
        request (valid until the next call)."""
        x = _dev_u8(x)
        o = _offs(offsets)
        rq = np.ascontiguousarray(np.asarray(req_blocks, dtype=np.uint32))
        nb, nr = o.size - 1, rq.size - 1
        if nr < 0:
            raise ValueError("req_blocks needs at least one entry")
        ok = rq.size and int(rq[0]) == 0 and int(rq[-1]) == nb and bool(np.all(np.diff(rq.astype(np.int64)) >= 0))
        ok = ok and bool(np.all(np.diff(o.astype(np.int64)) >= 0))
        # ranges the library will reject get no output space
        caps = [(compress_bound(int(o[rq[r + 1]]) - int(o[rq[r]]), int(rq[r + 1]) - int(rq[r])) + 3) & ~3
                if ok else 0 for r in range(nr)]
        oo = np.zeros(nr + 1, np.uint64)
        oo[1:] = np.cumsum(caps, dtype=np.uint64)
        need = max(int(oo[-1]), 4)
        if self.out is None or self.out.numel() < need or self.out.device != x.device:
            self.out = torch.empty(need, dtype=torch.uint8, device=x.device)
        ob = np.zeros(max(nr, 1), np.uint64)
        rc = lib().compress_batch(self.ctx.h, C.c_void_p(x.data_ptr()), _u64p(o), nb,
                                  rq.ctypes.data_as(C.POINTER(C.c_uint32)), nr, level,
                                  C.c_void_p(self.out.data_ptr()), _u64p(oo), _u64p(ob), _stream(x.device))
        self.ctx.check(rc)
        return [self.out[int(oo[r]): int(oo[r]) + int(ob[r])] for r in range(nr)]


def compress_batch(x: torch.Tensor, offsets, req_blocks, level: int = 9):
    """One bzip2 stream per request (list of uint8 tensors on x's device)."""
    return [z.clone() for z in BatchCompressor(x.device.index)(x, offsets, req_blocks, level)]
