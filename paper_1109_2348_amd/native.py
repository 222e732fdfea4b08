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

BZG_OK, BZG_EINVAL, BZG_EWORKSPACE, BZG_ECAPACITY, BZG_EHIP, BZG_ENOMEM, BZG_EDATA, BZG_EINTERNAL = (
    0, -1, -2, -3, -4, -5, -6, -7)
CALL_BWT, CALL_MTF, CALL_HUFFMAN, CALL_COMPRESS = 1, 2, 3, 4
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
        vp, u64p, u32p, i = C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.c_int
        sz, u32, u64 = C.c_size_t, C.c_uint32, C.c_uint64
        L.bzg_create.restype = i
        L.bzg_create.argtypes = [C.POINTER(C.c_void_p), i, C.c_char_p]
        L.bzg_destroy.restype = None
        L.bzg_destroy.argtypes = [vp]
        L.bzg_last_error.restype = C.c_char_p
        L.bzg_last_error.argtypes = [vp]
        L.bzg_check.restype = i
        L.bzg_check.argtypes = [vp, vp]
        L.bzg_workspace_size.restype = i
        L.bzg_workspace_size.argtypes = [vp, i, u64p, u32, i, u32, C.POINTER(C.c_size_t)]
        L.bzg_compress_bound.restype = u64
        L.bzg_compress_bound.argtypes = [u64, u32]
        L.bwt_forward_batch.restype = i
        L.bwt_forward_batch.argtypes = [vp, vp, vp, u64p, u32, vp, vp, vp, vp, sz, vp]
        L.mtf_encode_batch.restype = i
        L.mtf_encode_batch.argtypes = [vp, vp, vp, u64p, u32, vp, vp, vp, vp, sz, vp]
        L.huffman_encode_batch.restype = i
        L.huffman_encode_batch.argtypes = [vp, vp, vp, vp, vp, u64p, u32, vp, vp, u64p, vp, vp, vp, sz, vp]
        L.compress_blocks.restype = i
        L.compress_blocks.argtypes = [vp, vp, vp, u64p, u32, i, vp, u64, vp, vp, vp, sz, vp]
        L.compress_batch.restype = i
        L.compress_batch.argtypes = [vp, vp, vp, u64p, u32, vp, u32p, u32, i, vp, vp, u64p, vp, vp, sz, vp]
        L.compress_blocks_noalloc.restype = i
        L.compress_blocks_noalloc.argtypes = [vp, vp, vp, u64p, u32, i, vp, u64, vp, vp, vp]
        L.decompress.restype = i
        L.decompress.argtypes = [vp, vp, u64, vp, u64, vp, vp]
        L.bzg_set_tune.restype = i
        L.bzg_set_tune.argtypes = [vp, u32, u32, u32]
        L.bzg_tune.restype = i
        L.bzg_tune.argtypes = [vp, vp, u64p, u32, i, vp, u32p]
        L.bzg_field_bound.restype = u64
        L.bzg_field_bound.argtypes = [i, u64]
        L.field_encode.restype = i
        L.field_encode.argtypes = [vp, i, vp, u64, vp, u64, vp, vp]
        L.field_decode.restype = i
        L.field_decode.argtypes = [vp, i, vp, u64, vp, u64, vp]
        L.bzg_set_fixed_tables.restype = i
        L.bzg_set_fixed_tables.argtypes = [vp, vp, i]
        L.compress_host.restype = i
        L.compress_host.argtypes = [vp, vp, u64, u32, i, u64, vp, u64, C.POINTER(C.c_uint64), vp]
        L.bzg_profile.restype = i
        L.bzg_profile.argtypes = [vp, i]
        L.bzg_profile_read.restype = i
        L.bzg_profile_read.argtypes = [vp, C.c_char_p, C.c_size_t]
        _lib = L
    return _lib


EXPORTS = ("bzg_create", "bzg_destroy", "bzg_last_error", "bzg_check", "bzg_workspace_size", "bzg_compress_bound",
           "bwt_forward_batch", "mtf_encode_batch", "huffman_encode_batch", "compress_blocks", "compress_batch",
           "compress_blocks_noalloc", "compress_host", "bzg_set_fixed_tables", "decompress", "bzg_field_bound",
           "field_encode", "field_decode", "bzg_set_tune", "bzg_tune", "bzg_profile", "bzg_profile_read")


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

    def __init__(self, device: Optional[int] = None, tune_cache: Optional[str] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("bzgpu needs a HIP device")
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        rc = lib().bzg_create(C.byref(h), self.device, tune_cache.encode() if tune_cache else None)
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

    def sync_check(self, stream: C.c_void_p):
        """Waits for the stream and raises the errors the kernels recorded."""
        self.check(lib().bzg_check(self.h, stream))

    def set_tune(self, mtf_chunk: int = 0, assign_groups: int = 0, count_steps: int = 0):
        """Fixes the launch parameters (0 = tuned or built-in choice)."""
        self.check(lib().bzg_set_tune(self.h, mtf_chunk, assign_groups, count_steps))

    def tune(self, x: torch.Tensor, offsets, level: int = 9) -> Tuple[int, int, int]:
        """Times every launch-parameter point on this batch (outputs checked
        byte for byte) and keeps the fastest for its size bucket (and in the
        tune cache file, when the context has one)."""
        x = _dev_u8(x)
        o = _offs(offsets)
        chosen = (C.c_uint32 * 3)()
        self.check(lib().bzg_tune(self.h, _vp(x), _u64p(o), o.size - 1, level, _stream(x.device), chosen))
        return tuple(int(v) for v in chosen)

    def set_fixed_tables(self, lens: Optional[np.ndarray]):
        """Precomputed Huffman tables (G x 258 code lengths, G = 2..6) for
        every later call on this context; None returns to built tables."""
        if lens is None:
            self.check(lib().bzg_set_fixed_tables(self.h, None, 0))
            return
        a = np.ascontiguousarray(np.asarray(lens, dtype=np.uint8))
        if a.ndim != 2 or a.shape[1] != 258:
            raise ValueError("expected a G x 258 array of code lengths")
        self.check(lib().bzg_set_fixed_tables(self.h, C.c_void_p(a.ctypes.data), a.shape[0]))

    def workspace_size(self, call: int, offsets, n_blocks: Optional[int] = None, level: int = 9,
                       n_req: int = 1) -> int:
        o = _offs(offsets)
        nb = o.size - 1 if n_blocks is None else n_blocks
        out = C.c_size_t(0)
        self.check(lib().bzg_workspace_size(self.h, call, _u64p(o), nb, level, n_req, C.byref(out)))
        return int(out.value)


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


def _dev_u64(a: np.ndarray, dev) -> torch.Tensor:
    """A device copy of a host uint64 table (passed to the library as its d_ table)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(dev)


def _vp(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def bwt(x: torch.Tensor, offsets, want_sa: bool = False, ctx: Optional[Context] = None,
        check: bool = True) -> Tuple[torch.Tensor, torch.Tensor, Optional[torch.Tensor]]:
    """BWT of every block -> (last column uint8, primary int32[nb], sa int32 or None)."""
    x = _dev_u8(x)
    o = _offs(offsets)
    nb = o.size - 1
    ctx = ctx or context(x.device.index)
    L = torch.empty_like(x)
    prim = torch.empty(max(nb, 1), dtype=torch.int32, device=x.device)
    sa = torch.empty(x.numel(), dtype=torch.int32, device=x.device) if want_sa else None
    d_o = _dev_u64(o, x.device)
    st = _stream(x.device)
    rc = lib().bwt_forward_batch(ctx.h, _vp(x), _vp(d_o), _u64p(o), nb, _vp(L), _vp(prim), _vp(sa), None, 0, st)
    ctx.check(rc)
    if check:
        ctx.sync_check(st)
    return L, prim[:nb], sa


def mtf(L: torch.Tensor, offsets, ctx: Optional[Context] = None, check: bool = True):
    """MTF + RUNA/RUNB -> (syms int16 [n + nb] (uint16 values; block k at
    offsets[k] + k), nsyms int32[nb], inuse uint8[32 nb])."""
    L = _dev_u8(L)
    o = _offs(offsets)
    nb = o.size - 1
    ctx = ctx or context(L.device.index)
    syms = torch.zeros(L.numel() + nb + 1, dtype=torch.int16, device=L.device)
    nsyms = torch.zeros(max(nb, 1), dtype=torch.int32, device=L.device)
    inuse = torch.zeros(32 * max(nb, 1), dtype=torch.uint8, device=L.device)
    d_o = _dev_u64(o, L.device)
    st = _stream(L.device)
    rc = lib().mtf_encode_batch(ctx.h, _vp(L), _vp(d_o), _u64p(o), nb, _vp(syms), _vp(nsyms), _vp(inuse), None, 0, st)
    ctx.check(rc)
    if check:
        ctx.sync_check(st)
    return syms, nsyms[:nb], inuse[:32 * nb]


def body_capacity(n_syms_cap: int) -> int:
    """Bytes that always hold a block body of at most n_syms_cap symbols."""
    groups = (n_syms_cap + 49) // 50
    bits = 16 + 256 + 18 + groups * 6 + 6 * (5 + 258 * 33) + n_syms_cap * 17
    return ((bits + 7) // 8 + 3) // 4 * 4


def huffman(syms: torch.Tensor, nsyms: torch.Tensor, inuse: torch.Tensor, sym_offsets,
            out_offsets=None, want_tables: bool = False, ctx: Optional[Context] = None, check: bool = True):
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
    d_so, d_oo = _dev_u64(so, dev), _dev_u64(oo, dev)
    st = _stream(dev)
    rc = lib().huffman_encode_batch(ctx.h, _vp(syms), _vp(nsyms), _vp(inuse), _vp(d_so), _u64p(so), nb, _vp(out),
                                    _vp(d_oo), _u64p(oo), _vp(nbits), _vp(tabs), None, 0, st)
    ctx.check(rc)
    if check:
        ctx.sync_check(st)
    return out, oo, nbits[:nb], tabs


SAMPLE_SYMS = 900_000  # symbols a table sample contributes at most


def fixed_tables_from_sample(x: torch.Tensor, offsets, ctx: Optional[Context] = None) -> np.ndarray:
    """Precomputed Huffman tables from sample blocks on the GPU: the blocks'
    BWT and MTF + RUNA/RUNB symbols (no RLE1), mapped to the alphabet of a
    block with every byte in use (each block's EOB becomes 257), pooled and
    cut to the first SAMPLE_SYMS symbols, then this library's table
    heuristic on them as one block.  Returns uint8[G][258] for
    Context.set_fixed_tables.  ctx must not have fixed tables set."""
    x = _dev_u8(x)
    o = _offs(offsets)
    ctx = ctx or context(x.device.index)
    L, _, _ = bwt(x, o, ctx=ctx)
    syms, nsyms, _ = mtf(L, o, ctx=ctx)
    ns = nsyms.cpu().numpy().astype(np.int64)
    nb = o.size - 1
    starts = o[:-1].astype(np.int64) + np.arange(nb)
    keep = ns > 0
    idx = np.concatenate([np.arange(a, a + n) for a, n in zip(starts[keep], ns[keep])]) if keep.any() \
        else np.zeros(0, np.int64)
    eob = np.cumsum(ns[keep]) - 1
    pooled = syms[torch.from_numpy(idx).to(x.device)].clone()
    pooled[torch.from_numpy(eob).to(x.device)] = 257
    pooled = pooled[:SAMPLE_SYMS].contiguous()
    total = int(pooled.numel())
    if total == 0:
        raise ValueError("the sample holds no symbols")
    cnt = torch.tensor([total], dtype=torch.int32, device=x.device)
    inuse = torch.full((32,), 0xFF, dtype=torch.uint8, device=x.device)
    _, _, _, tabs = huffman(pooled, cnt, inuse, [0, total], want_tables=True, ctx=ctx)
    t = tabs.cpu().numpy()
    g = int(t[0])
    return t[16:16 + 258 * g].reshape(g, 258).copy()


def compress_bound(n_bytes: int, n_blocks: int) -> int:
    return int(lib().bzg_compress_bound(n_bytes, n_blocks))


class Compressor:
    """Reusable compress_blocks caller: keeps the output buffer between calls.
    ctx: the library context (default: the device's shared one; give each
    host thread that should overlap with others a Context of its own)."""

    def __init__(self, device: Optional[int] = None, ctx: Optional[Context] = None):
        self.ctx = ctx or context(device)
        self.out = None
        self.out_bytes = None
        self.n_blocks = None

    def enqueue(self, x: torch.Tensor, offsets, level: int = 9, d_offsets: Optional[torch.Tensor] = None,
                ws: Optional[torch.Tensor] = None):
        """Enqueues one compress_blocks call on the current stream and returns
        at once (no host wait).  d_offsets: a device copy of offsets (int64),
        made here when None; ws: a caller workspace (uint8), the context's
        pool when None.  The stream's length lands in self.out_bytes[0]."""
        o = _offs(offsets)
        nb = o.size - 1
        need = compress_bound(int(o[-1] - o[0]) if nb else 0, nb)
        if self.out is None or self.out.numel() < need or self.out.device != x.device:
            self.out = torch.empty(need, dtype=torch.uint8, device=x.device)
            self.out_bytes = torch.zeros(1, dtype=torch.int64, device=x.device)
            self.n_blocks = torch.zeros(1, dtype=torch.int32, device=x.device)
        if d_offsets is None:
            d_offsets = _dev_u64(o, x.device)
        rc = lib().compress_blocks(self.ctx.h, _vp(x) if x.numel() else None, _vp(d_offsets), _u64p(o), nb, level,
                                   _vp(self.out), self.out.numel(), _vp(self.out_bytes), _vp(self.n_blocks), _vp(ws),
                                   ws.numel() if ws is not None else 0, _stream(x.device))
        self.ctx.check(rc)
        return d_offsets

    def __call__(self, x: torch.Tensor, offsets=None, level: int = 9, block_bytes: Optional[int] = None):
        """Compresses and waits; returns a view of the kept output buffer,
        valid until this compressor's next call (clone it to keep it)."""
        x = _dev_u8(x)
        if offsets is None:
            offsets = uniform_offsets(x.numel(), block_bytes or 100000 * level)
        self.enqueue(x, offsets, level)
        self.ctx.sync_check(_stream(x.device))
        return self.out[: int(self.out_bytes.item())]


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

    def plan(self, offsets, req_blocks):
        """Output offsets for these requests (each range holds the stream's bound)."""
        o = _offs(offsets)
        rq = np.ascontiguousarray(np.asarray(req_blocks, dtype=np.uint32))
        nb, nr = o.size - 1, rq.size - 1
        ok = rq.size and int(rq[0]) == 0 and int(rq[-1]) == nb and bool(np.all(np.diff(rq.astype(np.int64)) >= 0))
        ok = ok and bool(np.all(np.diff(o.astype(np.int64)) >= 0))
        # ranges the library will reject get no output space
        caps = [(compress_bound(int(o[rq[r + 1]]) - int(o[rq[r]]), int(rq[r + 1]) - int(rq[r])) + 3) & ~3
                if ok else 0 for r in range(nr)]
        oo = np.zeros(nr + 1, np.uint64)
        oo[1:] = np.cumsum(caps, dtype=np.uint64)
        return o, rq, oo

    def enqueue(self, x: torch.Tensor, offsets, req_blocks, level: int = 9, out_offsets=None):
        """Enqueues one compress_batch call (no host wait); returns
        (out_offsets, device stream lengths)."""
        o, rq, oo = self.plan(offsets, req_blocks)
        if out_offsets is not None:
            oo = _offs(out_offsets)
        nb, nr = o.size - 1, rq.size - 1
        need = max(int(oo[-1]), 4)
        if self.out is None or self.out.numel() < need or self.out.device != x.device:
            self.out = torch.empty(need, dtype=torch.uint8, device=x.device)
        ob = torch.zeros(max(nr, 1), dtype=torch.int64, device=x.device)
        rc = lib().compress_batch(self.ctx.h, _vp(x) if x.numel() else None, None, _u64p(o), nb, None,
                                  rq.ctypes.data_as(C.POINTER(C.c_uint32)), nr, level, _vp(self.out), None,
                                  _u64p(oo), _vp(ob), None, 0, _stream(x.device))
        self.ctx.check(rc)
        return oo, ob

    def __call__(self, x: torch.Tensor, offsets, req_blocks, level: int = 9):
        """x: all requests' bytes on the GPU; offsets: block boundaries in x;
        req_blocks: n_req+1 block indices (request r = blocks
        [req_blocks[r], req_blocks[r+1])).  Returns one uint8 tensor view per
        request (valid until the next call)."""
        x = _dev_u8(x)
        oo, ob = self.enqueue(x, offsets, req_blocks, level)
        self.ctx.sync_check(_stream(x.device))
        obh = ob.cpu().numpy()
        return [self.out[int(oo[r]): int(oo[r]) + int(obh[r])] for r in range(oo.size - 1)]


def compress_batch(x: torch.Tensor, offsets, req_blocks, level: int = 9):
    """One bzip2 stream per request (list of uint8 tensors on x's device)."""
    return [z.clone() for z in BatchCompressor(x.device.index)(x, offsets, req_blocks, level)]


def compress_host(data, level: int = 9, block_bytes: Optional[int] = None, chunk_bytes: Optional[int] = None,
                  out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> np.ndarray:
    """Compresses input that lives in host memory (bytes, a numpy array or a
    CPU tensor, pinned or not) chunk by chunk with the uploads, the kernels
    and the downloads overlapped; one bzip2 stream per chunk, concatenated.
    out: optional CPU uint8 tensor for the result (pinned for an overlapped
    download).  Returns a numpy view of the output."""
    if isinstance(data, torch.Tensor):
        if data.is_cuda or data.dtype != torch.uint8:
            raise TypeError("expected a uint8 tensor in host memory")
        src = data.contiguous()
        ptr, n = src.data_ptr(), src.numel()
    else:
        src = np.ascontiguousarray(np.frombuffer(data, np.uint8) if isinstance(data, (bytes, bytearray))
                                   else np.asarray(data, dtype=np.uint8)).reshape(-1)
        ptr, n = src.ctypes.data, src.size
    ctx = ctx or context()
    bb = block_bytes or 100000 * level
    blocks = max(1, -(-n // bb))
    cap = compress_bound(n, blocks) + 64 * (blocks + 1) + 64
    if out is None:
        out = torch.empty(cap, dtype=torch.uint8)
    elif out.is_cuda or out.dtype != torch.uint8 or out.numel() < 1:
        raise TypeError("out must be a uint8 tensor in host memory")
    got = C.c_uint64(0)
    dev = torch.device("cuda", ctx.device)
    ctx.check(lib().compress_host(ctx.h, C.c_void_p(ptr) if n else None, n, block_bytes or 0, level,
                                  chunk_bytes or 0, C.c_void_p(out.data_ptr()), out.numel(), C.byref(got),
                                  _stream(dev)))
    return out[: got.value].numpy()


def decompress(z: torch.Tensor, out_cap: Optional[int] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Decodes one bzip2 stream, or several one after another, on the GPU:
    returns the original bytes (uint8 tensor on z's device).  When out_cap
    (default 4x the input, at least 1 MiB) is too small, the call is repeated
    with the size the first attempt reported."""
    z = _dev_u8(z)
    ctx = ctx or context(z.device.index)
    st = _stream(z.device)
    cap = out_cap or max(4 * z.numel(), 1 << 20)
    nbytes = torch.zeros(1, dtype=torch.int64, device=z.device)
    for attempt in range(2):
        out = torch.empty(max(cap, 1), dtype=torch.uint8, device=z.device)
        ctx.check(lib().decompress(ctx.h, _vp(z), z.numel(), _vp(out), cap, _vp(nbytes), st))
        try:
            ctx.sync_check(st)
        except BzgError as e:
            if e.code != BZG_ECAPACITY or attempt:
                raise
            cap = int(nbytes.item())
            continue
        return out[: int(nbytes.item())]
    raise BzgError(BZG_ECAPACITY, "output size changed between attempts")


FIELD_NS32, FIELD_EDELTA32, FIELD_GFC64 = 1, 2, 3


def field_encode(values: torch.Tensor, codec: int, ctx: Optional[Context] = None) -> torch.Tensor:
    """One field of values (uint32 / int32 for NS32 and EDELTA32, float64 for
    GFC64) as a compressed stream (uint8 tensor on the same device)."""
    if not values.is_cuda:
        raise TypeError("values must be on the GPU")
    want = torch.float64 if codec == FIELD_GFC64 else (torch.int32, torch.uint32)
    if (values.dtype != want) if codec == FIELD_GFC64 else (values.dtype not in want):
        raise TypeError("values of the wrong type for this codec")
    v = values.contiguous()
    n = v.numel()
    ctx = ctx or context(v.device.index)
    cap = int(lib().bzg_field_bound(codec, n))
    out = torch.empty((cap + 7) // 8 * 8, dtype=torch.uint8, device=v.device)
    nb = torch.zeros(1, dtype=torch.int64, device=v.device)
    st = _stream(v.device)
    ctx.check(lib().field_encode(ctx.h, codec, _vp(v) if n else None, n, _vp(out), out.numel(), _vp(nb), st))
    ctx.sync_check(st)
    return out[: int(nb.item())]


def field_decode(z: torch.Tensor, codec: int, n: int, ctx: Optional[Context] = None) -> torch.Tensor:
    """Decodes n values of a field stream (int32 values, or float64 for GFC64)."""
    z = _dev_u8(z)
    zz = torch.empty((z.numel() + 7) // 8 * 8, dtype=torch.uint8, device=z.device)  # 8-byte aligned copy
    zz[: z.numel()] = z
    ctx = ctx or context(z.device.index)
    dt = torch.float64 if codec == FIELD_GFC64 else torch.int32
    out = torch.empty(max(n, 1), dtype=dt, device=z.device)
    st = _stream(z.device)
    ctx.check(lib().field_decode(ctx.h, codec, _vp(zz), z.numel(), _vp(out), n, st))
    ctx.sync_check(st)
    return out[:n]

