"""The whole compressor enqueued without host round trips: compress_blocks
with caller-owned device tables and workspace is captured into a HIP graph
and replayed; every replay's stream equals the oracle's, bit for bit (Sec. 4:
all stages on the device, no PCIe round trips between them)."""

import sys

import numpy as np
import pytest

from oracle import cref
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def test_compress_blocks_graph_replay_bit_exact():
    import torch
    from paper_1109_2348_amd import native
    b = W.config2(total=5 * 100000 + 4321, block=100000, seed=23)
    level = 1  # 100000-byte limit: text and uniform blocks may be cut
    ref = cref.compress(b.data, b.offsets, level=level, threads=16)
    _say(f"graph capture of compress_blocks: {b.data.size} B, {b.n_blocks} blocks, level {level}")
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(b.data).to(dev)
    o = np.ascontiguousarray(b.offsets, dtype=np.uint64)
    ctx = native.Context(0)
    comp = native.Compressor(ctx=ctx)
    ws = torch.empty(ctx.workspace_size(native.CALL_COMPRESS, o, level=level), dtype=torch.uint8, device=dev)
    d_o = native._dev_u64(o, dev)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):  # one eager call: sizes the output buffers
        comp.enqueue(x, o, level, d_offsets=d_o, ws=ws)
    torch.cuda.current_stream(dev).wait_stream(side)
    ctx.sync_check(native._stream(dev))
    assert comp.out[: int(comp.out_bytes.item())].cpu().numpy().tobytes() == ref
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        comp.enqueue(x, o, level, d_offsets=d_o, ws=ws)
    for rep in range(4):
        comp.out.zero_()  # eager work between replays
        comp.out_bytes.zero_()
        g.replay()
        ctx.sync_check(native._stream(dev))
        n = int(comp.out_bytes.item())
        z = comp.out[:n].cpu().numpy().tobytes()
        assert z == ref, f"replay {rep}: stream differs from the oracle"
    _say("4 replays bit-exact")


def test_calls_enqueue_without_waiting():
    """A call returns before its work is done: with the device kept busy by
    a long chain of kernels queued first, compress_blocks returns at once
    (with the caller's device tables and workspace, and with the library
    copying the host offsets itself), and the stream completes later."""
    import ctypes as C
    import time
    import torch
    from paper_1109_2348_amd import native
    dev = torch.device("cuda", 0)
    b = W.config2(total=3 * 100000, block=100000, seed=29)
    x = torch.from_numpy(b.data).to(dev)
    o = np.ascontiguousarray(b.offsets, dtype=np.uint64)
    ctx = native.Context(0)
    comp = native.Compressor(ctx=ctx)
    ref = cref.compress(b.data, b.offsets, level=9, threads=16)
    d_o = native._dev_u64(o, dev)
    ws = torch.empty(ctx.workspace_size(native.CALL_COMPRESS, o, level=9), dtype=torch.uint8, device=dev)
    comp.enqueue(x, o, 9, d_offsets=d_o, ws=ws)  # sizes the output buffers
    ctx.sync_check(native._stream(dev))
    st = native._stream(dev)
    for mode in ("caller tables and workspace", "library upload and pool"):
        a = torch.randn(4096, 4096, device=dev)
        torch.cuda.synchronize()
        for _ in range(40):  # tens of ms of queued work
            a = a @ a
            a = a / a.norm()
        t0 = time.perf_counter()
        if mode.startswith("caller"):
            rc = native.lib().compress_blocks(ctx.h, native._vp(x), native._vp(d_o), native._u64p(o), o.size - 1, 9,
                                              native._vp(comp.out), comp.out.numel(), native._vp(comp.out_bytes),
                                              None, native._vp(ws), ws.numel(), st)
        else:
            rc = native.lib().compress_blocks(ctx.h, native._vp(x), None, native._u64p(o), o.size - 1, 9,
                                              native._vp(comp.out), comp.out.numel(), native._vp(comp.out_bytes),
                                              None, None, 0, st)
        t_call = time.perf_counter() - t0
        ctx.check(rc)
        ctx.sync_check(st)
        t_all = time.perf_counter() - t0
        _say(f"{mode}: enqueue {t_call * 1e3:.2f} ms, until done {t_all * 1e3:.2f} ms")
        assert t_call < 0.5 * t_all
        z = comp.out[: int(comp.out_bytes.item())].cpu().numpy().tobytes()
        assert z == ref
