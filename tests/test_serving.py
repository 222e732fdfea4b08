"""Serving loop: scheduling logic on the CPU with a fake backend whose passes
are run by the oracle, and (GPU) each request's stream identical alone and in
the mix."""

import bz2
import random
import threading
import time

import numpy as np
import pytest

from oracle import cref
from paper_1109_2348_amd import serving as S
import workloads as W


def _budget(max_pass, workers, arena):
    return workers * (S.WORKSPACE_PER_BYTE * max_pass + S.WORKSPACE_FIXED) + arena


class FakeBackend:
    """Host arena; a pass compresses each request's arena bytes with the
    oracle, so a stream equal to the oracle's on the request's own bytes shows
    the pass read that request's live range and nothing else."""

    def __init__(self, delay=0.0, fail_on=None):
        self.delay, self.fail_on = delay, fail_on
        self.lock = threading.Lock()
        self.inflight = 0
        self.max_inflight = 0
        self.passes = []

    def arena(self, n):
        return np.zeros(n, np.uint8)

    def upload(self, arena, pos, data, ready=None):
        a = np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else data
        arena[pos:pos + a.size] = a

    def worker(self, i):
        def run(arena, offs, rq, level):
            with self.lock:
                self.inflight += 1
                self.max_inflight = max(self.max_inflight, self.inflight)
                self.passes.append(len(rq) - 1)
            try:
                if self.delay:
                    time.sleep(self.delay)
                out = []
                for r in range(len(rq) - 1):
                    a, e = int(rq[r]), int(rq[r + 1])
                    data = arena[int(offs[a]):int(offs[e])].copy() if e > a else np.zeros(0, np.uint8)
                    if self.fail_on is not None and data.size and data[0] == self.fail_on:
                        raise RuntimeError("injected pass failure")
                    o = offs[a:e + 1] - offs[a] if e > a else np.zeros(1, np.uint64)
                    out.append(cref.compress(data, o, level=level))
                return out
            finally:
                with self.lock:
                    self.inflight -= 1
        return run


def _payloads(n, seed, lo=0, hi=30000):
    rnd = random.Random(seed)
    out = []
    for i in range(n):
        k = rnd.randrange(lo, hi)
        kind = ("uniform", "text", "sparse")[i % 3]
        out.append(W.source_blocks(kind, [k], seed, indices=[i])[0] if k else np.zeros(0, np.uint8))
    return out


def test_ring_fifo_wrap_and_reclaim():
    r = S.Ring(100)
    a = r.alloc(40)
    b = r.alloc(40)
    assert (a[0], b[0]) == (0, 40)
    assert r.alloc(30) is None           # 20 left at the end, nothing freed yet
    r.free(b)                            # out of order: space not reclaimed
    assert r.alloc(30) is None
    r.free(a)                            # oldest freed -> everything reclaimed
    c = r.alloc(90)
    assert c[0] == 0
    d = r.alloc(10)
    assert d[0] == 90
    r.free(c)
    e = r.alloc(50)                      # wraps to the front
    assert e[0] == 0
    assert r.alloc(41) is None           # 40 free between head 50 and tail 90
    f = r.alloc(40)
    assert f[0] == 50
    assert r.alloc(1) is None            # full
    r.free(d)
    g = r.alloc(10)                      # tail moved to e at 0: the end is free again
    assert g[0] == 90
    assert r.used() == 100


def test_ring_random_never_overlaps():
    rnd = random.Random(1)
    r = S.Ring(1000)
    live = []
    for _ in range(5000):
        if live and (rnd.random() < 0.5 or len(live) > 20):
            e = live.pop(rnd.randrange(len(live)))
            r.free(e)
        else:
            e = r.alloc(rnd.randrange(1, 300))
            if e is not None:
                assert 0 <= e[0] < e[1] <= 1000
                for o in live:
                    assert e[1] <= o[0] or o[1] <= e[0], "overlapping live ranges"
                live.append(e)


def test_plan_pass_offsets():
    reqs = [S._Req(None, 250, 0.0, None, pos=1000), S._Req(None, 0, 0.0, None),
            S._Req(None, 100, 0.0, None, pos=1250), S._Req(None, 0, 0.0, None)]
    offs, rq = S.plan_pass(reqs, 100)
    assert offs.tolist() == [1000, 1100, 1200, 1250, 1350]
    assert rq.tolist() == [0, 3, 3, 4, 4]
    offs, rq = S.plan_pass([S._Req(None, 0, 0.0, None)], 100)
    assert offs.tolist() == [0] and rq.tolist() == [0, 0]


def test_server_results_equal_oracle_alone():
    pl = _payloads(24, 3)
    be = FakeBackend(delay=0.01)
    with S.Server(be, hbm_budget=_budget(200000, 2, 400000), max_pass=200000, workers=2, level=1) as srv:
        futs = [srv.submit(p) for p in pl]
        outs = [f.result(60) for f in futs]
    for p, z in zip(pl, outs):
        assert z == cref.compress(p, [0, p.size] if p.size else [0], level=1)
        assert bz2.decompress(z) == p.tobytes()
    st = srv.stats
    assert st.done == 24 and st.failed == 0 and len(st.latencies) == 24
    assert all(x >= 0 for x in st.latencies)
    assert sum(st.pass_sizes) == 24


def test_server_batches_arrivals_during_a_pass_and_overlaps():
    pl = _payloads(40, 4, lo=1, hi=5000)
    be = FakeBackend(delay=0.05)
    with S.Server(be, hbm_budget=_budget(1 << 20, 2, 4 << 20), max_pass=1 << 20, workers=2, level=9) as srv:
        futs = []
        for p in pl:
            futs.append(srv.submit(p))
            time.sleep(0.004)
        srv.drain(futs, 60)
    assert all(f.exception() is None for f in futs)
    assert max(be.passes) > 1, "requests that arrived during a pass were not batched"
    assert be.max_inflight == 2, "the two workers never ran passes at the same time"
    assert srv.stats.passes < len(pl)


def test_server_budget_refusal_and_backpressure():
    with pytest.raises(ValueError):
        S.Server(FakeBackend(), hbm_budget=_budget(100000, 2, 50000), max_pass=100000, workers=2)
    be = FakeBackend(delay=0.02)
    # arena holds barely two requests: admission must wait for released space
    with S.Server(be, hbm_budget=_budget(60000, 1, 120000), max_pass=60000, workers=1, level=1) as srv:
        big = srv.submit(np.zeros(60001, np.uint8))
        with pytest.raises(S.AdmissionError):
            big.result(5)
        pl = _payloads(12, 5, lo=30000, hi=60000)
        futs = [srv.submit(p) for p in pl]
        outs = [f.result(60) for f in futs]
    assert srv.stats.refused == 1
    for p, z in zip(pl, outs):
        assert bz2.decompress(z) == p.tobytes()


def test_server_pass_failure_releases_space():
    pl = _payloads(10, 6, lo=1000, hi=3000)
    bad = np.full(2000, 0xAB, np.uint8)
    be = FakeBackend(fail_on=0xAB)
    with S.Server(be, hbm_budget=_budget(50000, 1, 60000), max_pass=50000, workers=1, level=9) as srv:
        f_bad = srv.submit(bad)
        with pytest.raises(RuntimeError):
            f_bad.result(30)
        futs = [srv.submit(p) for p in pl]
        outs = [f.result(60) for f in futs]
    for p, z in zip(pl, outs):
        assert bz2.decompress(z) == p.tobytes()
    assert srv.stats.failed >= 1 and srv.ring.used() == 0


def test_server_close_finishes_everything():
    pl = _payloads(16, 7, lo=0, hi=20000)
    srv = S.Server(FakeBackend(delay=0.02), hbm_budget=_budget(100000, 2, 100000), max_pass=100000, workers=2,
                   level=2)
    futs = [srv.submit(p) for p in pl]
    srv.close()
    assert all(f.done() and f.exception() is None for f in futs)
    with pytest.raises(RuntimeError):
        srv.submit(b"x")


@pytest.mark.gpu
def test_gpu_serving_alone_equals_in_mix():
    """Each request's stream from the loop (mixed with others, two workers,
    arrivals during passes) equals its stream compressed alone and the
    oracle's."""
    import torch
    from paper_1109_2348_amd import native
    assert torch.cuda.is_available()
    reqs = W.requests(30, 200.0, lo=4000, hi=3_000_000, seed=11)
    payloads = [r.data for r in reqs] + [np.zeros(0, np.uint8)]
    arrivals = [r.arrival_s - reqs[0].arrival_s for r in reqs] + [0.01]
    print(f"[case] serving mix: {len(payloads)} requests, {sum(p.size for p in payloads)} bytes", flush=True)
    backend = S.GpuBackend()
    with S.Server(backend, hbm_budget=8 << 30, max_pass=32 << 20, workers=2, level=9) as srv:
        hs = {w.comp.ctx.h.value for w in backend.workers}
        assert len(hs) == 2, "workers must not share a library context"
        futs, wall = S.poisson_run(srv, payloads, arrivals, timeout=120)
        outs = [bytes(f.result(1)) for f in futs]
        summ = srv.stats.summary()
    print(f"[case] serving summary {summ}", flush=True)
    assert summ["requests"] == len(payloads) and summ["failed"] == 0
    comp = native.Compressor()
    for i, (p, z) in enumerate(zip(payloads, outs)):
        x = torch.from_numpy(p).cuda()
        alone = comp(x, None, level=9).cpu().numpy().tobytes()
        assert z == alone, f"request {i} ({p.size} B): stream in the mix differs from the stream alone"
        if i % 5 == 0:
            assert z == cref.compress(p, native.uniform_offsets(p.size, 900000), level=9, threads=16)
        assert bz2.decompress(z) == p.tobytes()


@pytest.mark.gpu
def test_gpu_serving_device_tensors_wait_for_their_producer():
    """Device-tensor requests submitted right after the kernels that write
    them (queued behind a long one, no host wait): each stream equals the
    oracle's stream of the bytes those kernels produce."""
    import torch
    from paper_1109_2348_amd import native
    assert torch.cuda.is_available()
    payloads = [W.source_blocks(k, [n], 41)[0] for k, n in (("text", 700_000), ("uniform", 250_001),
                                                              ("sparse", 1_300_000))]
    want = [((p.astype(np.int32) * 3 + 7) % 256).astype(np.uint8) for p in payloads]
    srcs = [torch.from_numpy(p).cuda() for p in payloads]
    big = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    print(f"[case] serving device tensors: {[p.size for p in payloads]}", flush=True)
    backend = S.GpuBackend()
    with S.Server(backend, hbm_budget=8 << 30, max_pass=8 << 20, workers=2, level=9) as srv:
        futs = []
        for s in srcs:
            for _ in range(4):
                big = torch.mm(big, big).clamp_(-1, 1)  # a long kernel ahead of the producer
            y = ((s.to(torch.int32) * 3 + 7) % 256).to(torch.uint8)
            futs.append(srv.submit(y))
        outs = [bytes(f.result(120)) for f in futs]
    for i, (w, z) in enumerate(zip(want, outs)):
        assert z == cref.compress(w, native.uniform_offsets(w.size, 900000), level=9, threads=16), \
            f"request {i}: stream differs from the oracle's stream of the produced bytes"
