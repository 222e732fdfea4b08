"""Compression serving: continuous batching of independent compress requests.

The stages are data-parallel over blocks (Sec. 4 of the paper), so blocks of
different requests can share one pass of the pipeline and still come out as
separate bzip2 streams (``compress_batch``).  This loop turns a stream of
requests of any size into such passes:

* Admission.  The device holds one input arena, handed out as a FIFO ring:
  a request is admitted when its bytes fit the free part of the ring, then
  uploaded there (its blocks stay resident until its stream is done).  The
  arena is what the HBM budget leaves after each worker's worst-case pipeline
  workspace for its largest pass; a request larger than one pass is refused
  at submission.
* Batching.  Each worker (its own library context and HIP stream) takes, as
  soon as it is free, every uploaded request at the front of the queue whose
  bytes follow on in the arena, up to one pass's size.  Requests that arrive
  while one pass runs are admitted and uploaded meanwhile and go to the next
  free worker, so passes of different workers overlap on the device.
* Completion.  A pass ends when its streams are copied to the host; the
  requests' futures resolve, their arena space is released from the oldest
  end, and waiting requests are admitted.

Latency is measured from a request's arrival to its stream on the host.

The device work is behind a small backend interface (``arena``, ``upload``,
``worker``) so the scheduling logic can be exercised without a GPU.
"""

from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

# Device bytes the pipeline may use per input byte of one pass: the sort's
# index, rank, key and two segment-list buffers (about 45 per RLE1 byte),
# text/BWT/symbol arrays (4) and the worst-case output (3), with RLE1 output
# up to 1.25x the input.
WORKSPACE_PER_BYTE = 66
WORKSPACE_FIXED = 64 << 20
MAX_PASS_BYTES = (1 << 31) - 1
MAX_PASS_REQUESTS = 65535


class AdmissionError(RuntimeError):
    """The request can never fit the server's HBM budget."""


@dataclass
class _Req:
    data: object                 # host uint8 array or device uint8 tensor
    n: int
    arrival: float
    fut: Future
    pos: int = -1                # arena offset once admitted
    slot: Optional[list] = None  # ring entry
    t_start: float = 0.0
    t_done: float = 0.0
    ready: object = None         # device tensor: event on its producer's stream at submit


class Ring:
    """Byte ranges of a fixed arena, handed out in FIFO order and released in
    any order; space is reclaimed from the oldest live range."""

    def __init__(self, cap: int):
        self.cap = int(cap)
        self.head = 0
        self.live = collections.deque()  # [start, end, done]

    def alloc(self, n: int):
        if n > self.cap:
            return None
        if not self.live:
            self.head = 0
        tail = self.live[0][0] if self.live else 0
        wrapped = bool(self.live) and self.head <= tail
        if not wrapped:
            if self.head + n <= self.cap:
                start = self.head
            elif n <= tail:
                start = 0
            else:
                return None
        else:
            if self.head + n > tail:
                return None
            start = self.head
        e = [start, start + n, False]
        self.live.append(e)
        self.head = start + n
        return e

    def free(self, e):
        e[2] = True
        while self.live and self.live[0][2]:
            self.live.popleft()

    def used(self) -> int:
        return sum(e[1] - e[0] for e in self.live if not e[2])


def plan_pass(reqs: Sequence[_Req], block: int):
    """Block offsets (arena coordinates) and request -> block ranges of one
    pass.  The requests' bytes are adjacent in the arena."""
    offs, rq = [], [0]
    pos = None
    for r in reqs:
        if r.n:
            if pos is None:
                pos = r.pos
                offs.append(pos)
            assert r.pos == pos, "pass requests must be adjacent in the arena"
            for a in range(0, r.n, block):
                offs.append(pos + min(a + block, r.n))
            pos += r.n
        rq.append(len(offs) - 1 if offs else 0)
    if not offs:
        offs = [0]
    return np.array(offs, np.uint64), np.array(rq, np.uint32)


@dataclass
class ServerStats:
    done: int = 0
    failed: int = 0
    refused: int = 0
    bytes_in: int = 0
    bytes_out: int = 0
    passes: int = 0
    latencies: List[float] = field(default_factory=list)
    pass_sizes: List[int] = field(default_factory=list)
    first_arrival: float = float("inf")
    last_done: float = 0.0

    def summary(self) -> dict:
        lat = np.array(self.latencies) * 1e3 if self.latencies else np.zeros(1)
        span = self.last_done - self.first_arrival if self.done else 0.0
        return {"requests": self.done, "failed": self.failed, "refused": self.refused, "passes": self.passes,
                "mean_requests_per_pass": round(float(np.mean(self.pass_sizes)), 2) if self.pass_sizes else 0.0,
                "input_bytes": self.bytes_in, "output_bytes": self.bytes_out,
                "MB_per_s": round(self.bytes_in / span / 1e6, 2) if span > 0 else None,
                "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3)}


class Server:
    """Continuous-batching compression server.

    backend      device backend (``GpuBackend`` by default).
    hbm_budget   device bytes for the arena plus every worker's workspace.
    max_pass     input bytes of one pass (also the largest request).
    workers      passes that may be in flight at once (each its own stream).
    level        bzip2 level: blocks of 100000*level bytes and header digit.
    """

    def __init__(self, backend=None, hbm_budget: int = 32 << 30, max_pass: int = 256 << 20, workers: int = 2,
                 level: int = 9, clock: Callable[[], float] = time.perf_counter):
        if backend is None:
            backend = GpuBackend()
        if not 1 <= level <= 9:
            raise ValueError("level must be 1..9")
        if workers < 1:
            raise ValueError("at least one worker")
        self.max_pass = min(int(max_pass), MAX_PASS_BYTES)
        arena = int(hbm_budget) - workers * (WORKSPACE_PER_BYTE * self.max_pass + WORKSPACE_FIXED)
        if arena < self.max_pass:
            raise ValueError(f"HBM budget {hbm_budget} B leaves {arena} B of arena for passes of {self.max_pass} B")
        self.level, self.block = level, 100000 * level
        self.clock = clock
        self.backend = backend
        self.arena_bytes = arena
        self.arena = backend.arena(arena)
        self.ring = Ring(arena)
        self.stats = ServerStats()
        self._lock = threading.Condition()
        self._pending = collections.deque()  # submitted, not yet admitted
        self._ready = collections.deque()    # uploaded, waiting for a worker
        self._closing = False
        self._admit_done = False
        self._threads = [threading.Thread(target=self._admit_loop, name="bz-admit", daemon=True)]
        self._threads += [threading.Thread(target=self._work_loop, args=(backend.worker(i),), name=f"bz-work{i}",
                                           daemon=True) for i in range(workers)]
        for t in self._threads:
            t.start()

    # ---- client side
    def submit(self, data, arrival: Optional[float] = None) -> Future:
        """Queue one request (host uint8 array or bytes, host or device uint8
        tensor); the future resolves to its bzip2 stream, a bytes-like object
        (a uint8 array from the GPU backend)."""
        if isinstance(data, (bytes, bytearray, memoryview)):
            data = np.frombuffer(bytes(data), np.uint8)
        n = int(data.numel() if hasattr(data, "numel") else data.size)
        fut: Future = Future()
        t = self.clock() if arrival is None else arrival
        if n > self.max_pass:
            with self._lock:
                self.stats.refused += 1
            fut.set_exception(AdmissionError(f"request of {n} B exceeds one pass ({self.max_pass} B)"))
            return fut
        with self._lock:
            if self._closing:
                raise RuntimeError("server is closed")
            ready = None
            if getattr(data, "is_cuda", False):
                # the upload must not start before whatever produced the
                # tensor on the submitter's stream has written it
                import torch
                ready = torch.cuda.Event()
                ready.record(torch.cuda.current_stream(data.device))
            self._pending.append(_Req(data, n, t, fut, ready=ready))
            self.stats.first_arrival = min(self.stats.first_arrival, t)
            self._lock.notify_all()
        return fut

    def close(self):
        """Finish every submitted request, then stop the threads."""
        with self._lock:
            self._closing = True
            self._lock.notify_all()
        for t in self._threads:
            t.join()
        for r in list(self._pending) + list(self._ready):
            if not r.fut.done():
                r.fut.set_exception(RuntimeError("server closed"))

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def drain(self, futures: Sequence[Future], timeout: Optional[float] = None):
        for f in futures:
            try:
                f.result(timeout)
            except Exception:  # noqa: BLE001 - failures are counted in stats
                pass

    # ---- admission: reserve arena space in FIFO order, upload
    def _admit_loop(self):
        while True:
            with self._lock:
                while not self._pending:
                    if self._closing:
                        self._admit_done = True
                        self._lock.notify_all()
                        return
                    self._lock.wait()
                r = self._pending[0]
                slot = self.ring.alloc(r.n) if r.n else None
                if r.n and slot is None:
                    self._lock.wait()  # space comes back when a pass completes
                    continue
                self._pending.popleft()
                r.slot = slot
                r.pos = slot[0] if slot else -1
            if r.n:
                try:
                    self.backend.upload(self.arena, r.pos, r.data, r.ready)
                except Exception as e:  # noqa: BLE001
                    with self._lock:
                        self.ring.free(r.slot)
                        self.stats.failed += 1
                        self._lock.notify_all()
                    r.fut.set_exception(e)
                    continue
            r.data = None
            with self._lock:
                self._ready.append(r)
                self._lock.notify_all()

    # ---- workers: take the adjacent front of the ready queue, run one pass
    def _take_pass(self) -> List[_Req]:
        batch, nbytes, end = [], 0, None
        while self._ready and len(batch) < MAX_PASS_REQUESTS:
            r = self._ready[0]
            if r.n:
                if end is not None and r.pos != end:
                    break
                if batch and nbytes + r.n > self.max_pass:
                    break
                end = r.pos + r.n
                nbytes += r.n
            batch.append(self._ready.popleft())
        return batch

    def _work_loop(self, run):
        while True:
            with self._lock:
                while not self._ready:
                    if self._closing and self._admit_done:
                        return
                    self._lock.wait()
                batch = self._take_pass()
            t0 = self.clock()
            try:
                offs, rq = plan_pass(batch, self.block)
                outs = run(self.arena, offs, rq, self.level)
                err = None
            except Exception as e:  # noqa: BLE001
                outs, err = None, e
            t1 = self.clock()
            with self._lock:
                for r in batch:
                    if r.slot is not None:
                        self.ring.free(r.slot)
                self.stats.passes += 1
                self.stats.pass_sizes.append(len(batch))
                for i, r in enumerate(batch):
                    r.t_start, r.t_done = t0, t1
                    if err is None:
                        self.stats.done += 1
                        self.stats.bytes_in += r.n
                        self.stats.bytes_out += len(outs[i])
                        self.stats.latencies.append(t1 - r.arrival)
                        self.stats.last_done = max(self.stats.last_done, t1)
                    else:
                        self.stats.failed += 1
                self._lock.notify_all()
            for i, r in enumerate(batch):
                if err is None:
                    r.fut.set_result(outs[i])
                else:
                    r.fut.set_exception(err)


class GpuBackend:
    """Arena in HBM; uploads on a stream of their own; one library context and
    stream per worker.

    Host arrays are uploaded through two pinned staging buffers (the copy
    into one overlaps the DMA out of the other); pinned host tensors and
    device tensors are copied directly.  A pass's streams come back in one
    pinned buffer and are returned as uint8 array views of it."""

    STAGE = 32 << 20

    def __init__(self, device: int = 0):
        import torch
        from . import native
        native.lib()  # fail here, loudly, if the library is not built
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.up_stream = torch.cuda.Stream(self.device)
        self.stage = [torch.empty(self.STAGE, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self.stage_ev = [None, None]
        self.workers = []

    def arena(self, nbytes: int):
        return self.torch.empty(max(int(nbytes), 4), dtype=self.torch.uint8, device=self.device)

    def upload(self, arena, pos: int, data, ready=None):
        torch = self.torch
        with torch.cuda.stream(self.up_stream):
            if ready is not None:
                self.up_stream.wait_event(ready)
            if torch.is_tensor(data):
                src = data.reshape(-1)
                arena[pos:pos + src.numel()].copy_(src, non_blocking=True)
            else:
                a = np.ascontiguousarray(data, dtype=np.uint8).reshape(-1)
                for i, c in enumerate(range(0, a.size, self.STAGE)):
                    k = i % 2
                    if self.stage_ev[k] is not None:
                        self.stage_ev[k].synchronize()  # its previous DMA is done
                    m = min(self.STAGE, a.size - c)
                    self.stage[k][:m].numpy()[:] = a[c:c + m]
                    arena[pos + c:pos + c + m].copy_(self.stage[k][:m], non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(self.up_stream)
                    self.stage_ev[k] = ev
        self.up_stream.synchronize()

    def worker(self, i: int):
        w = _GpuWorker(self.torch, self.device)
        self.workers.append(w)
        return w


class _GpuWorker:
    """One pass at a time on a library context and stream of its own (calls
    on one context never overlap, so workers must not share one)."""

    def __init__(self, torch, device):
        from .native import BatchCompressor, Context
        self.torch = torch
        self.stream = torch.cuda.Stream(device)
        self.comp = BatchCompressor(device.index, ctx=Context(device.index))

    def __call__(self, arena, offsets, req_blocks, level) -> List[np.ndarray]:
        torch = self.torch
        with torch.cuda.stream(self.stream):
            zs = self.comp(arena, offsets, req_blocks, level)
            lens = [int(z.numel()) for z in zs]
            total = sum(lens)
            host = torch.empty(max(total, 1), dtype=torch.uint8, pin_memory=True)
            if total:
                host[:total].copy_(torch.cat(zs), non_blocking=True)
            self.stream.synchronize()
        arr = host.numpy()
        out, p = [], 0
        for n in lens:
            out.append(arr[p:p + n])
            p += n
        return out


def poisson_run(server: Server, payloads: Sequence, arrivals: Sequence[float], timeout: float = 600.0):
    """Submit payloads[i] at arrivals[i] seconds after the start (a driver
    thread sleeps until each arrival); returns the futures and the wall time
    from the first arrival to the last completion."""
    t0 = server.clock()
    futs = []
    for data, t in zip(payloads, arrivals):
        now = server.clock() - t0
        if t > now:
            time.sleep(t - now)
        futs.append(server.submit(data, arrival=t0 + t))
    server.drain(futs, timeout)
    return futs, server.clock() - t0
