"""Continuous-batching sort server on one GPU.

Requests (an [n, R] uint8 device tensor to sort in place by its first K
bytes) arrive at any time.  A scheduler thread admits them in arrival order
while the scratch budget (n*R bytes of tmp per request) and the slot count
allow, packs the admitted requests into one batched launch
(raduls_sort_batch) on whichever of its streams is idle, and completes them
when that stream's event fires.  Requests that arrive while batches run are
admitted as soon as budget and slots free up, and batches on different
streams overlap on the device.  Each request's result is exactly what the
plain raduls_sort would produce (the sort is deterministic and stable).

The device work goes through a backend object; ``GpuBackend`` drives the
HIP library (optionally replaying one captured HIP graph per stream), and the
tests plug in a CPU stand-in to exercise admission, back-pressure,
cancellation and failure handling without a GPU.
"""

from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Any


class Rejected(RuntimeError):
    """The request can never be admitted (larger than the whole budget)."""


class Cancelled(RuntimeError):
    pass


class BackendError(RuntimeError):
    pass


@dataclass
class Request:
    recs: Any                     # device tensor [n, R], sorted in place
    n: int
    t_arrival: float
    rid: int
    future: Future = field(default_factory=Future)
    t_admit: float = 0.0
    t_launch: float = 0.0
    t_done: float = 0.0
    tmp: Any = None
    cancelled: bool = False
    ready: Any = None             # backend token: the input has been written


@dataclass
class Stats:
    submitted: int = 0
    completed: int = 0
    rejected: int = 0
    cancelled: int = 0
    failed: int = 0
    batches: int = 0
    records: int = 0
    latencies: list = field(default_factory=list)
    t_first: float = 0.0
    t_last: float = 0.0

    def summary(self) -> dict:
        lat = sorted(self.latencies)

        def pct(p):
            if not lat:
                return None
            return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]

        span = max(self.t_last - self.t_first, 1e-12)
        return {
            "requests": self.completed, "batches": self.batches, "records": self.records,
            "rejected": self.rejected, "cancelled": self.cancelled, "failed": self.failed,
            "p50_ms": None if not lat else pct(50) * 1e3,
            "p99_ms": None if not lat else pct(99) * 1e3,
            "max_ms": None if not lat else lat[-1] * 1e3,
            "records_per_s": self.records / span if self.completed else 0.0,
            "span_s": span,
        }


class Arena:
    """First-fit allocator of byte ranges inside one preallocated buffer; each
    launched batch takes one contiguous range for the scratch of all its
    requests, so the number of live ranges never exceeds the stream count."""

    ALIGN = 256

    def __init__(self, size: int):
        self.size = size
        self.free = [(0, size)]  # sorted, coalesced (offset, length)

    def alloc(self, nbytes: int) -> int | None:
        nbytes = max(self.ALIGN, -(-nbytes // self.ALIGN) * self.ALIGN)
        for i, (off, ln) in enumerate(self.free):
            if ln >= nbytes:
                if ln == nbytes:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + nbytes, ln - nbytes)
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        nbytes = max(self.ALIGN, -(-nbytes // self.ALIGN) * self.ALIGN)
        self.free.append((off, nbytes))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


class GpuBackend:
    """Device side of the server: per-stream batch workspaces, launches and
    completion events."""

    def __init__(self, rec_bytes: int, key_bytes: int, n_streams: int, max_batch: int,
                 max_records: int, use_graphs: bool = True, device: str = "cuda"):
        import torch
        from . import binding as b
        self.torch, self.b = torch, b
        self.rec_bytes, self.key_bytes = rec_bytes, key_bytes
        self.n_streams, self.max_batch = n_streams, max_batch
        self.device = torch.device(device)
        # scratch for every admitted request comes from one resident buffer
        self.arena_buf = torch.empty(max_records * rec_bytes + Arena.ALIGN * (max_batch + 1),
                                     dtype=torch.uint8, device=self.device)
        self.arena = Arena(self.arena_buf.numel())
        self.chunks = {}
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.batches = [b.Batch(max_batch, max_records, rec_bytes, key_bytes, device=self.device)
                        for _ in range(n_streams)]
        self.graphs = [None] * n_streams
        self.use_graphs = use_graphs
        self.capacity_bytes = max_records * rec_bytes  # scratch the arena holds for requests
        if use_graphs:
            self._capture()

    def producer_event(self, recs) -> Any:
        """An event on the submitting thread's current stream: the sort of
        `recs` waits for it, so work that stream queued to write the input
        (not yet finished at submission) comes first."""
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(recs.device))
        return ev

    def _capture(self):
        torch = self.torch
        for i, (s, bt) in enumerate(zip(self.streams, self.batches)):
            bt.host_desc.zero_()
            bt.desc.zero_()
            with torch.cuda.stream(s):
                bt.launch(stream=s)  # warm-up outside capture (sets kernel attributes)
            s.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                bt.launch(stream=s)
            self.graphs[i] = g
        torch.cuda.synchronize()

    def prepare(self, stream_idx: int, reqs: list) -> bool:
        """Carve the batch's scratch out of the arena; False if it does not fit
        yet (the server retries after a batch completes)."""
        step = [-(-(r.n * self.rec_bytes) // 16) * 16 for r in reqs]
        total = sum(step)
        off = self.arena.alloc(total)
        if off is None:
            return False
        self.chunks[stream_idx] = (off, total)
        base = self.arena_buf.data_ptr() + off
        for r, sz in zip(reqs, step):
            r.tmp = base
            base += sz
        return True

    def launch(self, stream_idx: int, reqs: list) -> Any:
        torch = self.torch
        s = self.streams[stream_idx]
        bt = self.batches[stream_idx]
        hd = bt.host_desc
        h = hd.numpy()
        h[:] = 0
        for i, r in enumerate(reqs):
            h[i, 0] = r.recs.data_ptr()
            h[i, 1] = r.tmp
            h[i, 2] = r.n
        ev = torch.cuda.Event()
        with torch.cuda.stream(s):
            for r in reqs:
                if r.ready is not None:
                    s.wait_event(r.ready)  # the producer's writes of the input come first
                # the caching allocator must not hand the input's memory to
                # another stream's work before this sort is done with it
                r.recs.record_stream(s)
            bt.desc.copy_(hd, non_blocking=True)
            if self.graphs[stream_idx] is not None:
                self.graphs[stream_idx].replay()
            else:
                bt.launch(stream=s)
            ev.record(s)
        return ev

    def done(self, token) -> bool:
        return token.query()

    def release(self, stream_idx: int) -> None:
        chunk = self.chunks.pop(stream_idx, None)
        if chunk is not None:
            self.arena.release(*chunk)

    def finish(self, stream_idx: int, token, reqs: list) -> list:
        token.synchronize()
        st, stats = self.batches[stream_idx].check(self.streams[stream_idx])
        err = None if st == self.b.OK else f"device error {stats}"
        for r in reqs:
            r.tmp = None
        self.release(stream_idx)
        return [err] * len(reqs)


class Server:
    """Admission by scratch budget and slots, continuous batching over streams."""

    def __init__(self, backend, rec_bytes: int, budget_bytes: int, max_slots: int,
                 max_batch: int | None = None, poll_s: float = 2e-5):
        self.backend = backend
        self.rec_bytes = rec_bytes
        cap = getattr(backend, "capacity_bytes", None)
        if cap is not None and budget_bytes > cap:
            # an admitted batch could then never get its scratch from the
            # backend and would be retried for ever
            raise ValueError(f"budget {budget_bytes} B exceeds the backend's scratch {cap} B")
        if max_batch is not None and max_batch > backend.max_batch:
            raise ValueError(f"max_batch {max_batch} exceeds the backend's {backend.max_batch}")
        self.budget = budget_bytes
        self.free = budget_bytes
        self.max_slots = max_slots
        self.slots = max_slots
        self.max_batch = max_batch or backend.max_batch
        self.poll_s = poll_s
        self.pending: collections.deque = collections.deque()
        self.admitted: list = []
        self.inflight: dict = {}          # stream -> (token, reqs)
        self.lock = threading.Condition()
        self.stats = Stats()
        self._rid = 0
        self._stop = False
        self._thread = None

    # ------------------------------------------------------------ client side
    def need(self, n: int) -> int:
        return n * self.rec_bytes

    def submit(self, recs, t_arrival: float | None = None) -> Future:
        n = int(recs.shape[0])
        with self.lock:
            req = Request(recs=recs, n=n, t_arrival=time.perf_counter() if t_arrival is None
                          else t_arrival, rid=self._rid)
            self._rid += 1
            self.stats.submitted += 1
            if self.need(n) > self.budget:
                self.stats.rejected += 1
                req.future.set_exception(Rejected(f"request of {n} records exceeds the budget"))
                return req.future
            if self.stats.t_first == 0.0:
                self.stats.t_first = req.t_arrival
            mark = getattr(self.backend, "producer_event", None)
            if mark is not None:
                req.ready = mark(recs)
            self.pending.append(req)
            self.lock.notify_all()
        return req.future

    def cancel(self, fut: Future) -> bool:
        """Cancel a request that has not been launched yet."""
        with self.lock:
            for q, reserved in ((self.pending, False), (self.admitted, True)):
                for r in list(q):
                    if r.future is fut:
                        q.remove(r)
                        if reserved:  # admitted requests hold budget and a slot
                            self.free += self.need(r.n)
                            self.slots += 1
                        r.tmp = None
                        self.stats.cancelled += 1
                        fut.set_exception(Cancelled("cancelled before launch"))
                        self.lock.notify_all()
                        return True
        return False

    # ------------------------------------------------------------ scheduler
    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._run, name="raduls-server", daemon=True)
        self._thread.start()
        return self

    def stop(self, drain: bool = True) -> dict:
        with self.lock:
            if not drain:
                for r in list(self.pending):
                    r.future.set_exception(Cancelled("server stopped"))
                    self.stats.cancelled += 1
                self.pending.clear()
            self._stop = True
            self.lock.notify_all()
        if self._thread is not None:
            self._thread.join()
        return self.stats.summary()

    def _idle_stream(self):
        for s in range(self.backend.n_streams):
            if s not in self.inflight:
                return s
        return None

    def step(self) -> bool:
        """One scheduling pass; returns True if it did any work."""
        worked = False
        # completions
        for s, (tok, reqs) in list(self.inflight.items()):
            if self.backend.done(tok):
                try:
                    errs = self.backend.finish(s, tok, reqs)
                except Exception as e:  # backend failure: fail the batch, keep serving
                    errs = [f"backend failure: {e}"] * len(reqs)
                now = time.perf_counter()
                with self.lock:
                    del self.inflight[s]
                    for r, err in zip(reqs, errs):
                        self.free += self.need(r.n)
                        self.slots += 1
                        r.t_done = now
                        if err:
                            self.stats.failed += 1
                            r.future.set_exception(BackendError(err))
                        else:
                            self.stats.completed += 1
                            self.stats.records += r.n
                            self.stats.latencies.append(now - r.t_arrival)
                            self.stats.t_last = now
                            r.future.set_result(r.recs)
                    self.lock.notify_all()
                worked = True
        # admission, in arrival order (no overtaking)
        with self.lock:
            s_idx = self._idle_stream()
            while self.pending and self.slots > 0 and len(self.admitted) < self.max_batch:
                r = self.pending[0]
                if self.need(r.n) > self.free:
                    break
                self.pending.popleft()
                self.free -= self.need(r.n)
                self.slots -= 1
                r.t_admit = time.perf_counter()
                self.admitted.append(r)
                worked = True
            if s_idx is None or not self.admitted:
                return worked
            batch, self.admitted = self.admitted, []
        # launch on the idle stream
        try:
            if not self.backend.prepare(s_idx, batch):
                with self.lock:  # scratch fragmented: retry after a completion
                    self.admitted = batch + self.admitted
                return worked
            tok = self.backend.launch(s_idx, batch)
        except Exception as e:
            if hasattr(self.backend, "release"):
                self.backend.release(s_idx)
            with self.lock:
                for r in batch:
                    self.free += self.need(r.n)
                    self.slots += 1
                    r.tmp = None
                    self.stats.failed += 1
                    r.future.set_exception(BackendError(f"launch failed: {e}"))
            return True
        now = time.perf_counter()
        for r in batch:
            r.t_launch = now
        with self.lock:
            self.inflight[s_idx] = (tok, batch)
            self.stats.batches += 1
        return True

    def _run(self):
        while True:
            worked = self.step()
            with self.lock:
                if self._stop and not self.pending and not self.admitted and not self.inflight:
                    return
                if not worked:
                    if not self.inflight and not self.pending and not self._stop:
                        self.lock.wait(timeout=0.01)
            if not worked:
                time.sleep(self.poll_s)
