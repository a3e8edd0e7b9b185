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
from dataclasses import dataclass, field
from typing import Any

import numpy as np


class Rejected(RuntimeError):
    """The request can never be admitted (larger than the whole budget)."""


class Cancelled(RuntimeError):
    pass


class BackendError(RuntimeError):
    pass


class Request:
    """One queued sort, and its result handle: the subset of
    concurrent.futures.Future that callers use (result, exception, done).
    It holds no lock of its own: every request of a server waits on the
    server's one completion condition, which the scheduler notifies once per
    completed batch, so a batch of thousands of requests costs one wake-up
    instead of one per request."""

    __slots__ = ("recs", "n", "t_arrival", "ready", "t_admit", "t_launch", "t_done", "tmp",
                 "_cv", "_state", "_value")
    _PENDING, _OK, _ERR = 0, 1, 2

    def __init__(self, recs, n: int, t_arrival: float, cv: threading.Condition,
                 ready: Any = None):
        self.recs = recs          # device tensor [n, R], sorted in place
        self.n = n
        self.t_arrival = t_arrival
        self.ready = ready        # backend token: the input has been written
        self.t_admit = self.t_launch = self.t_done = 0.0
        self.tmp = None
        self._cv = cv
        self._state = Request._PENDING
        self._value = None

    def done(self) -> bool:
        return self._state != Request._PENDING

    def _wait(self, timeout):
        if self._state == Request._PENDING:
            with self._cv:
                if not self._cv.wait_for(self.done, timeout):
                    raise TimeoutError("request not completed in time")

    def result(self, timeout: float | None = None):
        self._wait(timeout)
        if self._state == Request._ERR:
            raise self._value
        return self._value

    def exception(self, timeout: float | None = None):
        self._wait(timeout)
        return self._value if self._state == Request._ERR else None

    # scheduler side: set, then notify the condition (once for many requests)
    def _resolve(self, value) -> None:
        self._value = value
        self._state = Request._OK

    def _fail(self, exc: BaseException) -> None:
        self._value = exc
        self._state = Request._ERR


@dataclass
class Stats:
    completed: int = 0
    rejected: int = 0
    cancelled: int = 0
    failed: int = 0
    batches: int = 0
    records: int = 0
    latencies: list = field(default_factory=list)
    t_first: float = 0.0
    t_last: float = 0.0
    launch_host_s: float = 0.0    # host time spent preparing and enqueuing batches

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
            "mean_batch": self.completed / self.batches if self.batches else 0.0,
            "launch_host_s": self.launch_host_s,
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
    completion events, and optionally a resident server (raduls_server_*)
    for requests that fit one LDS job: those are sorted by workgroups that
    stay on the device, with no launch and no scratch.  Its kernel leaves
    after `resident_lease_ms` of service (or as long without a request) and
    is relaunched by the next call that needs it: a PyTorch process has more
    streams than the device has hardware queues, so a batch stream may share
    the kernel's queue, and then waits at most that long.  While the kernel
    runs, a device-wide synchronize would wait for it: callers synchronize
    their own streams instead, and ``close`` stops it.

    The resident path is experimental: it is tested with a few hundred
    requests, but a run that sent 40,192 of 65,536 requests to a
    32-workgroup resident server beside three batch streams did not finish
    (with a 10-minute and again with a 2 ms lease; cause not found)."""

    def __init__(self, rec_bytes: int, key_bytes: int, n_streams: int, max_batch: int,
                 max_records: int, use_graphs: bool = True, device: str = "cuda",
                 resident_workgroups: int = 0, resident_slots: int = 8192,
                 resident_lease_ms: int = 2):
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
        # (after the capture, which synchronizes the device)
        self.resident = None
        self.resident_cap = -1
        if resident_workgroups:
            self.resident = b.ResidentServer(rec_bytes, key_bytes, slots=resident_slots,
                                             workgroups=resident_workgroups,
                                             idle_ms=resident_lease_ms, lease_ms=resident_lease_ms)
            self.resident_cap = self.resident.max_records

    # ---- resident path: requests of at most resident_cap records
    def ready_done(self, token) -> bool:
        """Whether the work a producer event stands for has finished."""
        return token is None or token[1].query()

    def resident_submit(self, req) -> tuple[int, int]:
        """(0, ticket), (1, 0) when the ring is full, or (negative status, 0)
        (also after close)."""
        if self.resident is None:
            return self.b.E_STOPPED, 0
        st, t = self.resident.submit_status(req.recs, req.n)
        if st == self.b.E_BUSY:
            return 1, 0
        return (0, t) if st == self.b.OK else (st, 0)

    def resident_completed(self) -> tuple[int, int]:
        if self.resident is None:
            raise self.b.RadulsError(self.b.E_STOPPED, "resident server closed")
        return self.resident.completed()

    def resident_status(self, ticket: int) -> int:
        if self.resident is None:
            return -1
        return self.resident.poll(ticket)[1]

    def close(self) -> None:
        """Stop the resident server, if any (its kernel leaves)."""
        if self.resident is not None:
            r, self.resident = self.resident, None
            self.resident_cap = -1
            r.close()

    def producer_event(self, recs) -> Any:
        """(stream, event) recorded on the submitting thread's current
        stream: the sort of `recs` waits for it, so work that stream queued to
        write the input (not yet finished at submission) comes first."""
        s = self.torch.cuda.current_stream(recs.device)
        ev = self.torch.cuda.Event()
        ev.record(s)
        return (s.cuda_stream, ev)

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
        """Carve the batch's scratch out of the arena (one 16-byte aligned
        slice per request, in order); False if it does not fit yet (the
        server retries after a batch completes)."""
        k = len(reqs)
        ns = np.fromiter((r.n for r in reqs), dtype=np.int64, count=k)
        step = (ns * self.rec_bytes + 15) // 16 * 16
        total = int(step.sum())
        off = self.arena.alloc(total)
        if off is None:
            return False
        self.chunks[stream_idx] = (off, total)
        h = self.batches[stream_idx].host_desc.numpy()
        h[k:] = 0
        h[:k, 1] = self.arena_buf.data_ptr() + off + np.cumsum(step) - step
        h[:k, 2] = ns
        return True

    def launch(self, stream_idx: int, reqs: list) -> Any:
        torch = self.torch
        s = self.streams[stream_idx]
        bt = self.batches[stream_idx]
        hd = bt.host_desc
        k = len(reqs)
        hd.numpy()[:k, 0] = np.fromiter((r.recs.data_ptr() for r in reqs), dtype=np.int64,
                                        count=k)
        # the producers' writes of the inputs come first: events on one
        # stream complete in order, so the last one per producing stream
        # (requests are in arrival order) covers the others.  (The server
        # keeps every request, and with it its tensor, until the batch has
        # completed, so the caching allocator cannot hand the memory to other
        # work meanwhile.)
        last = {}
        for r in reqs:
            if r.ready is not None:
                last[r.ready[0]] = r.ready[1]
        ev = torch.cuda.Event()
        with torch.cuda.stream(s):
            for e in last.values():
                s.wait_event(e)
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
        self.release(stream_idx)
        return [err] * len(reqs)


class Server:
    """Admission by scratch budget and slots, continuous batching over streams.

    Clients append to a lock-free deque (submit / submit_many take no lock
    the scheduler holds); the scheduler thread moves what has arrived into
    its pending queue under its own lock, admits in arrival order, launches,
    and resolves a completed batch's tickets together."""

    SUBMIT_CHUNK = 256   # requests submit_many queues at a time

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
        # clients append without a lock; the scheduler, cancel and stop take
        # requests out only under `lock`
        self.pending: collections.deque = collections.deque()
        # requests small enough for the backend's resident server (if any):
        # no budget, no slot, no batch; published to its ring in arrival
        # order once their input is ready, completed in ticket order
        self.resident_cap = getattr(backend, "resident_cap", -1)
        self.res_pending: collections.deque = collections.deque()
        self.res_inflight: collections.deque = collections.deque()  # (ticket, request)
        self.admitted: list = []
        self.inflight: dict = {}          # stream -> (token, reqs)
        self.lock = threading.Condition()
        self.done_cv = threading.Condition(threading.Lock())  # tickets wait here
        self.stats = Stats()
        self._sleeping = False
        self._stop = False
        self._thread = None

    # ------------------------------------------------------------ client side
    def need(self, n: int) -> int:
        return n * self.rec_bytes

    def _ready_token(self, recs, ready):
        if ready is True:
            mark = getattr(self.backend, "producer_event", None)
            return mark(recs) if mark is not None else None
        return None if ready is False else ready

    def _reject(self, req: Request) -> None:
        with self.lock:
            self.stats.rejected += 1
        req._fail(Rejected(f"request of {req.n} records exceeds the budget"))
        self._notify_done()

    def _wake(self) -> None:
        if self._sleeping:
            with self.lock:
                self.lock.notify_all()

    def submit(self, recs, t_arrival: float | None = None, ready: Any = True) -> Request:
        """Queue `recs` (an [n, R] device tensor) for sorting in place; the
        returned request is its result handle.  ready=True (default): the
        sort waits for the work the calling thread's current stream has
        queued so far (the backend records an event there); ready=False: the
        caller guarantees the input is already written (e.g. after a
        synchronize); otherwise a backend token to wait for."""
        n = int(recs.shape[0])
        req = Request(recs, n, time.perf_counter() if t_arrival is None else t_arrival,
                      self.done_cv)
        if n <= self.resident_cap:
            req.ready = self._ready_token(recs, ready)
            self.res_pending.append(req)
            self._wake()
            return req
        if n * self.rec_bytes > self.budget:
            self._reject(req)
            return req
        req.ready = self._ready_token(recs, ready)
        self.pending.append(req)   # deque appends are atomic: no lock
        self._wake()
        return req

    def submit_many(self, arrays, t_arrival: float | None = None, ready: Any = True) -> list:
        """submit() for several arrays at once, in order: one readiness token
        covers them all (they come from the same stream).  Requests are handed
        to the scheduler in chunks, so the first batch can launch while later
        requests are still being queued."""
        if not len(arrays):
            return []
        token = self._ready_token(arrays[0], ready)
        t = time.perf_counter() if t_arrival is None else t_arrival
        lim, cv, mk = self.budget // self.rec_bytes, self.done_cv, Request
        small = self.resident_cap
        out = []
        for c in range(0, len(arrays), self.SUBMIT_CHUNK):
            chunk = arrays[c:c + self.SUBMIT_CHUNK]
            ns = [a.shape[0] for a in chunk]
            reqs = [mk(a, n, t, cv, token) for a, n in zip(chunk, ns)]
            if small < min(ns) and max(ns) <= lim:  # (the usual case: all batched)
                self.pending.extend(reqs)
            else:
                if small >= 0:
                    self.res_pending.extend(r for r in reqs if r.n <= small)
                self.pending.extend(r for r in reqs if small < r.n <= lim)
                for r in reqs:
                    if r.n > small and r.n > lim:
                        self._reject(r)
            self._wake()
            out += reqs
        return out

    def _notify_done(self) -> None:
        with self.done_cv:
            self.done_cv.notify_all()

    def cancel(self, fut: Request) -> bool:
        """Cancel a request that has not been launched yet."""
        with self.lock:
            for q, reserved in ((self.pending, False), (self.admitted, True),
                                (self.res_pending, False)):
                if fut in q:     # identity: requests define no equality
                    q.remove(fut)
                    if reserved:  # admitted requests hold budget and a slot
                        self.free += self.need(fut.n)
                        self.slots += 1
                    fut.tmp = None
                    self.stats.cancelled += 1
                    fut._fail(Cancelled("cancelled before launch"))
                    self._notify_done()
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
                for q in (self.pending, self.res_pending):
                    while q:
                        q.popleft()._fail(Cancelled("server stopped"))
                        self.stats.cancelled += 1
                self._notify_done()
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

    def _complete(self, s, tok, reqs) -> None:
        try:
            errs = self.backend.finish(s, tok, reqs)
        except Exception as e:  # backend failure: fail the batch, keep serving
            errs = [f"backend failure: {e}"] * len(reqs)
        now = time.perf_counter()
        R = self.rec_bytes
        with self.lock:
            del self.inflight[s]
            st = self.stats
            lat = st.latencies
            if not any(errs):  # (the usual case: the whole batch sorted)
                recs = 0
                ok = Request._OK
                for r in reqs:
                    recs += r.n
                    r.t_done = now
                    r._value = r.recs
                    r._state = ok
                lat.extend([now - r.t_arrival for r in reqs])
                st.completed += len(reqs)
                st.records += recs
                freed = recs * R
            else:
                freed = 0
                for r, err in zip(reqs, errs):
                    freed += r.n * R
                    r.t_done = now
                    if err:
                        st.failed += 1
                        r._fail(BackendError(err))
                    else:
                        st.completed += 1
                        st.records += r.n
                        lat.append(now - r.t_arrival)
                        r._resolve(r.recs)
            if st.completed:
                st.t_last = now
            self.free += freed
            self.slots += len(reqs)
            self.lock.notify_all()
        self._notify_done()

    def _resident_step(self) -> bool:
        """Publish ready small requests to the resident server in arrival
        order (stopping at the first whose input is not ready yet, or when
        the ring is full) and complete the ones it has finished."""
        be, worked = self.backend, False
        pend, infl = self.res_pending, self.res_inflight
        while pend:
            r = pend[0]
            if not be.ready_done(r.ready):
                break
            # (published under the lock, so that a request cancelled before
            # this point is never handed to the device)
            with self.lock:
                if not pend or pend[0] is not r:  # cancelled meanwhile
                    continue
                code, t = be.resident_submit(r)
                if code == 1:  # ring full: after a completion
                    break
                pend.popleft()
                if code < 0:
                    self.stats.failed += 1
                    r._fail(BackendError(f"resident submit failed: {code}"))
                else:
                    r.t_admit = r.t_launch = time.perf_counter()
                    if not self.stats.t_first:
                        self.stats.t_first = r.t_arrival
                    infl.append((t, r))
            if code < 0:
                self._notify_done()
            worked = True
        if infl:
            try:
                through, status_or = be.resident_completed()
                failure = None
            except Exception as e:  # the resident kernel left: fail what it holds
                through, status_or, failure = infl[-1][0] + 1, 0, f"resident server: {e}"
            if infl[0][0] < through:
                now = time.perf_counter()
                with self.lock:
                    st = self.stats
                    while infl and infl[0][0] < through:
                        t, r = infl.popleft()
                        r.t_done = now
                        err = failure or (be.resident_status(t) if status_or else 0)
                        if err:
                            st.failed += 1
                            r._fail(BackendError(f"device error {err}"))
                        else:
                            st.completed += 1
                            st.records += r.n
                            st.latencies.append(now - r.t_arrival)
                            st.t_last = now
                            r._resolve(r.recs)
                    self.lock.notify_all()
                self._notify_done()
                worked = True
        return worked

    def step(self) -> bool:
        """One scheduling pass; returns True if it did any work."""
        worked = False
        if self.res_pending or self.res_inflight:
            worked = self._resident_step()
        for s, (tok, reqs) in list(self.inflight.items()):
            if self.backend.done(tok):
                self._complete(s, tok, reqs)
                worked = True
        # admission, in arrival order (no overtaking)
        with self.lock:
            s_idx = self._idle_stream()
            pend, adm, R = self.pending, self.admitted, self.rec_bytes
            room = min(self.slots, self.max_batch - len(adm))
            took = 0
            if pend and room > 0:
                free, popleft, push = self.free, pend.popleft, adm.append
                now = time.perf_counter()
                while pend and took < room:
                    r = pend[0]
                    nb = r.n * R
                    if nb > free:
                        break
                    free -= nb
                    popleft()
                    r.t_admit = now
                    push(r)
                    took += 1
                self.free = free
            if took:
                self.slots -= took
                if not self.stats.t_first:  # admission is in arrival order
                    self.stats.t_first = adm[-took].t_arrival
                worked = True
            if s_idx is None or not adm:
                return worked
            batch, self.admitted = adm, []
        # launch on the idle stream
        t_host = time.perf_counter()
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
                    r._fail(BackendError(f"launch failed: {e}"))
            self._notify_done()
            return True
        now = time.perf_counter()
        for r in batch:
            r.t_launch = now
        with self.lock:
            self.inflight[s_idx] = (tok, batch)
            self.stats.batches += 1
            self.stats.launch_host_s += now - t_host
        return True

    def _run(self):
        while True:
            if self.step():
                continue
            with self.lock:
                idle = not (self.pending or self.admitted or self.inflight or self.res_pending
                            or self.res_inflight)
                if self._stop and idle:
                    return
                if idle:
                    # a client that appends after this check sees _sleeping
                    # set and notifies; the timeout only bounds a lost race
                    self._sleeping = True
                    if not (self.pending or self.res_pending):
                        self.lock.wait(timeout=0.01)
                    self._sleeping = False
                    continue
            time.sleep(self.poll_s)
