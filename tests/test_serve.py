"""The serving loop's scheduling logic on the CPU, with a stand-in backend
that sorts with the oracle after a simulated device delay."""

import threading
import time

import numpy as np
import pytest

import oracle
from paper_1703_00687_amd import serve
from paper_1703_00687_amd import workloads as wl


class FakeBackend:
    def __init__(self, n_streams=2, max_batch=8, key_bytes=8, delay_s=0.002, fail_launch=None,
                 fail_finish=None):
        self.n_streams, self.max_batch, self.key_bytes = n_streams, max_batch, key_bytes
        self.delay_s = delay_s
        self.fail_launch = fail_launch or (lambda reqs: False)
        self.fail_finish = fail_finish or (lambda reqs: False)
        self.lock = threading.Lock()
        self.inflight_bytes = 0
        self.max_inflight_bytes = 0
        self.max_concurrent_batches = 0
        self.active = 0
        self.batch_sizes = []

    def prepare(self, stream_idx, reqs):
        for r in reqs:
            r.tmp = np.empty((max(r.n, 1), 16), dtype=np.uint8)
        return True

    def launch(self, stream_idx, reqs):
        if self.fail_launch(reqs):
            raise RuntimeError("injected launch failure")
        with self.lock:
            self.active += 1
            self.max_concurrent_batches = max(self.max_concurrent_batches, self.active)
            b = sum(r.n * r.recs.shape[1] for r in reqs)
            self.inflight_bytes += b
            self.max_inflight_bytes = max(self.max_inflight_bytes, self.inflight_bytes)
            self.batch_sizes.append(len(reqs))
        return (time.perf_counter() + self.delay_s, b)

    def done(self, token):
        return time.perf_counter() >= token[0]

    def finish(self, stream_idx, token, reqs):
        with self.lock:
            self.active -= 1
            self.inflight_bytes -= token[1]
        if self.fail_finish(reqs):
            return ["injected device error"] * len(reqs)
        for r in reqs:
            r.recs[:] = oracle.sort(r.recs, self.key_bytes)
            r.tmp = None
        return [None] * len(reqs)


def _arrays(count, seed=0, max_log2=12):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(0, 1 << max_log2, size=count)
    return [wl.random_records(rng, int(s), 16, 8, distinct_keys=max(1, int(s) // 4)) for s in sizes]


def test_all_requests_sorted_and_counted():
    be = FakeBackend()
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=16).start()
    arrays = _arrays(200)
    expect = [oracle.sort(a, 8) for a in arrays]
    futs = [srv.submit(a) for a in arrays]
    outs = [f.result(timeout=30) for f in futs]
    summary = srv.stop()
    for o, e in zip(outs, expect):
        assert np.array_equal(o, e)
    assert summary["requests"] == 200 and summary["failed"] == 0
    assert summary["p99_ms"] >= summary["p50_ms"] >= 0
    assert summary["records"] == sum(a.shape[0] for a in arrays)


def test_budget_and_slots_bound_what_is_in_flight():
    be = FakeBackend(n_streams=3, max_batch=4, delay_s=0.003)
    budget = 200_000
    srv = serve.Server(be, rec_bytes=16, budget_bytes=budget, max_slots=5).start()
    futs = [srv.submit(a) for a in _arrays(120, seed=1)]
    for f in futs:
        f.result(timeout=30)
    srv.stop()
    assert be.max_inflight_bytes <= budget
    assert max(be.batch_sizes) <= 4


def test_batches_overlap_across_streams():
    be = FakeBackend(n_streams=2, max_batch=2, delay_s=0.02)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 24, max_slots=8).start()
    futs = [srv.submit(a) for a in _arrays(12, seed=2)]
    for f in futs:
        f.result(timeout=30)
    srv.stop()
    assert be.max_concurrent_batches == 2


def test_arrival_order_admission_and_continuous_batching():
    # a request larger than what is free waits at the head; nothing overtakes it
    be = FakeBackend(n_streams=1, max_batch=8, delay_s=0.02)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=16 * 1000, max_slots=8).start()
    small = wl.random_records(np.random.default_rng(3), 600, 16, 8)
    big = wl.random_records(np.random.default_rng(4), 900, 16, 8)
    tail = wl.random_records(np.random.default_rng(5), 10, 16, 8)
    f1 = srv.submit(small)
    time.sleep(0.005)          # small is running now
    f2 = srv.submit(big)       # needs 900 > 400 free: waits
    f3 = srv.submit(tail)      # would fit, but must not overtake big
    f1.result(timeout=10)
    f2.result(timeout=10)
    f3.result(timeout=10)
    srv.stop()
    assert f2.result().shape[0] == 900
    # big and tail were admitted after small completed, as one batch
    assert be.batch_sizes[0] == 1 and be.batch_sizes[1] == 2


def test_oversize_request_rejected():
    be = FakeBackend()
    srv = serve.Server(be, rec_bytes=16, budget_bytes=16 * 100, max_slots=4).start()
    f = srv.submit(wl.random_records(np.random.default_rng(6), 101, 16, 8))
    with pytest.raises(serve.Rejected):
        f.result(timeout=5)
    ok = srv.submit(wl.random_records(np.random.default_rng(7), 100, 16, 8))
    assert ok.result(timeout=5).shape[0] == 100
    assert srv.stop()["rejected"] == 1


def test_cancel_before_launch():
    be = FakeBackend(n_streams=1, max_batch=1, delay_s=0.05)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=1).start()
    a = _arrays(3, seed=8)
    f1 = srv.submit(a[0])
    f2 = srv.submit(a[1])
    time.sleep(0.01)
    assert srv.cancel(f2)
    with pytest.raises(serve.Cancelled):
        f2.result(timeout=5)
    f3 = srv.submit(a[2])
    f1.result(timeout=5)
    f3.result(timeout=5)
    s = srv.stop()
    assert s["cancelled"] == 1 and s["requests"] == 2


def test_backend_failures_fail_only_their_batch():
    state = {"n": 0}

    def fail_every_third(reqs):
        state["n"] += 1
        return state["n"] % 3 == 0

    be = FakeBackend(n_streams=1, max_batch=1, fail_finish=fail_every_third)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=4).start()
    futs = [srv.submit(a) for a in _arrays(9, seed=9)]
    errors = 0
    for f in futs:
        try:
            f.result(timeout=10)
        except serve.BackendError:
            errors += 1
    s = srv.stop()
    assert errors == 3 and s["failed"] == 3 and s["requests"] == 6

    be2 = FakeBackend(fail_launch=lambda reqs: True)
    srv2 = serve.Server(be2, rec_bytes=16, budget_bytes=1 << 20, max_slots=4).start()
    f = srv2.submit(_arrays(1, seed=10)[0])
    with pytest.raises(serve.BackendError):
        f.result(timeout=5)
    srv2.stop()
    assert srv2.free == srv2.budget and srv2.slots == srv2.max_slots


def test_stop_without_drain_cancels_pending():
    be = FakeBackend(n_streams=1, max_batch=1, delay_s=0.05)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=1).start()
    futs = [srv.submit(a) for a in _arrays(5, seed=11)]
    time.sleep(0.01)
    s = srv.stop(drain=False)
    assert s["cancelled"] >= 3
    done = sum(1 for f in futs if f.done() and f.exception() is None)
    assert done >= 1


def test_arena_first_fit_and_coalescing():
    a = serve.Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(2000) is None
    a.release(y, 1000)
    assert a.alloc(1100) is None      # the hole is 1024 bytes
    a.release(x, 1000)
    assert a.alloc(2000) == 0          # coalesced with the first hole
    a.release(0, 2000)
    a.release(z, 1000)
    assert a.free == [(0, 4096)]


def test_budget_above_backend_capacity_is_refused():
    be = FakeBackend(n_streams=1, max_batch=4)
    be.capacity_bytes = 1000
    with pytest.raises(ValueError):
        serve.Server(be, rec_bytes=16, budget_bytes=1001, max_slots=4)
    serve.Server(be, rec_bytes=16, budget_bytes=1000, max_slots=4)  # at the capacity: fine


def test_submit_many_keeps_order_and_rejects_only_oversize():
    be = FakeBackend(n_streams=2, max_batch=4, delay_s=0.001)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=16 * 5000, max_slots=8).start()
    arrays = _arrays(12, seed=21)
    big = wl.random_records(np.random.default_rng(22), 6000, 16, 8)  # above the budget
    batch = arrays[:6] + [big] + arrays[6:]
    expect = [oracle.sort(a, 8) for a in batch]
    futs = srv.submit_many(batch)
    with pytest.raises(serve.Rejected):
        futs[6].result(timeout=5)
    for i, f in enumerate(futs):
        if i != 6:
            assert np.array_equal(f.result(timeout=30), expect[i])
    s = srv.stop()
    assert s["requests"] == 12 and s["rejected"] == 1
    assert srv.free == srv.budget and srv.slots == srv.max_slots


def test_ticket_times_out_while_pending():
    be = FakeBackend(n_streams=1, max_batch=1, delay_s=0.2)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=1).start()
    f = srv.submit(_arrays(1, seed=23)[0])
    with pytest.raises(TimeoutError):
        f.result(timeout=0.01)
    assert f.result(timeout=10) is not None and f.done()
    srv.stop()


class FakeResidentBackend(FakeBackend):
    """FakeBackend plus a resident path for requests of at most `cap`
    records: a ring of `slots` entries that the stand-in device completes in
    ticket order `res_delay_s` after submission (sorting with the oracle);
    a readiness token is a callable that says whether the input is written."""

    def __init__(self, cap=100, slots=4, res_delay_s=0.002, fail_ticket=None, **kw):
        super().__init__(**kw)
        self.resident_cap = cap
        self.slots, self.res_delay_s, self.fail_ticket = slots, res_delay_s, fail_ticket
        self.ring = []            # (ticket, due, request)
        self.next = self.through = 0
        self.resident_sizes = []
        self.max_outstanding = 0

    def ready_done(self, token):
        return token is None or token()

    def _advance(self):
        now = time.perf_counter()
        while self.ring and self.ring[0][1] <= now:
            t, _, req = self.ring.pop(0)
            req.recs[:] = oracle.sort(req.recs, self.key_bytes)
            self.through = t + 1

    def resident_submit(self, req):
        self._advance()
        if self.next - self.through >= self.slots:
            return 1, 0
        t = self.next
        self.next += 1
        self.ring.append((t, time.perf_counter() + self.res_delay_s, req))
        self.resident_sizes.append(req.n)
        self.max_outstanding = max(self.max_outstanding, self.next - self.through)
        return 0, t

    def resident_completed(self):
        before = self.through
        self._advance()
        bad = self.fail_ticket is not None and before <= self.fail_ticket < self.through
        return self.through, (7 if bad else 0)

    def resident_status(self, ticket):
        return 7 if ticket == self.fail_ticket else 0


def test_resident_path_takes_small_requests_and_batches_the_rest():
    be = FakeResidentBackend(cap=100, n_streams=2, max_batch=8)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=8).start()
    rng = np.random.default_rng(31)
    sizes = [50, 500, 20, 1000, 0, 100, 101, 7]
    arrays = [wl.random_records(rng, n, 16, 8, distinct_keys=max(1, n // 3)) for n in sizes]
    expect = [oracle.sort(a, 8) for a in arrays]
    futs = [srv.submit(a) for a in arrays[:4]] + srv.submit_many(arrays[4:])
    for f, e in zip(futs, expect):
        assert np.array_equal(f.result(timeout=30), e)
    s = srv.stop()
    assert be.resident_sizes == [n for n in sizes if n <= 100]  # in arrival order
    assert sum(be.batch_sizes) == 3  # the three larger requests went to batches
    assert s["requests"] == len(sizes) and srv.free == srv.budget and srv.slots == srv.max_slots


def test_resident_request_waits_for_its_input():
    be = FakeResidentBackend(cap=100)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=8).start()
    written = threading.Event()
    a = wl.random_records(np.random.default_rng(32), 60, 16, 8)
    f = srv.submit(a, ready=written.is_set)
    b2 = srv.submit(wl.random_records(np.random.default_rng(33), 30, 16, 8), ready=False)
    time.sleep(0.05)
    # nothing overtakes a request whose input is not written yet
    assert be.resident_sizes == [] and not f.done() and not b2.done()
    written.set()
    assert np.array_equal(f.result(timeout=10), oracle.sort(a, 8))
    b2.result(timeout=10)
    srv.stop()
    assert be.resident_sizes == [60, 30]


def test_resident_ring_full_holds_requests_back():
    be = FakeResidentBackend(cap=100, slots=2, res_delay_s=0.003)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=8).start()
    arrays = _arrays(12, seed=34, max_log2=6)
    futs = [srv.submit(a) for a in arrays]
    for f, a in zip(futs, arrays):
        assert np.array_equal(f.result(timeout=30), oracle.sort(a, 8))
    srv.stop()
    assert be.max_outstanding <= 2 and len(be.resident_sizes) == 12


def test_resident_failure_fails_only_its_request():
    be = FakeResidentBackend(cap=100, fail_ticket=1)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=8).start()
    arrays = _arrays(4, seed=35, max_log2=6)
    futs = [srv.submit(a) for a in arrays]
    with pytest.raises(serve.BackendError):
        futs[1].result(timeout=10)
    for i in (0, 2, 3):
        assert np.array_equal(futs[i].result(timeout=10), oracle.sort(arrays[i], 8))
    s = srv.stop()
    assert s["failed"] == 1 and s["requests"] == 3


def test_resident_request_cancelled_before_publication():
    be = FakeResidentBackend(cap=100)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=8).start()
    never = threading.Event()
    f = srv.submit(wl.random_records(np.random.default_rng(36), 40, 16, 8), ready=never.is_set)
    time.sleep(0.01)
    assert srv.cancel(f)
    with pytest.raises(serve.Cancelled):
        f.result(timeout=5)
    s = srv.stop()
    assert be.resident_sizes == [] and s["cancelled"] == 1


def test_resident_server_gone_fails_small_requests_and_serves_the_rest():
    """A backend whose resident server has stopped (submits refused with a
    negative status, completions raising): small requests fail with a
    backend error, larger ones still go to batches, and nothing hangs."""

    class Gone(FakeResidentBackend):
        def resident_submit(self, req):
            return -9, 0

        def resident_completed(self):
            raise RuntimeError("resident server closed")

    be = Gone(cap=100, n_streams=2, max_batch=8)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=1 << 20, max_slots=8).start()
    rng = np.random.default_rng(37)
    sizes = [40, 400, 7, 1000]
    arrays = [wl.random_records(rng, n, 16, 8) for n in sizes]
    futs = [srv.submit(a) for a in arrays]
    for f, a, n in zip(futs, arrays, sizes):
        if n <= 100:
            with pytest.raises(serve.BackendError):
                f.result(timeout=10)
        else:
            assert np.array_equal(f.result(timeout=10), oracle.sort(a, 8))
    s = srv.stop()
    assert s["failed"] == 2 and s["requests"] == 2
