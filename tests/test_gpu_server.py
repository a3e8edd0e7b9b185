"""The resident server (raduls_server_* in raduls.h): requests sorted by
workgroups that stay on the device, checked against the oracle alone and,
in a mix with plain calls running meanwhile, against the plain call's bytes;
and its host-side contracts (oversize, alignment, busy slots, the idle limit,
stop)."""

import time

import numpy as np
import pytest
import torch

import oracle
from paper_1703_00687_amd import binding as b
from paper_1703_00687_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
IDLE_MS = 30000  # every test's server leaves by itself within this if a test breaks


def _device(h: np.ndarray) -> torch.Tensor:
    t = torch.empty(h.shape, dtype=torch.uint8, device=DEV)
    if h.size:
        t.copy_(torch.from_numpy(h))
    return t


@pytest.mark.parametrize("r,k", [(16, 8), (8, 8), (32, 16), (16, 16), (24, 5)])
def test_server_alone_matches_oracle(r, k):
    cap = b.raduls_server_max_records(r, k)
    sizes = [n for n in (0, 1, 2, 3, 17, 64, 65, 255, 256, 257, 1000, 3000) if n < cap]
    sizes += [cap - 1, cap]
    rng = np.random.default_rng(r * 100 + k)
    hosts = [wl.random_records(rng, n, r, k, distinct_keys=max(1, n // 3)) for n in sizes]
    devs = [_device(h) for h in hosts]
    torch.cuda.synchronize()  # inputs written before they are submitted
    with b.ResidentServer(r, k, slots=64, workgroups=4, idle_ms=IDLE_MS) as srv:
        assert srv.max_records == cap
        tickets = [srv.submit(d) for d in devs]
        assert tickets == list(range(len(sizes)))
        for t in tickets:
            assert srv.wait(t) == 0
        for h, d in zip(hosts, devs):
            got = d.cpu().numpy()
            assert np.array_equal(got, oracle.sort(h, k)), (r, k, h.shape)
        _, _, running, _ = srv.info()
        assert running


def test_server_in_mix_matches_plain_calls():
    """Requests of random sizes through a ring of 32 slots (so slots are
    reused many times) while plain raduls_sort calls run on the default
    stream; every served array equals the plain call's output on a copy."""
    r, k = 16, 8
    cap = b.raduls_server_max_records(r, k)
    rng = np.random.default_rng(5)
    count = 400
    sizes = rng.integers(0, cap + 1, size=count)
    sizes[:8] = [0, 1, 2, cap, cap, 64, 65, 256]
    hosts = [wl.random_records(rng, int(n), r, k, distinct_keys=max(1, int(n) // 2)) for n in sizes]
    served = [_device(h) for h in hosts]
    plain = [d.clone() for d in served]
    # plain calls on other arrays keep the rest of the GPU busy meanwhile
    other = _device(wl.random_records(rng, 1 << 20, r, k))
    tmp_other = torch.empty(b.raduls_tmp_bytes(1 << 20, r, k), dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    with b.ResidentServer(r, k, slots=32, workgroups=8, idle_ms=IDLE_MS) as srv:
        tickets = []
        for i, d in enumerate(served):
            if i % 50 == 0:
                b.raduls_sort(other, tmp_other, 1 << 20, r, k)
            while True:
                st, t = srv.submit_status(d)
                if st == b.OK:
                    tickets.append(t)
                    break
                assert st == b.E_BUSY, b.strerror(st)
                # the slot's previous request is still being sorted
                assert srv.wait(tickets[-32]) == 0
        for t in tickets:
            assert srv.wait(t) == 0
    torch.cuda.synchronize()
    for d, n in zip(plain, sizes):
        if n > 1:
            tmp = torch.empty(b.raduls_tmp_bytes(int(n), r, k), dtype=torch.uint8, device=DEV)
            b.raduls_sort(d, tmp, int(n), r, k)
    torch.cuda.synchronize()
    for i, (s, p) in enumerate(zip(served, plain)):
        assert torch.equal(s, p), (i, int(sizes[i]))
    # and a sample against the oracle
    for i in rng.choice(count, size=12, replace=False):
        assert np.array_equal(served[i].cpu().numpy(), oracle.sort(hosts[i], k))


def test_server_rejects_oversize_and_misaligned():
    r, k = 16, 8
    cap = b.raduls_server_max_records(r, k)
    buf = torch.zeros((cap + 2) * r + 64, dtype=torch.uint8, device=DEV)
    with b.ResidentServer(r, k, slots=8, workgroups=1, idle_ms=IDLE_MS) as srv:
        assert srv.submit_status(buf, cap + 1)[0] == b.E_UNSUPPORTED
        assert srv.submit_status(buf.data_ptr() + 8, 10)[0] == b.E_ALIGN
        assert srv.submit_status(None, 5)[0] == b.E_INVALID
        # nothing was queued by the refused calls: the next ticket is 0
        t = srv.submit(buf, 3)
        assert t == 0 and srv.wait(t) == 0


def test_server_busy_slot_then_free():
    r, k = 16, 8
    h = wl.random_records(np.random.default_rng(9), 3000, r, k)
    d = _device(h)
    e = _device(h)
    torch.cuda.synchronize()
    with b.ResidentServer(r, k, slots=1, workgroups=1, idle_ms=IDLE_MS) as srv:
        t0 = srv.submit(d)
        st, t1 = srv.submit_status(e)
        # the one slot is free again only once request 0 has completed
        assert st in (b.OK, b.E_BUSY)
        assert srv.wait(t0) == 0
        if st == b.E_BUSY:
            t1 = srv.submit(e)
        assert t1 == 1 and srv.wait(t1) == 0
    expect = oracle.sort(h, k)
    assert np.array_equal(d.cpu().numpy(), expect) and np.array_equal(e.cpu().numpy(), expect)


def test_server_idle_limit_ends_the_kernel_and_submit_relaunches():
    r, k = 16, 8
    h = wl.random_records(np.random.default_rng(21), 700, r, k, distinct_keys=90)
    d = _device(h)
    torch.cuda.synchronize()
    srv = b.ResidentServer(r, k, slots=8, workgroups=2, idle_ms=50)
    try:
        deadline = time.time() + 20
        while srv.info()[2] and time.time() < deadline:
            time.sleep(0.05)
        _, _, running, reason = srv.info()
        assert not running and reason == 2
        # the next submit relaunches the kernel on the same ring and state
        t = srv.submit(d)
        assert t == 0 and srv.wait(t) == 0
        assert np.array_equal(d.cpu().numpy(), oracle.sort(h, k))
    finally:
        srv.close()


def test_server_lease_relaunches_under_load():
    """A lease of 1 ms: the kernel leaves many times while requests are
    queued and the host's waits relaunch it; every request completes."""
    r, k = 16, 8
    cap = b.raduls_server_max_records(r, k)
    rng = np.random.default_rng(23)
    sizes = [int(x) for x in rng.integers(cap // 2, cap + 1, size=600)]
    hosts = [wl.random_records(rng, n, r, k, distinct_keys=max(1, n // 4)) for n in sizes]
    devs = [_device(h) for h in hosts]
    torch.cuda.synchronize()
    with b.ResidentServer(r, k, slots=1024, workgroups=2, idle_ms=IDLE_MS, lease_ms=1) as srv:
        first, acc = srv.submit_many([d.data_ptr() for d in devs], sizes)
        assert first == 0 and acc == len(sizes)
        assert srv.wait_range(0, len(sizes)) == 0
        reason = srv.info()[3]
        assert reason in (0, 3)  # running, or last left at its lease
    for i in rng.choice(len(sizes), size=40, replace=False):
        assert np.array_equal(devs[i].cpu().numpy(), oracle.sort(hosts[i], k)), i


def test_server_stop_is_prompt():
    r, k = 8, 8
    srv = b.ResidentServer(r, k, slots=8, workgroups=16, idle_ms=IDLE_MS)
    time.sleep(0.05)
    t = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t < 2.0


def test_server_submit_many_stops_at_a_busy_slot():
    r, k = 16, 8
    cap = b.raduls_server_max_records(r, k)
    rng = np.random.default_rng(13)
    sizes = [int(x) for x in rng.integers(0, cap + 1, size=40)]
    hosts = [wl.random_records(rng, n, r, k, distinct_keys=max(1, n // 4)) for n in sizes]
    devs = [_device(h) for h in hosts]
    torch.cuda.synchronize()
    ptrs = [d.data_ptr() if n else 0 for d, n in zip(devs, sizes)]
    with b.ResidentServer(r, k, slots=16, workgroups=2, idle_ms=IDLE_MS) as srv:
        # one oversize request: nothing is submitted
        with pytest.raises(b.RadulsError):
            srv.submit_many(ptrs[:3] + [ptrs[3]], sizes[:3] + [cap + 1])
        done = 0
        while done < len(sizes):
            first, acc = srv.submit_many(ptrs[done:], sizes[done:])
            assert first == done and acc <= 16
            if acc == 0:  # every slot in use: free the oldest
                assert srv.wait(done - 16) == 0
            done += acc
        assert srv.wait_range(0, len(sizes)) == 0
        with pytest.raises(b.RadulsError):
            srv.wait_range(0, len(sizes) + 1)  # a ticket not submitted yet
    for h, d in zip(hosts, devs):
        assert np.array_equal(d.cpu().numpy(), oracle.sort(h, k))


def test_two_servers_side_by_side():
    """Two servers of different record layouts at once, each with its own
    ring, queue and stream, while a plain sort runs on the default stream."""
    rng = np.random.default_rng(17)
    a_h = [wl.random_records(rng, int(n), 16, 8, distinct_keys=max(1, int(n) // 5))
           for n in rng.integers(0, 5121, size=40)]
    b_h = [wl.random_records(rng, int(n), 32, 16, distinct_keys=max(1, int(n) // 5))
           for n in rng.integers(0, b.raduls_server_max_records(32, 16) + 1, size=40)]
    a_d = [_device(h) for h in a_h]
    b_d = [_device(h) for h in b_h]
    big = _device(wl.random_records(rng, 1 << 20, 16, 8))
    big_h = big.cpu().numpy()
    tmp = torch.empty(b.raduls_tmp_bytes(1 << 20, 16, 8), dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    with b.ResidentServer(16, 8, slots=64, workgroups=4, idle_ms=IDLE_MS) as sa, \
            b.ResidentServer(32, 16, slots=64, workgroups=4, idle_ms=IDLE_MS) as sb:
        b.raduls_sort(big, tmp, 1 << 20, 16, 8)
        ta = [sa.submit(d) for d in a_d]
        tb = [sb.submit(d) for d in b_d]
        assert sa.wait_range(ta[0], len(ta)) == 0
        assert sb.wait_range(tb[0], len(tb)) == 0
        torch.cuda.current_stream().synchronize()
    for h, d in zip(a_h, a_d):
        assert np.array_equal(d.cpu().numpy(), oracle.sort(h, 8))
    for h, d in zip(b_h, b_d):
        assert np.array_equal(d.cpu().numpy(), oracle.sort(h, 16))
    assert np.array_equal(big.cpu().numpy(), oracle.sort(big_h, 8))
