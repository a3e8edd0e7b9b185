"""GPU: the serving loop returns for every request exactly what the plain
per-call sort returns for it alone, while requests arrive during running
batches and batches overlap on several streams."""

import random
import threading
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1703_00687_amd import binding as b
from paper_1703_00687_amd import serve
from paper_1703_00687_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _requests(count, seed, max_log2=16):
    sizes = wl.batch_sizes(count, seed=seed, max_log2=max_log2)
    out, off = [], 0
    for j, s in enumerate(sizes):
        out.append(wl.batch_array(j, int(s), off, seed=seed))
        off += int(s)
    return out


def _alone(host):
    n = host.shape[0]
    t = torch.from_numpy(host.copy()).cuda()
    tmp = torch.empty(b.raduls_tmp_bytes(n, 16, 8), dtype=torch.uint8, device="cuda")
    b.raduls_sort(t, tmp, n, 16, 8)
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("use_graphs", [True, False])
def test_results_identical_alone_and_in_the_mix(use_graphs):
    hosts = _requests(300, seed=21 + int(use_graphs))
    alone = [_alone(h) for h in hosts]
    for h, a in zip(hosts[:40], alone[:40]):
        assert np.array_equal(a, oracle.sort(h, 8))
    budget = 64 << 20
    be = serve.GpuBackend(16, 8, n_streams=3, max_batch=32, max_records=budget // 16,
                          use_graphs=use_graphs)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=budget, max_slots=48).start()
    devs = [torch.from_numpy(h.copy()).cuda() for h in hosts]
    torch.cuda.synchronize()
    futs = [None] * len(devs)
    rng = random.Random(5)

    def producer():
        for i, d in enumerate(devs):
            futs[i] = srv.submit(d)
            time.sleep(rng.expovariate(1.0 / 50e-6))  # Poisson arrivals, 50 us mean gap

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    outs = [f.result(timeout=60) for f in futs]
    summary = srv.stop()
    for o, a in zip(outs, alone):
        assert np.array_equal(o.cpu().numpy(), a)
    assert summary["requests"] == len(hosts) and summary["failed"] == 0
    assert summary["batches"] >= 2


def test_submit_orders_after_the_producing_stream():
    # inputs written on a side stream and submitted at once, with no global
    # synchronize: each sort must wait for its input's writes
    hosts = _requests(40, seed=31, max_log2=18)
    budget = 64 << 20
    be = serve.GpuBackend(16, 8, n_streams=3, max_batch=16, max_records=budget // 16,
                          use_graphs=True)
    srv = serve.Server(be, rec_bytes=16, budget_bytes=budget, max_slots=32).start()
    srcs = [torch.from_numpy(h.copy()).cuda() for h in hosts]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    futs, outs = [], []
    with torch.cuda.stream(side):
        for s in srcs:
            d = torch.empty_like(s)
            torch.cuda._sleep(200_000)  # keeps the side stream busy past submission
            d.copy_(s)
            outs.append(d)
            futs.append(srv.submit(d))
    res = [f.result(timeout=60) for f in futs]
    srv.stop()
    torch.cuda.synchronize()
    for r, h in zip(res, hosts):
        assert np.array_equal(r.cpu().numpy(), oracle.sort(h, 8))


def test_budget_larger_than_backend_scratch_is_refused():
    be = serve.GpuBackend(16, 8, n_streams=1, max_batch=4, max_records=1024, use_graphs=False)
    with pytest.raises(ValueError):
        serve.Server(be, rec_bytes=16, budget_bytes=1024 * 16 + 1, max_slots=4)


def test_small_requests_through_the_resident_server():
    """With a resident server in the backend, requests of at most one LDS
    job go to it and the others to batched launches; every result equals the
    plain call's.  The inputs are written on the current stream and
    submitted at once (each sort waits for its producer's event); nothing
    synchronizes the whole device while the resident kernel runs."""
    hosts = _requests(200, seed=27)
    alone = [_alone(h) for h in hosts]
    budget = 64 << 20
    be = serve.GpuBackend(16, 8, n_streams=2, max_batch=16, max_records=budget // 16,
                          resident_workgroups=4, resident_slots=64)
    try:
        cap = be.resident_cap
        assert cap == b.raduls_server_max_records(16, 8)
        srv = serve.Server(be, rec_bytes=16, budget_bytes=budget, max_slots=32).start()
        stream = torch.cuda.current_stream()
        devs = []
        futs = []
        for h in hosts:
            d = torch.empty(h.shape, dtype=torch.uint8, device="cuda")
            d.copy_(torch.from_numpy(h), non_blocking=False)
            d.add_(0)  # (a kernel on the current stream writes it last)
            devs.append(d)
            futs.append(srv.submit(d))
        res = [f.result(timeout=60) for f in futs]
        s = srv.stop()
        stream.synchronize()
        assert s["requests"] == len(hosts) and s["failed"] == 0
        assert any(h.shape[0] <= cap for h in hosts) and any(h.shape[0] > cap for h in hosts)
        for r, a in zip(res, alone):
            assert np.array_equal(r.cpu().numpy(), a)
    finally:
        be.close()
    torch.cuda.synchronize()
