"""GPU parity of the batched entry point (many uneven arrays in one set of
launches) and of its replay from a captured HIP graph."""

import numpy as np
import pytest
import torch

import oracle
from paper_1703_00687_amd import binding as b
from paper_1703_00687_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run_batch(host_arrays, r, k):
    devs = [torch.from_numpy(a.reshape(-1).copy()).cuda() if a.shape[0] else
            torch.empty(16, dtype=torch.uint8, device="cuda") for a in host_arrays]
    views = [d[: a.shape[0] * r].view(a.shape[0], r) if a.shape[0] else d[:0].view(0, r)
             for d, a in zip(devs, host_arrays)]
    tmps = [torch.empty_like(d) for d in devs]
    total = sum(a.shape[0] for a in host_arrays)
    bt = b.Batch(len(host_arrays), total, r, k)
    bt.set_arrays(views, tmps)
    bt.launch()
    st, stats = bt.check()
    assert st == b.OK, stats
    return [v.cpu().numpy() for v in views], stats


@pytest.mark.parametrize("r,k", [(16, 8), (32, 16), (8, 8), (24, 11)])
def test_batch_uneven_sizes(r, k):
    cap = b.raduls_mid_capacity(r, k)
    sizes = [0, 1, 2, 5, 33, 1000, cap - 1, cap, cap + 1, 50000, 123457, 3, 0, 77]
    rng = np.random.default_rng(r + k)
    arrays = [wl.random_records(rng, s, r, k, distinct_keys=max(1, s // 3)) for s in sizes]
    outs, stats = _run_batch(arrays, r, k)
    for a, o in zip(arrays, outs):
        assert np.array_equal(o, oracle.sort(a, k))


def test_batch_many_small_arrays():
    sizes = wl.batch_sizes(3000, max_log2=12)
    arrays = []
    off = 0
    for j, s in enumerate(sizes):
        arrays.append(wl.batch_array(j, int(s), off))
        off += int(s)
    outs, stats = _run_batch(arrays, 16, 8)
    for a, o in zip(arrays, outs):
        assert np.array_equal(o, oracle.sort(a, 8))



@pytest.mark.parametrize("r,k", [(16, 8), (32, 16)])
def test_batch_runs_finished_in_tmp(r, k):
    """Arrays whose records hold two keys that differ in the top byte, each
    key on more records than one LDS job: every array's runs end in tmp
    after the top round and come back as copy jobs (pieces of at most
    mid_max) among the other arrays' sort jobs."""
    cap = b.raduls_server_max_records(r, k)  # mid_max of this layout
    rng = np.random.default_rng(41 + r)
    arrays, pieces = [], 0
    for ca, cb in ((cap + 1, cap + 3), (2 * cap, 5), (3 * cap + 1, 2 * cap + 1), (0, 0),
                   (700, 1200)):
        a = wl.random_records(rng, ca + cb, r, k)
        lo, hi = np.zeros(k, np.uint8), np.zeros(k, np.uint8)
        lo[k - 1], hi[k - 1] = 0x21, 0xC4
        which = rng.permutation(np.r_[np.zeros(ca, bool), np.ones(cb, bool)])
        a[:, :k] = np.where(which[:, None], hi, lo)
        arrays.append(a)
        if ca + cb > cap:  # (a smaller array is one LDS job as a whole)
            pieces += sum(-(-c // cap) for c in (ca, cb) if c > cap)
    outs, stats = _run_batch(arrays, r, k)
    for a, o in zip(arrays, outs):
        assert np.array_equal(o, oracle.sort(a, k))
    assert stats["copy_jobs"] == pieces, stats

def test_batch_total_capacity_error_is_reported():
    a = torch.from_numpy(wl.uniform16(1000).reshape(-1).copy()).cuda().view(1000, 16)
    t = torch.empty_like(a)
    bt = b.Batch(1, 500, 16, 8)  # sized for fewer records than given
    bt.set_arrays([a], [t])
    bt.launch()
    st, stats = bt.check()
    assert st == b.E_DEVICE and stats["error"] & 8


def test_batch_graph_replay_new_contents():
    sizes = [3, 700, 9000, 40000, 1, 0, 12345]
    r, k = 16, 8
    devs = [torch.empty((max(s, 1), r), dtype=torch.uint8, device="cuda") for s in sizes]
    views = [d[:s] for d, s in zip(devs, sizes)]
    tmps = [torch.empty_like(d) for d in devs]
    bt = b.Batch(len(sizes), sum(sizes), r, k)
    bt.set_arrays(views, tmps)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.launch(stream=s)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.launch()
    for rep in range(3):
        rng = np.random.default_rng(100 + rep)
        hosts = [wl.random_records(rng, sz, r, k, distinct_keys=max(1, sz // 5)) for sz in sizes]
        for v, h in zip(views, hosts):
            if h.shape[0]:
                v.copy_(torch.from_numpy(h))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st, stats = bt.check()
        assert st == b.OK, stats
        for v, h in zip(views, hosts):
            assert np.array_equal(v.cpu().numpy(), oracle.sort(h, k))
