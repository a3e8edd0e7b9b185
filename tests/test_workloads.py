"""The device twins of the workload generators draw exactly the host
streams (run here on torch's CPU backend, so no GPU is needed)."""

import numpy as np
import pytest

from paper_1703_00687_amd import workloads as wl


@pytest.mark.parametrize("n", [0, 1, 1000, 70001])
def test_device_twins_match_host_generators(n):
    torch = pytest.importorskip("torch")
    assert np.array_equal(wl.uniform16(n), wl.uniform16_torch(n, device="cpu", chunk=4096).numpy())
    # a small dictionary keeps the test quick; the draws are the same code
    assert np.array_equal(wl.zipf16(n, values=1 << 12),
                          wl.zipf16_torch(n, values=1 << 12, device="cpu", chunk=4096).numpy())
    assert np.array_equal(wl.deep32(n), wl.deep32_torch(n, device="cpu", chunk=4096).numpy())
    starts = np.array([0, 7, 7, 100], dtype=np.int64)
    sizes = np.array([7, 0, 93, 13], dtype=np.int64)
    for j, (a, s) in enumerate(zip(starts, sizes)):
        dev = wl.batch_array_torch(j, int(s), int(a), device="cpu").numpy()
        assert np.array_equal(dev, wl.batch_array(j, int(s), int(a)))


def test_zipf_shape():
    recs = wl.zipf16(1 << 16, values=1 << 16)
    keys = recs[:, :8].copy().view("<u8").ravel()
    _, counts = np.unique(keys, return_counts=True)
    # the shared override key takes about 5% of the records, and the most
    # frequent Zipf rank several percent more
    assert 0.03 < counts.max() / keys.size < 0.2
    assert np.array_equal(recs[:, 8:].copy().view("<u8").ravel(), np.arange(1 << 16))


@pytest.mark.parametrize("r,k", [(8, 8), (16, 8), (16, 16), (24, 8), (24, 16), (32, 16),
                                 (48, 8), (64, 16)])
def test_sweep_records_twins_and_layout(r, k):
    pytest.importorskip("torch")
    n = 5003
    host = wl.sweep_records(n, r, k)
    assert host.shape == (n, r)
    assert np.array_equal(host, wl.sweep_records_torch(n, r, k, device="cpu", chunk=1024).numpy())
    w = host.view("<u8").reshape(n, r // 8)
    if r > k:  # the word after the key holds the index
        assert np.array_equal(w[:, k // 8], np.arange(n, dtype=np.uint64))
    # key words look uniform: each of the 8 top bits is set about half the time
    top = (w[:, k // 8 - 1] >> np.uint64(56)).astype(np.int64)
    for bit in range(8):
        assert abs(((top >> bit) & 1).mean() - 0.5) < 0.05


def test_named_device_builders_match_host():
    pytest.importorskip("torch")
    for name in ("uniform8", "uniform16", "deep32", "keys16"):
        host, _ = wl.make(name, 4099)
        assert np.array_equal(host, wl.make_torch(name, 4099, device="cpu").numpy()), name
