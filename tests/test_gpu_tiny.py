"""GPU parity of the wave-level sorter for jobs of at most 64 records (tiny
arrays and tiny bins): exhaustive 0-1 inputs for small sizes (the 0-1
principle, Knuth 5.3.4, is what pins a comparator network), and random keys
with many duplicates for every size 1..64, element by element against the
oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_1703_00687_amd import binding as b
from paper_1703_00687_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _batch_sort(flat, sizes, r, k):
    """Sort arrays of `sizes` records stored back to back in `flat` ([N, r]
    uint8) with one batched call; returns the sorted records."""
    dev = torch.device("cuda:0")
    recs = torch.from_numpy(flat.reshape(-1).copy()).to(dev).view(-1, r)
    tmp = torch.empty_like(recs)
    starts = np.zeros(len(sizes), dtype=np.int64)
    starts[1:] = np.cumsum(sizes)[:-1]
    bt = b.Batch(len(sizes), int(sizes.sum()), r, k, device=dev)
    h = bt.host_desc.numpy()
    h[:, 0] = recs.data_ptr() + starts * r
    h[:, 1] = tmp.data_ptr() + starts * r
    h[:, 2] = sizes
    bt.desc.copy_(bt.host_desc)
    bt.launch()
    st, stats = bt.check()
    assert st == b.OK, stats
    return recs.cpu().numpy(), starts


@pytest.mark.parametrize("r,k", [(16, 8), (8, 3), (32, 16)])
def test_every_zero_one_input_up_to_12(r, k):
    """Every sequence of 0/1 keys of length 1..12 (8190 arrays); where the
    record has room, the word after the key carries the input index, so the
    stable result is unique: the zeros in input order, then the ones (with
    no room, records with equal keys are identical)."""
    arrays = []
    for n in range(1, 13):
        bits = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)
        for row in bits:
            a = np.zeros((n, r), dtype=np.uint8)
            a[:, k - 1] = row  # the key's most significant byte
            if r >= k + 8:  # room for the index after the key
                a[:, r - 8:] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
            arrays.append(a)
    sizes = np.array([a.shape[0] for a in arrays], dtype=np.int64)
    out, starts = _batch_sort(np.concatenate(arrays), sizes, r, k)
    for a, s in zip(arrays, starts):
        n = a.shape[0]
        exp = np.concatenate([a[a[:, k - 1] == 0], a[a[:, k - 1] == 1]])
        assert np.array_equal(out[s:s + n], exp)


@pytest.mark.parametrize("r,k", [(16, 8), (24, 13), (64, 16), (8, 8)])
def test_sizes_1_to_64_against_the_oracle(r, k):
    rng = np.random.default_rng(r * 100 + k)
    arrays = []
    for n in range(1, 65):
        for distinct in (None, 2, max(1, n // 3)):
            arrays.append(wl.random_records(rng, n, r, k, distinct_keys=distinct))
    sizes = np.array([a.shape[0] for a in arrays], dtype=np.int64)
    out, starts = _batch_sort(np.concatenate(arrays), sizes, r, k)
    for a, s in zip(arrays, starts):
        assert np.array_equal(out[s:s + a.shape[0]], oracle.sort(a, k))


def test_tiny_and_lds_jobs_in_one_batch():
    """Arrays on both sides of the 64-record boundary in one call."""
    rng = np.random.default_rng(9)
    sizes = np.array([63, 64, 65, 1, 2, 128, 64, 5000, 17], dtype=np.int64)
    arrays = [wl.random_records(rng, int(n), 16, 8, distinct_keys=7) for n in sizes]
    out, starts = _batch_sort(np.concatenate(arrays), sizes, 16, 8)
    for a, s in zip(arrays, starts):
        assert np.array_equal(out[s:s + a.shape[0]], oracle.sort(a, 8))
