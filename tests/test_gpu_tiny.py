"""GPU parity of the wave-level sorter for jobs of at most 256 records (tiny
arrays and tiny bins): exhaustive 0-1 inputs for small sizes (the 0-1
principle, Knuth 5.3.4, is what pins a comparator network), and random keys
with many duplicates for every size 1..256, element by element against the
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


def _zero_one_rows(n):
    """Every 0/1 sequence of length n, one per row."""
    return ((np.arange(1 << n, dtype=np.int64)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)


@pytest.mark.parametrize("n_lo,n_hi", [(13, 16), (17, 20)])
def test_every_zero_one_input_13_to_20(n_lo, n_hi):
    """Every 0/1 key sequence of each length n_lo..n_hi: the 16-lane segments
    (four jobs per pass) up to 16 records, the 32-lane ones (two per pass)
    above.  16-byte records, the key's top byte 0 or 1, the input index in
    the payload word; checked at once per length: the zeros in input order,
    then the ones."""
    r, k = 16, 8
    for n in range(n_lo, n_hi + 1):
        bits = _zero_one_rows(n)
        cnt = bits.shape[0]
        a = np.zeros((cnt, n, 2), dtype="<u8")
        a[:, :, 0] = bits.astype(np.uint64) << np.uint64(56)
        a[:, :, 1] = np.arange(n, dtype=np.uint64)[None, :]
        flat = a.view(np.uint8).reshape(cnt * n, r)
        sizes = np.full(cnt, n, dtype=np.int64)
        out, _ = _batch_sort(flat, sizes, r, k)
        got = out.reshape(cnt, n, r).view("<u8").reshape(cnt, n, 2)
        order = np.argsort(bits, axis=1, kind="stable")
        exp = np.take_along_axis(a, order[:, :, None], axis=1)
        assert np.array_equal(got, exp), f"n = {n}"


@pytest.mark.parametrize("n", [65, 100, 128, 129, 200, 256])
def test_random_zero_one_inputs_wide_jobs(n):
    """Random 0/1 keys for the two- and four-records-per-lane networks
    (exhaustive inputs are out of reach there), many arrays per size."""
    r, k = 16, 8
    rng = np.random.default_rng(n)
    cnt = 2048
    bits = rng.integers(0, 2, size=(cnt, n), dtype=np.uint8)
    bits[0] = 0
    bits[1] = 1
    bits[2, : n // 2] = 1
    a = np.zeros((cnt, n, 2), dtype="<u8")
    a[:, :, 0] = bits.astype(np.uint64) << np.uint64(56)
    a[:, :, 1] = np.arange(n, dtype=np.uint64)[None, :]
    out, _ = _batch_sort(a.view(np.uint8).reshape(cnt * n, r), np.full(cnt, n, dtype=np.int64), r, k)
    got = out.reshape(cnt, n, r).view("<u8").reshape(cnt, n, 2)
    exp = np.take_along_axis(a, np.argsort(bits, axis=1, kind="stable")[:, :, None], axis=1)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("r,k", [(16, 8), (8, 8), (32, 16), (16, 16)])
def test_sizes_1_to_256_against_the_oracle(r, k):
    rng = np.random.default_rng(r * 1000 + k)
    arrays = []
    for n in range(1, 257):
        for distinct in (None, 2, max(1, n // 3)):
            arrays.append(wl.random_records(rng, n, r, k, distinct_keys=distinct))
    sizes = np.array([a.shape[0] for a in arrays], dtype=np.int64)
    out, starts = _batch_sort(np.concatenate(arrays), sizes, r, k)
    for a, s in zip(arrays, starts):
        assert np.array_equal(out[s:s + a.shape[0]], oracle.sort(a, k))


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
    """Arrays on both sides of the 64-, 128- and 256-record boundaries in one
    call, in mixed groups of four."""
    rng = np.random.default_rng(9)
    sizes = np.array([63, 64, 65, 1, 2, 128, 64, 5000, 17, 129, 255, 256, 257, 3, 130, 300, 16,
                      200], dtype=np.int64)
    arrays = [wl.random_records(rng, int(n), 16, 8, distinct_keys=7) for n in sizes]
    out, starts = _batch_sort(np.concatenate(arrays), sizes, 16, 8)
    for a, s in zip(arrays, starts):
        assert np.array_equal(out[s:s + a.shape[0]], oracle.sort(a, 8))


@pytest.mark.parametrize("knobs", [{"wave_job_max": 1}, {"wave_job_max": 1, "es_job_max": 256, "tiny_max": 256},
                                   {"wave_job_max": 100, "es_job_max": 40}, {"wave_job_max": 64}])
@pytest.mark.parametrize("r,k", [(16, 8), (32, 16), (8, 5)])
def test_small_array_methods_against_the_oracle(knobs, r, k):
    """The same arrays of 1..300 records through each small-array method the
    tuning can select (wave network off or capped, one enumeration sort over
    whole jobs of up to 256 records)."""
    from gpu_helpers import tuned
    rng = np.random.default_rng(r + k)
    arrays = [wl.random_records(rng, n, r, k, distinct_keys=d)
              for n in list(range(1, 70)) + [100, 127, 128, 129, 200, 255, 256, 257, 300]
              for d in (None, 3)]
    sizes = np.array([a.shape[0] for a in arrays], dtype=np.int64)
    with tuned(**knobs):
        out, starts = _batch_sort(np.concatenate(arrays), sizes, r, k)
    for a, s in zip(arrays, starts):
        assert np.array_equal(out[s:s + a.shape[0]], oracle.sort(a, k))
