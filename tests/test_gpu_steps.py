"""GPU parity of the individual hot-path steps through their C entry points:
digit histogram (a1), bucket offsets (a2) and one stable scatter pass (a3)."""

import numpy as np
import pytest
import torch

import oracle
from paper_1703_00687_amd import binding as b
from paper_1703_00687_amd import workloads as wl
from gpu_helpers import GUARD, guarded, guards_intact

pytestmark = pytest.mark.gpu

DIGITS = [(64, 8), (8, 8), (61, 8), (5, 8), (3, 3), (77, 1), (128, 8), (100, 7), (59, 6)]


def _inp(bits, n, seed):
    r, k = (32, 16) if bits > 64 else (16, 8)
    rng = np.random.default_rng(seed)
    return wl.random_records(rng, n, r, k, distinct_keys=max(2, n // 7)), k


def _ws(n, r, k):
    nbytes = b.raduls_step_ws_bytes(n, r, k)
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda"), nbytes


@pytest.mark.parametrize("bits,width", DIGITS)
@pytest.mark.parametrize("n", [0, 1, 5, 4097, 100003])
def test_histogram_step(bits, width, n):
    inp, k = _inp(bits, n, bits * 7 + width + n)
    r = inp.shape[1]
    src = torch.from_numpy(inp.reshape(-1).copy()).cuda() if n else torch.empty(16, dtype=torch.uint8, device="cuda")
    w = min(width, bits)
    counts = torch.full((1 << w,), 0xFFFFFFFF, dtype=torch.int64, device="cuda").to(torch.int32)
    ws, nb = _ws(n, r, k)
    b.raduls_histogram(src, n, r, k, bits, width, counts, ws, nb)
    st, stats = b.raduls_check(ws, 0, r, True)
    assert st == b.OK, stats
    got = counts.cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal(got, oracle.histogram(inp, k, bits, width))


@pytest.mark.parametrize("bits,width", DIGITS)
@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097, 70001, 300007])
def test_partition_step(bits, width, n):
    inp, k = _inp(bits, n, bits * 13 + width + n)
    r = inp.shape[1]
    src = torch.from_numpy(inp.reshape(-1).copy()).cuda()
    dbuf, dst = guarded(n * r, 0x77)
    w = min(width, bits)
    offs = torch.zeros(1 << w, dtype=torch.int32, device="cuda")
    ws, nb = _ws(n, r, k)
    b.raduls_partition(src, dst, n, r, k, bits, width, offs, ws, nb)
    st, stats = b.raduls_check(ws, 0, r, True)
    assert st == b.OK, stats
    assert guards_intact(dbuf, n * r, 0x77)
    out = dst.cpu().numpy().reshape(n, r)
    assert np.array_equal(out, oracle.partition(inp, k, bits, width))
    exp_off = oracle.exclusive_scan(oracle.histogram(inp, k, bits, width))
    assert np.array_equal(offs.cpu().numpy().view(np.uint32).astype(np.uint64), exp_off)
    # the source is left untouched
    assert np.array_equal(src.cpu().numpy().reshape(n, r), inp)


@pytest.mark.parametrize("lookback", [0, 1])
def test_partition_full_tile_grid_uniform(lookback):
    """Several thousand tiles with ragged tail: the prefix across tiles, by
    carry scan and by look-back."""
    from gpu_helpers import tuned
    with tuned(lookback=lookback):
        _partition_full_tile_grid()


def _partition_full_tile_grid():
    n = (1 << 22) + 123
    inp = wl.uniform16(n)
    src = torch.from_numpy(inp.reshape(-1).copy()).cuda()
    dst = torch.empty_like(src)
    offs = torch.zeros(256, dtype=torch.int32, device="cuda")
    ws, nb = _ws(n, 16, 8)
    b.raduls_partition(src, dst, n, 16, 8, 64, 8, offs, ws, nb)
    st, stats = b.raduls_check(ws, 0, 16, True)
    assert st == b.OK, stats
    assert np.array_equal(dst.cpu().numpy().reshape(n, 16), oracle.partition(inp, 8, 64, 8))
