"""GPU parity: the HIP path through the C ABI against the CPU oracle.

The library's sort is stable, so its output must be byte-identical to the
oracle's stable sort (which also implies the weaker rule: equal key sequence
and equal record multiset per run of equal keys)."""

import numpy as np
import pytest
import torch

import oracle
from paper_1703_00687_amd import binding as b
from paper_1703_00687_amd import workloads as wl
from gpu_helpers import gpu_sort, tuned

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8), (8, 3), (16, 8), (16, 16), (16, 12), (24, 8), (24, 20), (32, 16), (40, 8),
          (48, 33), (56, 8), (64, 64), (64, 9)]


def _recs(seed, n, r, k, distinct=None):
    return wl.random_records(np.random.default_rng(seed), n, r, k, distinct)


def _assert_parity(out, inp, k):
    exp = oracle.sort(inp, k)
    if not np.array_equal(out, exp):
        assert oracle.parity(out, exp, k), "key sequence or run multisets differ"
        raise AssertionError("not byte-identical to the stable oracle")


@pytest.mark.parametrize("r,k", SHAPES)
def test_sizes_and_shapes(r, k):
    cap = b.raduls_mid_capacity(r, k)
    sizes = [0, 1, 2, 3, 31, 32, 33, 100, 1000, cap - 1, cap, cap + 1, 3 * cap + 7, 60000]
    for i, n in enumerate(sizes):
        for distinct in (None, 7):
            inp = _recs(1000 * r + 10 * k + i, n, r, k, distinct)
            out, _ = gpu_sort(inp, k)
            _assert_parity(out, inp, k)


@pytest.mark.parametrize("digit_bits,tiny_max,mid_max", [
    (8, 32, 0), (8, 8, 0), (8, 256, 0), (8, 32, 64), (8, 16, 300), (1, 32, 2000),
    (3, 24, 700), (5, 64, 0), (7, 1, 128), (4, 32, 40)])
@pytest.mark.parametrize("r,k", [(16, 8), (32, 16), (24, 13)])
def test_tuning_variants(digit_bits, tiny_max, mid_max, r, k):
    lookback = (digit_bits + tiny_max) % 2  # both scatter scans across the grid
    with tuned(digit_bits=digit_bits, tiny_max=tiny_max, mid_max=mid_max, lookback=lookback):
        for seed, distinct in ((1, None), (2, 300), (3, 3)):
            inp = _recs(seed + r + k + digit_bits, 40000, r, k, distinct)
            out, _ = gpu_sort(inp, k)
            _assert_parity(out, inp, k)


@pytest.mark.parametrize("tile_items", [1, 2, 3, 5])
@pytest.mark.parametrize("r,k,lookback", [(16, 8, 0), (32, 16, 1), (8, 8, 0), (24, 13, 0)])
def test_tile_sizes(tile_items, r, k, lookback):
    # smaller histogram / scatter tiles than the LDS staging holds (several
    # tiles per bin, bins that end inside a tile, both prefix schemes)
    with tuned(tile_items=tile_items, lookback=lookback):
        for seed, distinct in ((5, None), (6, 40)):
            inp = _recs(seed + r + tile_items, 300_000, r, k, distinct)
            out, _ = gpu_sort(inp, k)
            _assert_parity(out, inp, k)


@pytest.mark.parametrize("nontemporal,lookback", [(1, 0), (2, 0), (1, 1), (2, 1)])
def test_store_policies_and_scans(nontemporal, lookback):
    with tuned(nontemporal=nontemporal, lookback=lookback):
        inp = wl.uniform16(1 << 20)
        out, stats = gpu_sort(inp, 8)
        _assert_parity(out, inp, 8)
        assert stats["rounds"] >= 1 and stats["moved_records"] >= (1 << 20)


@pytest.mark.parametrize("name,n", [("uniform8", 1 << 20), ("uniform16", 1 << 22),
                                    ("zipf16", 1 << 21), ("deep32", 1 << 20),
                                    ("keys16", 1 << 21)])
def test_workloads_reduced(name, n):
    inp, k = wl.make(name, n)
    out, _ = gpu_sort(inp, k)
    _assert_parity(out, inp, k)


@pytest.mark.parametrize("r,k", [(8, 8), (16, 8), (16, 16), (24, 8), (24, 16), (32, 8),
                                 (32, 16), (48, 8), (48, 16), (64, 8), (64, 16)])
def test_record_size_sweep_reduced(r, k):
    """The record shapes of the record-size sweep, element by element against
    the oracle, at a size that still takes two radix rounds."""
    inp = wl.sweep_records(1 << 19, r, k)
    out, stats = gpu_sort(inp, k)
    _assert_parity(out, inp, k)
    assert stats["rounds"] >= 1


@pytest.mark.parametrize("r,k", [(16, 8), (8, 2), (16, 16), (24, 13), (32, 16)])
def test_pair_counts_on_and_off(r, k):
    """Inputs large enough that the top level counts (top, second) digit
    pairs and the second round takes its histograms from them; the result
    must be the same with that path switched off."""
    n = 1 << 22
    inp = _recs(77 + r + k, n, r, k)
    for pair, used in ((0, 1), (2, 0)):
        with tuned(pair_hist=pair):
            out, stats = gpu_sort(inp, k)
        _assert_parity(out, inp, k)
        assert stats["pair_rounds"] == used, stats


def test_pair_counts_declined_for_uneven_bins():
    """Skewed keys make the second round's bins uneven (one holds a fifth of
    the records): the pair counts are not used, and the sort is unchanged."""
    n = 1 << 22
    inp = _recs(5, n, 16, 8)
    heavy = np.random.default_rng(6).random(n) < 0.2
    inp[heavy, 7] = 0x5A
    out, stats = gpu_sort(inp, 8)
    _assert_parity(out, inp, 8)
    assert stats["pair_rounds"] == 0, stats


def test_pair_counts_declined_for_constant_second_digit():
    """One top digit whose records all share the second key byte: that bin
    would have to jump digits, so the pair counts are not used."""
    n = 1 << 22
    inp = _recs(8, n, 16, 8)
    sel = inp[:, 7] == 0x33
    inp[sel, 6] = 0x44
    out, stats = gpu_sort(inp, 8)
    _assert_parity(out, inp, 8)
    assert stats["pair_rounds"] == 0, stats


def _adversarial(r, k, n, seed):
    rng = np.random.default_rng(seed)
    base = wl.random_records(rng, n, r, k)
    cases = {"random": base}
    eq = base.copy()
    eq[:, :k] = base[0, :k]
    cases["all_equal"] = eq
    two = base.copy()
    two[:, :k] = np.where(rng.integers(0, 2, size=(n, 1)) == 1, base[0, :k], base[1, :k])
    cases["two_values"] = two
    cases["sorted"] = oracle.sort(base, k)
    cases["reverse"] = cases["sorted"][::-1].copy()
    last = base.copy()
    last[:, 1:k] = 0x5A
    cases["last_byte_only"] = last
    low = base.copy()
    low[:, :k] = base[0, :k]
    low[:, 0] = rng.integers(0, 4, size=n, dtype=np.uint8)
    cases["low_byte_only"] = low
    one_off = eq.copy()
    one_off[n // 2, k - 1] ^= 0x80
    cases["one_different"] = one_off
    return cases


@pytest.mark.parametrize("r,k", [(16, 8), (32, 16), (24, 13), (8, 8)])
def test_adversarial_keys(r, k):
    for name, inp in _adversarial(r, k, 150000, r + k).items():
        out, _ = gpu_sort(inp, k)
        try:
            _assert_parity(out, inp, k)
        except AssertionError as e:
            raise AssertionError(f"{name}: {e}")


def test_deterministic_reruns():
    inp = wl.zipf16(1 << 19)
    a, _ = gpu_sort(inp, 8)
    for _ in range(2):
        c, _ = gpu_sort(inp, 8)
        assert np.array_equal(a, c)


@pytest.mark.parametrize("block", [1, 63, 64, 65, 200])
@pytest.mark.parametrize("n", [128, 1000, 5000])
def test_runs_of_equal_keys_across_waves(block, n):
    """Runs of one key that line up with (or straddle) the 64-lane waves of
    the LDS sorter: every wave may see a single key while the job does not."""
    r, k = 16, 8
    rng = np.random.default_rng(block * 7919 + n)
    inp = wl.random_records(rng, n, r, k)
    run_keys = rng.integers(0, 256, size=((n + block - 1) // block, k), dtype=np.uint8)
    inp[:, :k] = np.repeat(run_keys, block, axis=0)[:n]
    out, _ = gpu_sort(inp, k)
    _assert_parity(out, inp, k)


@pytest.mark.parametrize("r,k", [(8, 8), (16, 8), (24, 13), (32, 16), (64, 9)])
def test_finished_runs_in_tmp_copied_in_pieces(r, k):
    """Runs of one key that end in tmp after the top round (two keys that
    differ in the top byte, each with more records than one LDS job) go back
    to recs as copy jobs on the LDS sorter's list, in pieces of at most
    mid_max records: sizes at and around the piece boundaries."""
    cap = b.raduls_server_max_records(r, k)  # mid_max of this layout
    rng = np.random.default_rng(r * 31 + k)
    for ca, cb in ((cap + 1, cap + 1), (2 * cap, 2 * cap + 1), (3 * cap + 7, cap + 2)):
        n = ca + cb
        inp = wl.random_records(rng, n, r, k)
        lo = np.zeros(k, np.uint8)
        hi = np.zeros(k, np.uint8)
        lo[k - 1], hi[k - 1] = 0x10, 0xE0  # (the top byte is the key's last)
        which = rng.permutation(np.r_[np.zeros(ca, bool), np.ones(cb, bool)])
        inp[:, :k] = np.where(which[:, None], hi, lo)
        out, stats = gpu_sort(inp, k)
        _assert_parity(out, inp, k)
        pieces = -(-ca // cap) + -(-cb // cap)
        assert stats["copy_jobs"] == pieces, (ca, cb, stats)


@pytest.mark.parametrize("r,k", [(8, 5), (24, 13), (40, 9), (16, 16)])
@pytest.mark.parametrize("rare", [0, 3])
def test_narrow_keys_in_wide_fields(r, k, rare):
    """Keys whose bytes above the lowest three are one constant, non-zero
    pattern (the top of the key field is constant but not zero), at a size
    where the root's first digit is guessed from a sample of the records;
    `rare` records differ in the key's top byte, which the sample most
    likely misses.  Byte-identical to the stable oracle either way."""
    n = 1 << 21
    if n <= 256 * b.raduls_server_max_records(r, k):
        n = 512 * b.raduls_server_max_records(r, k)
    rng = np.random.default_rng(r * 100 + k + rare)
    inp = wl.random_records(rng, n, r, k)
    inp[:, 3:k] = 0x5A
    if rare:
        inp[rng.choice(n, size=rare, replace=False), k - 1] = 0x7E
    out, stats = gpu_sort(inp, k)
    _assert_parity(out, inp, k)
