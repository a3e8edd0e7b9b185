"""GPU: the recursion's bins after round l, pinned against the oracle.

After each radix phase the array is split into bins that are processed
independently (Sec. 1); bins still larger than the LDS capacity get another
global pass (Sec. 3.1-3.2).  raduls_inspect_rounds runs only the first l
global rounds and returns the large bins they left.  Each one must be a
maximal run of the oracle's sorted output whose keys agree on every bit from
the bin's `bits` up, larger than mid_max, and its records (on the side the
entry names) must be exactly those of that run in input order (every pass is
a stable partition; the payload holds the input index).  A bin that is one
side of an equality split (a key range inside such a run, flag bit 1) must
pass the same checks except maximality.  With uniform keys and a fixed digit
width no digit is skipped, so the list must also be exactly the oracle's
bins at level l (oracle.bins_at_level) that exceed mid_max."""

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import tuned
from paper_1703_00687_amd import binding as b
from paper_1703_00687_amd import workloads as wl

pytestmark = pytest.mark.gpu


def masked_keys(recs: np.ndarray, key_bytes: int, bits: int) -> np.ndarray:
    """The key bytes with key bits [0, bits) cleared."""
    k = np.ascontiguousarray(recs[:, :key_bytes]).copy()
    full = bits // 8
    k[:, :min(full, key_bytes)] = 0
    if bits % 8 and full < key_bytes:
        k[:, full] &= np.uint8(0xFF ^ ((1 << (bits % 8)) - 1))
    return k


def check_round(host, key_bytes, idx_word, rounds, exact_level_width=None):
    n, R = host.shape
    mid_max = b.raduls_get_tuning()["mid_max"] or b.raduls_mid_capacity(R, key_bytes)
    mid_max = min(mid_max, b.raduls_mid_capacity(R, key_bytes))
    recs = torch.from_numpy(host.reshape(-1).copy()).cuda()
    tmp = torch.empty(b.raduls_tmp_bytes(n, R, key_bytes), dtype=torch.uint8, device="cuda")
    bins = b.raduls_inspect_rounds(recs, tmp, n, R, key_bytes, rounds)
    sides = [recs.cpu().numpy().reshape(n, R), tmp[:n * R].cpu().numpy().reshape(n, R)]
    srt = oracle.sort(host, key_bytes)
    idx = srt.view("<u8")[:, idx_word]
    covered = np.zeros(n, dtype=bool)
    for start, size, bits, side, flags in bins:
        assert size > mid_max and start + size <= n and side in (0, 1)
        assert 0 < bits <= 8 * key_bytes
        assert not covered[start:start + size].any(), "bins overlap"
        covered[start:start + size] = True
        mk = masked_keys(srt[max(start - 1, 0):start + size + 1], key_bytes, bits)
        body = mk[(1 if start > 0 else 0):][:size]
        assert (body == body[0]).all(), "a bin's records differ above its bits"
        if not flags & 2:
            if start > 0:
                assert not np.array_equal(mk[0], body[0]), "bin is not maximal (left)"
            if start + size < n:
                assert not np.array_equal(mk[-1], body[0]), "bin is not maximal (right)"
        expect = srt[start:start + size][np.argsort(idx[start:start + size], kind="stable")]
        assert np.array_equal(sides[side][start:start + size], expect), \
            "a bin's records are not the stable partition"
    if exact_level_width is not None:
        starts, sizes = oracle.bins_at_level(srt, key_bytes, exact_level_width, rounds)
        want = sorted((int(s), int(z)) for s, z in zip(starts, sizes) if z > mid_max)
        got = sorted((s, z) for s, z, _, _, _ in bins)
        assert got == want
        # (no equality split; bits 2-5 may set a narrower digit for the
        # bin's next split, which does not change the bin itself)
        assert all(bt == 8 * key_bytes - exact_level_width * rounds and (fl & 3) == 0
                   for _, _, bt, _, fl in bins)
    return bins


@pytest.mark.parametrize("rounds", [1, 2, 3])
def test_bins_uniform_four_bit_digits(rounds):
    host = wl.uniform16(1 << 20, seed=41)
    with tuned(digit_bits=4, mid_max=64):
        bins = check_round(host, 8, 1, rounds, exact_level_width=4)
    assert len(bins) == 16 ** rounds


@pytest.mark.parametrize("rounds", [1, 2, 3])
def test_bins_skewed_keys(rounds):
    host = wl.zipf16(1 << 20, seed=42, values=1 << 12)
    check_round(host, 8, 1, rounds)


@pytest.mark.parametrize("rounds", [1, 2])
def test_bins_deep_keys_skip_constant_digits(rounds):
    host = wl.deep32(1 << 20, seed=43)
    bins = check_round(host, 16, 2, rounds)
    if rounds == 1:
        # the top 44 key bits are zero for every record: the first round's
        # children already lie below them
        assert bins and all(bt <= 84 for _, _, bt, _, _ in bins)


def test_bins_small_input_runs_no_round():
    host = wl.uniform16(1000, seed=44)
    recs = torch.from_numpy(host.reshape(-1).copy()).cuda()
    tmp = torch.empty(b.raduls_tmp_bytes(1000, 16, 8), dtype=torch.uint8, device="cuda")
    assert b.raduls_inspect_rounds(recs, tmp, 1000, 16, 8, 1) == []


def test_equality_splits_of_dominated_bins():
    """A few keys dominate: bins they fill are split on them (stats count the
    splits), the bins left after such a round pass the checks above, and the
    whole sort equals the oracle's."""
    host = wl.zipf16(1 << 22, seed=45, values=1 << 12)
    marked = False
    for rounds in (1, 2, 3):
        bins = check_round(host, 8, 1, rounds)
        marked = marked or any(fl & 1 for *_, fl in bins)
    assert marked, "no bin was marked for a split on a dominant key"
    n = host.shape[0]
    recs = torch.from_numpy(host.reshape(-1).copy()).cuda()
    tmp = torch.empty(b.raduls_tmp_bytes(n, 16, 8), dtype=torch.uint8, device="cuda")
    b.raduls_sort(recs, tmp, n, 16, 8)
    st, stats = b.raduls_check(tmp, n, 16, False)
    assert st == b.OK and stats["eq_bins"] > 0, stats
    assert np.array_equal(recs.cpu().numpy().reshape(n, 16), oracle.sort(host, 8))


def test_narrow_digit_for_bins_of_a_few_jobs():
    """A bin of a few LDS jobs' worth of records is marked to be split on
    just enough bits for children of one job each (flag bits 2-5): 2^20
    uniform keys with mid_max 1024 leave 256 bins of ~4096 records after the
    top round, split next on 3 bits (children of ~512 <= 0.9 * 1024), not on
    a byte; the whole sort still equals the oracle."""
    host = wl.uniform16(1 << 20, seed=46)
    with tuned(mid_max=1024, pair_hist=2):
        bins = check_round(host, 8, 1, 1)
        assert len(bins) == 256 and all((fl >> 2) & 15 == 3 for _, _, _, _, fl in bins)
        n = host.shape[0]
        recs = torch.from_numpy(host.reshape(-1).copy()).cuda()
        tmp = torch.empty(b.raduls_tmp_bytes(n, 16, 8), dtype=torch.uint8, device="cuda")
        b.raduls_sort(recs, tmp, n, 16, 8)
        st, stats = b.raduls_check(tmp, n, 16, False)
        assert st == b.OK, stats
        assert np.array_equal(recs.cpu().numpy().reshape(n, 16), oracle.sort(host, 8))


def test_root_top_guessed_from_a_sample():
    """Deep keys (the top 44 key bits zero) at a size where the root's first
    digit is guessed from sampled records: round 0 already splits below the
    constant bits (no round that only finds them constant)."""
    host = wl.deep32(1 << 21, seed=44)
    bins = check_round(host, 16, 2, 1)
    assert bins and all(bt <= 76 for _, _, bt, _, _ in bins)
    bins = check_round(host, 16, 2, 2)


@pytest.mark.parametrize("hi_count", [1, 3, 1000])
def test_root_top_guess_missed(hi_count):
    """Keys below 2^40 except a few records with bit 62 set, which the
    sample (most likely) misses: round 0's histogram sees the true spread,
    moves nothing, and the root is split from its true top next round; the
    sort is still the stable sort."""
    n = 1 << 21
    rng = np.random.default_rng(45 + hi_count)
    host = wl.random_records(rng, n, 16, 8)
    keys = host[:, :8].copy().view("<u8").ravel()
    keys &= np.uint64((1 << 40) - 1)
    hit = rng.choice(n, size=hi_count, replace=False)
    keys[hit] |= np.uint64(1 << 62)
    host[:, :8] = keys.view(np.uint8).reshape(n, 8)
    host[:, 8:] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    bins = check_round(host, 8, 1, 1)
    assert bins
    recs = torch.from_numpy(host.reshape(-1).copy()).cuda()
    tmp = torch.empty(b.raduls_tmp_bytes(n, 16, 8), dtype=torch.uint8, device="cuda")
    b.raduls_sort(recs, tmp, n, 16, 8)
    st, stats = b.raduls_check(tmp, n, 16, False)
    assert st == b.OK, stats
    assert np.array_equal(recs.cpu().numpy().reshape(n, 16), oracle.sort(host, 8))


@pytest.mark.parametrize("rare_high", [0, 2])
def test_root_top_guess_two_word_keys(rare_high):
    """16-byte keys below 2^40 (the guess falls in the low key word, three
    words of zeros above it), optionally with a couple of records that set a
    bit of the high word, which the sample most likely misses."""
    n = 1 << 21
    rng = np.random.default_rng(47 + rare_high)
    host = wl.random_records(rng, n, 32, 16)
    w = host.view("<u8").reshape(n, 4)
    w[:, 0] &= np.uint64((1 << 40) - 1)
    w[:, 1] = 0
    w[:, 2] = np.arange(n, dtype="<u8")
    if rare_high:
        w[rng.choice(n, size=rare_high, replace=False), 1] = np.uint64(1 << 20)
    host = w.view(np.uint8).reshape(n, 32)
    bins = check_round(host, 16, 2, 1)
    if not rare_high:
        assert bins and all(bt <= 32 for _, _, bt, _, _ in bins)
    recs = torch.from_numpy(host.reshape(-1).copy()).cuda()
    tmp = torch.empty(b.raduls_tmp_bytes(n, 32, 16), dtype=torch.uint8, device="cuda")
    b.raduls_sort(recs, tmp, n, 32, 16)
    st, stats = b.raduls_check(tmp, n, 32, False)
    assert st == b.OK, stats
    assert np.array_equal(recs.cpu().numpy().reshape(n, 32), oracle.sort(host, 16))
