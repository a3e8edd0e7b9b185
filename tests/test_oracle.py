"""Pins for the CPU oracle: each check compares it with something other than
itself (Python's own sort on Python-int keys, numpy's lexsort, brute force
over permutations, closed forms, a hand-derived fixture)."""

import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_1703_00687_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = [(8, 8), (8, 3), (16, 8), (16, 16), (16, 12), (24, 8), (24, 20), (32, 16),
          (40, 8), (64, 64), (64, 9)]


def int_key(rec, k):
    return int.from_bytes(bytes(rec[:k]), "little")


def python_sorted(recs, k):
    order = sorted(range(recs.shape[0]), key=lambda i: int_key(recs[i], k))
    return recs[order]


def rand_recs(seed, n, r, k, distinct=None):
    rng = np.random.default_rng(seed)
    return wl.random_records(rng, n, r, k, distinct)


# ---------------------------------------------------------------- full sort

@pytest.mark.parametrize("r,k", SHAPES)
def test_sort_equals_python_sorted(r, k):
    for seed, distinct in ((1, None), (2, 5), (3, 40)):
        recs = rand_recs(seed * 100 + r + k, 700, r, k, distinct)
        assert np.array_equal(oracle.sort(recs, k), python_sorted(recs, k))


@pytest.mark.parametrize("r,k", SHAPES)
@pytest.mark.parametrize("threads", [1, 2, 4, 0])
def test_parallel_sort_equals_python_sorted(r, k, threads):
    # the CPU-baseline variant (several threads) against Python's own stable
    # sort; large enough that every thread gets a share of the merge
    for seed, distinct in ((11, None), (12, 3), (13, 200)):
        recs = rand_recs(seed * 100 + r + k, 5000, r, k, distinct)
        out, used = oracle.sort_parallel(recs, k, threads)
        assert used >= 1 and (threads == 0 or used == threads)
        assert np.array_equal(out, python_sorted(recs, k))


@pytest.mark.parametrize("r,k", SHAPES)
def test_sort_equals_numpy_lexsort(r, k):
    recs = rand_recs(r * 7 + k, 20000, r, k, distinct=3000)
    order = np.lexsort([recs[:, j] for j in range(k)])  # last column is primary
    assert np.array_equal(oracle.sort(recs, k), recs[order])


def test_sort_bruteforce_tiny():
    rng = np.random.default_rng(5)
    for n in range(0, 7):
        for trial in range(6):
            recs = wl.random_records(rng, n, 8, 2, distinct_keys=3)
            keys = [int_key(recs[i], 2) for i in range(n)]
            winners = []
            for p in itertools.permutations(range(n)):
                ok = all(keys[p[i]] < keys[p[i + 1]] or
                         (keys[p[i]] == keys[p[i + 1]] and p[i] < p[i + 1])
                         for i in range(n - 1))
                if ok:
                    winners.append(p)
            assert len(winners) == 1
            assert np.array_equal(oracle.sort(recs, 2), recs[list(winners[0])])


def test_sort_closed_form_permutation():
    rng = np.random.default_rng(9)
    n = 50000
    keys = rng.permutation(n).astype(np.uint64)
    recs = wl.records_from_words([keys, np.arange(n, dtype=np.uint64)])
    out = oracle.sort(recs, 8).view("<u8").reshape(n, 2)
    assert np.array_equal(out[:, 0], np.arange(n, dtype=np.uint64))
    # record with key v came from input position argsort(keys)[v]
    assert np.array_equal(out[:, 1], np.argsort(keys).astype(np.uint64))


def _read_golden(path):
    cases = []
    cur = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("case"):
                _, name, r, k = line.split()
                cur = dict(name=name, r=int(r), k=int(k), recs=[], expect=None)
                cases.append(cur)
            elif line.startswith("expect"):
                cur["expect"] = [int(x) for x in line.split()[1:]]
            else:
                cur["recs"].append(bytes.fromhex(line))
    return cases


def test_golden_key_byte_order():
    cases = _read_golden(os.path.join(GOLDEN, "key_byte_order.txt"))
    assert len(cases) == 3
    for c in cases:
        recs = np.frombuffer(b"".join(c["recs"]), dtype=np.uint8).reshape(-1, c["r"])
        out = oracle.sort(recs, c["k"])
        assert np.array_equal(out, recs[c["expect"]]), c["name"]
        assert np.array_equal(oracle.msd_sort(recs, c["k"], 8, 1), recs[c["expect"]])


def test_payload_never_affects_order():
    rng = np.random.default_rng(11)
    n = 3000
    recs = wl.random_records(rng, n, 24, 5, distinct_keys=50)
    recs[:, 5:13] = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)
    recs2 = recs.copy()
    recs2[:, 13:] = rng.integers(0, 256, size=recs2[:, 13:].shape, dtype=np.uint8)
    a = oracle.sort(recs, 5)
    b = oracle.sort(recs2, 5)
    # the input position carried in bytes 5..12 comes out in the same order
    assert np.array_equal(a[:, :13], b[:, :13])


def test_validate_rules():
    assert oracle.validate(10, 16, 8) == oracle.OK
    assert oracle.validate(10, 12, 8) == oracle.E_UNSUPPORTED
    assert oracle.validate(10, 72, 8) == oracle.E_UNSUPPORTED
    assert oracle.validate(10, 0, 0) == oracle.E_UNSUPPORTED
    assert oracle.validate(10, 16, 0) == oracle.E_INVALID
    assert oracle.validate(10, 16, 17) == oracle.E_INVALID
    assert oracle.validate(1 << 32, 16, 8) == oracle.E_UNSUPPORTED
    assert oracle.validate(0, 8, 8) == oracle.OK


# ------------------------------------------------------------- hot-path steps

DIGITS = [(64, 8), (8, 8), (61, 8), (5, 8), (128, 8), (100, 11), (3, 3), (77, 1), (16, 16)]


def _py_digit(rec, k, bits, width):
    w = min(width, bits)
    return (int_key(rec, k) >> (bits - w)) & ((1 << w) - 1)


@pytest.mark.parametrize("bits,width", DIGITS)
def test_histogram_equals_bincount(bits, width):
    r, k = (16, 16) if bits > 64 else (16, 8)
    recs = rand_recs(bits * 31 + width, 3000, r, k, distinct=200)
    h = oracle.histogram(recs, k, bits, width)
    d = np.array([_py_digit(recs[i], k, bits, width) for i in range(recs.shape[0])])
    assert h.size == 1 << min(width, bits)
    assert np.array_equal(h, np.bincount(d, minlength=h.size).astype(np.uint64))
    assert int(h.sum()) == recs.shape[0]


def test_exclusive_scan_closed_form():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 1000, size=256).astype(np.uint64)
    off = oracle.exclusive_scan(c, base=77)
    for b in range(256):
        assert int(off[b]) == 77 + int(sum(int(x) for x in c[:b]))
    assert int(off[-1] + c[-1]) == 77 + int(c.sum())
    assert oracle.exclusive_scan(np.zeros(0, np.uint64)).size == 0


@pytest.mark.parametrize("bits,width", DIGITS)
def test_partition_is_stable_digit_sort(bits, width):
    r, k = (16, 16) if bits > 64 else (24, 8)
    recs = rand_recs(bits + 1000 * width, 4000, r, k, distinct=300)
    d = np.array([_py_digit(recs[i], k, bits, width) for i in range(recs.shape[0])])
    expect = recs[np.argsort(d, kind="stable")]
    assert np.array_equal(oracle.partition(recs, k, bits, width), expect)


def test_partition_bruteforce_tiny():
    rng = np.random.default_rng(21)
    for n in range(1, 7):
        recs = wl.random_records(rng, n, 8, 1, distinct_keys=3)
        recs[:, 0] &= 0x3  # two-bit keys
        out = oracle.partition(recs, 1, 2, 2)
        want = []
        for v in range(4):  # bucket order, input order inside a bucket
            want += [i for i in range(n) if recs[i, 0] == v]
        assert np.array_equal(out, recs[want])


def test_enum_sort_all_multiset_permutations():
    for n in range(1, 8):
        base = [i % 3 for i in range(n)]
        seen = set()
        for p in itertools.permutations(base):
            if p in seen:
                continue
            seen.add(p)
            recs = np.zeros((n, 8), dtype=np.uint8)
            recs[:, 0] = p
            recs[:, 1] = np.arange(n)  # data byte records the input position
            out = oracle.enum_sort(recs, 1)
            assert np.array_equal(out, python_sorted(recs, 1))


@pytest.mark.parametrize("r,k", [(8, 8), (16, 8), (32, 16), (24, 20)])
def test_enum_sort_random_duplicates(r, k):
    recs = rand_recs(r + k, 300, r, k, distinct=20)
    assert np.array_equal(oracle.enum_sort(recs, k), python_sorted(recs, k))


def _adversarial(r, k, n, seed):
    rng = np.random.default_rng(seed)
    out = {}
    base = wl.random_records(rng, n, r, k)
    out["random"] = base
    eq = base.copy()
    eq[:, :k] = base[0, :k]
    out["all_equal"] = eq
    two = base.copy()
    two[:, :k] = np.where(rng.integers(0, 2, size=(n, 1)) == 1, base[0, :k], base[1, :k])
    out["two_values"] = two
    out["sorted"] = python_sorted(base, k)
    out["reverse"] = out["sorted"][::-1].copy()
    last = base.copy()
    last[:, 1:k] = 0x5A
    out["last_byte_only"] = last
    low = base.copy()
    low[:, :k] = base[0, :k]
    low[:, 0] = rng.integers(0, 4, size=n, dtype=np.uint8)
    out["low_byte_only"] = low
    return out


@pytest.mark.parametrize("r,k", [(8, 8), (16, 8), (16, 16), (24, 13), (32, 16)])
@pytest.mark.parametrize("width,tiny", [(8, 1), (8, 32), (1, 4), (3, 16), (11, 64), (8, 100000)])
def test_msd_sort_equals_definition(r, k, width, tiny):
    n = 600 if tiny >= 100000 else 2500
    for name, recs in _adversarial(r, k, n, r * 13 + k).items():
        assert np.array_equal(oracle.msd_sort(recs, k, width, tiny), oracle.sort(recs, k)), name


@pytest.mark.parametrize("width,levels", [(8, 1), (8, 2), (8, 3), (5, 2), (11, 1), (8, 9)])
def test_bins_at_level_are_prefix_runs(width, levels):
    r, k = 16, 8
    recs = rand_recs(width * 10 + levels, 5000, r, k, distinct=800)
    recs[:, 7] &= 0x03  # few top-byte values so bins are large
    s = oracle.sort(recs, k)
    starts, sizes = oracle.bins_at_level(s, k, width, levels)
    top = min(8 * k, width * levels)
    prefix = [int_key(s[i], k) >> (8 * k - top) for i in range(s.shape[0])]
    vals, counts = np.unique(np.array(prefix, dtype=object).astype(np.uint64), return_counts=True)
    assert np.array_equal(sizes, counts.astype(np.uint64))
    assert int(starts[0]) == 0
    assert np.array_equal(starts[1:], np.cumsum(sizes)[:-1])


# ---------------------------------------------------------------- checkers

def test_checkers_catch_planted_faults():
    recs = rand_recs(77, 5000, 16, 8, distinct=500)
    recs[:, 8:] = np.arange(5000, dtype="<u8").view(np.uint8).reshape(5000, 8)
    good = oracle.sort(recs, 8)
    assert oracle.check_sorted(good, 8) and oracle.first_unsorted(good, 8) == 5000
    assert oracle.parity(good, good, 8)
    # a swapped pair of distinct keys
    bad = good.copy()
    i = next(i for i in range(100, 5000) if not np.array_equal(good[i, :8], good[i + 1, :8]))
    bad[[i, i + 1]] = bad[[i + 1, i]]
    assert not oracle.check_sorted(bad, 8) and oracle.first_unsorted(bad, 8) == i
    assert not oracle.parity(bad, good, 8)
    # a duplicated record inside an equal-key run (keys stay sorted)
    j = next(j for j in range(5000 - 1) if np.array_equal(good[j, :8], good[j + 1, :8]))
    dup = good.copy()
    dup[j + 1] = dup[j]
    assert oracle.check_sorted(dup, 8)
    assert not oracle.parity(dup, good, 8)
    assert not oracle.same_multiset(dup, good)
    # a corrupted payload byte
    cor = good.copy()
    cor[j, 12] ^= 0xFF
    assert not oracle.parity(cor, good, 8)
    # reordering inside an equal-key run is accepted by the parity rule
    perm = good.copy()
    perm[[j, j + 1]] = perm[[j + 1, j]]
    assert oracle.parity(perm, good, 8)


# ---------------------------------------------------------------- generators

def test_splitmix64_published_values():
    # First outputs of SplitMix64 started at state 0 (Vigna's splitmix64.c).
    z = wl.splitmix64(0, 0, 3)
    assert [int(x) for x in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    st = 0x1234567890ABCDEF
    ref = [wl.mix64_int(st + (i + 1) * wl.GAMMA) for i in range(1000)]
    assert [int(x) for x in wl.splitmix64(st, 0, 1000)] == ref


def test_generators_deterministic_and_shaped():
    a = wl.uniform16(1 << 16)
    b = wl.uniform16(1 << 16)
    assert np.array_equal(a, b) and a.shape == (1 << 16, 16)
    w = a.view("<u8").reshape(-1, 2)
    assert np.array_equal(w[:, 1], np.arange(1 << 16, dtype=np.uint64))
    # chi-square on the top key byte (255 degrees of freedom)
    top = (w[:, 0] >> np.uint64(56)).astype(np.int64)
    obs = np.bincount(top, minlength=256)
    exp = w.shape[0] / 256
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)
    d = wl.deep32(1 << 14).view("<u8").reshape(-1, 4)
    assert int(d[:, 1].max()) < (1 << 20)
    assert np.array_equal(d[:, 2], np.arange(1 << 14, dtype=np.uint64))


def test_zipf_workload_frequencies():
    from scipy.special import zeta
    n = 1 << 20
    recs = wl.zipf16(n)
    keys = recs.view("<u8").reshape(n, 2)[:, 0]
    d, special = wl.zipf_dictionary(3, wl.ZIPF_VALUES)
    # override fraction 5% within 4 sigma
    p = wl.ZIPF_OVERRIDE
    frac = np.count_nonzero(keys == np.uint64(special))
    assert abs(frac - n * p) < 4 * math.sqrt(n * p * (1 - p))
    # rank-1 share of the rest = 1 / H(2^24, 1.1), H via Hurwitz zeta
    h = zeta(wl.ZIPF_S, 1) - zeta(wl.ZIPF_S, wl.ZIPF_VALUES + 1)
    p1 = 1.0 / h
    rest = n - frac
    top = np.count_nonzero(keys == d[0])
    assert abs(top - rest * p1) < 4 * math.sqrt(rest * p1 * (1 - p1))
    assert abs(p1 - 0.115) < 0.01


def test_batch_sizes_log_uniform():
    s = wl.batch_sizes(65536)
    assert s.min() >= 1 and s.max() <= 1 << 20
    # log(size+1) ~ uniform on [0, ln(2^20+1)]: mean close to half the range
    lg = np.log(s.astype(np.float64))
    assert abs(lg.mean() - 0.5 * math.log(2 ** 20 + 1)) < 0.1


def test_device_generator_matches_host_generator():
    import torch
    st = wl.stream_seed(2, 0)
    a = wl.splitmix64(st, 12345, 5000)
    b = wl.splitmix64_torch(st, 12345, 5000, device="cpu").numpy().view(np.uint64)
    assert np.array_equal(a, b)
    assert np.array_equal(wl.uniform16_torch(3000, device="cpu", chunk=1000).numpy(), wl.uniform16(3000))
    assert np.array_equal(wl.batch_array_torch(7, 999, 31337, device="cpu").numpy(),
                          wl.batch_array(7, 999, 31337))
