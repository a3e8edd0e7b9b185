"""Seeded synthetic inputs shaped like the paper's sorting workloads.

This module only draws numbers; it holds none of the sorting method's
arithmetic.  The CPU oracle, the parity tests and the benchmark all take
their inputs from here.

Every value is a pure function of (workload seed, stream tag, index), built on
SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the i-th output of a stream started at state s is
mix(s + (i + 1) * GAMMA).

Workloads (record = key bytes first, little-endian, then payload):

* ``uniform8``   2^20 records of 8 B, the key only, uniform over 64 bits.
* ``uniform16``  2^28 records of 16 B: uint64 key uniform, uint64 payload = index
                 (the paper's 16 B records with 8 B key and 8 B data, Sec. 4.2).
* ``zipf16``     2^28 records of 16 B: key = D[rank], rank ~ Zipf(s=1.1) over
                 2^24 distinct random uint64 values, and 5% of records replaced by
                 one extra key; payload = index (the paper's Zipf runs, Sec. 4.2,
                 whose parameters it does not give).
* ``deep32``     2^27 records of 32 B: 16 B key (low word uniform, high word
                 uniform over the values 0 .. 2^20-1) + 16 B payload (index and
                 a random word).
* ``batch16``    many arrays of 16 B records, sizes log-uniform in
                 [1, 2^max_log2]; key uniform, payload = index in its array.
* ``keys16``     2^28 records of 16 B that are all key (uniform over 128 bits,
                 no payload): the shape of the 16 B k-mer records the paper's
                 application sorts (Sec. 4.2), synthetic.
* ``sweep_records(n, R, K)``  the record-size sweep (Sec. 4.2, records of
                 various sizes): K key bytes uniform, then a payload word
                 holding the index when R > K, then random words.
"""

from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_G = np.uint64(GAMMA)


def mix64_int(z: int) -> int:
    """SplitMix64 output function on a Python int (reference form)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def stream_seed(seed: int, tag: int) -> int:
    """Start state of stream `tag` of workload seed `seed`."""
    return mix64_int((seed * GAMMA + tag) & MASK64)


def splitmix64(state: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the stream that begins at `state`."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(state & MASK64) + i * _G
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _chunked(state: int, count: int, out: np.ndarray, chunk: int = 1 << 24) -> None:
    for s in range(0, count, chunk):
        c = min(chunk, count - s)
        out[s:s + c] = splitmix64(state, s, c)


def uniform_keys(seed: int, n: int, tag: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _chunked(stream_seed(seed, tag), n, out)
    return out


def unit_doubles(seed: int, tag: int, start: int, count: int) -> np.ndarray:
    """53-bit uniform doubles in [0, 1)."""
    z = splitmix64(stream_seed(seed, tag), start, count)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def records_from_words(words: list[np.ndarray]) -> np.ndarray:
    """Pack uint64 columns (word 0 first) into an [n, 8*len(words)] uint8 array."""
    n = words[0].shape[0]
    rec = np.empty((n, len(words)), dtype="<u8")
    for j, w in enumerate(words):
        rec[:, j] = w
    return rec.view(np.uint8).reshape(n, 8 * len(words))


# --------------------------------------------------------------------------
# Workloads


def uniform8(n: int = 1 << 20, seed: int = 1) -> np.ndarray:
    return records_from_words([uniform_keys(seed, n)])


def uniform16(n: int = 1 << 28, seed: int = 2) -> np.ndarray:
    out = np.empty((n, 2), dtype="<u8")
    chunk = 1 << 24
    st = stream_seed(seed, 0)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        out[s:s + c, 0] = splitmix64(st, s, c)
        out[s:s + c, 1] = np.arange(s, s + c, dtype=np.uint64)
    return out.view(np.uint8).reshape(n, 16)


ZIPF_S = 1.1
ZIPF_VALUES = 1 << 24
ZIPF_OVERRIDE = 0.05


def zipf_cdf(values: int = ZIPF_VALUES, s: float = ZIPF_S) -> np.ndarray:
    """CDF of Zipf(s) over ranks 0 .. values-1 with P(r) proportional to (r+1)^-s."""
    p = np.arange(1, values + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    return cdf


def zipf_dictionary(seed: int, values: int) -> tuple[np.ndarray, int]:
    """`values` distinct random uint64 keys and one extra key not among them."""
    d = uniform_keys(seed, values, tag=10)
    extra_tag = 11
    while True:
        u, first = np.unique(d, return_index=True)
        if u.size == values:
            break
        dup = np.ones(values, dtype=bool)
        dup[first] = False
        idx = np.nonzero(dup)[0]
        d[idx] = splitmix64(stream_seed(seed, extra_tag), 0, idx.size)
        extra_tag += 1
    special_start = 0
    while True:
        special = int(splitmix64(stream_seed(seed, 12), special_start, 1)[0])
        if not np.any(d == np.uint64(special)):
            return d, special
        special_start += 1


def zipf16(n: int = 1 << 28, seed: int = 3, values: int = ZIPF_VALUES,
           s: float = ZIPF_S, override: float = ZIPF_OVERRIDE) -> np.ndarray:
    d, special = zipf_dictionary(seed, values)
    cdf = zipf_cdf(values, s)
    thresh = np.uint64(min(int(override * 2.0 ** 64), MASK64))
    out = np.empty((n, 2), dtype="<u8")
    chunk = 1 << 22
    st_o = stream_seed(seed, 2)
    for a in range(0, n, chunk):
        c = min(chunk, n - a)
        u = unit_doubles(seed, 1, a, c)
        rank = np.searchsorted(cdf, u, side="right")
        np.minimum(rank, values - 1, out=rank)
        key = d[rank]
        hit = splitmix64(st_o, a, c) < thresh
        key[hit] = np.uint64(special)
        out[a:a + c, 0] = key
        out[a:a + c, 1] = np.arange(a, a + c, dtype=np.uint64)
    return out.view(np.uint8).reshape(n, 16)


DEEP_HI_VALUES = 1 << 20


def deep32(n: int = 1 << 27, seed: int = 4, hi_values: int = DEEP_HI_VALUES) -> np.ndarray:
    out = np.empty((n, 4), dtype="<u8")
    chunk = 1 << 23
    for a in range(0, n, chunk):
        c = min(chunk, n - a)
        out[a:a + c, 0] = splitmix64(stream_seed(seed, 1), a, c)
        out[a:a + c, 1] = splitmix64(stream_seed(seed, 0), a, c) % np.uint64(hi_values)
        out[a:a + c, 2] = np.arange(a, a + c, dtype=np.uint64)
        out[a:a + c, 3] = splitmix64(stream_seed(seed, 2), a, c)
    return out.view(np.uint8).reshape(n, 32)


def batch_sizes(count: int = 65536, seed: int = 5, max_log2: int = 20) -> np.ndarray:
    """Sizes floor(exp(u * ln(2^max_log2 + 1))), u uniform in [0,1): log-uniform
    over [1, 2^max_log2]."""
    u = unit_doubles(seed, 0, 0, count)
    sizes = np.floor(np.exp(u * math.log((1 << max_log2) + 1))).astype(np.int64)
    return np.clip(sizes, 1, 1 << max_log2)


def batch_array(j: int, size: int, offset: int, seed: int = 5) -> np.ndarray:
    """Array j of the batch workload; `offset` = sum of the sizes before it."""
    out = np.empty((size, 2), dtype="<u8")
    out[:, 0] = splitmix64(stream_seed(seed, 1), offset, size)
    out[:, 1] = np.arange(size, dtype=np.uint64)
    return out.view(np.uint8).reshape(size, 16)


SWEEP_SEED = 6


def sweep_records(n: int, rec_bytes: int, key_bytes: int, seed: int = SWEEP_SEED) -> np.ndarray:
    """n records of rec_bytes (a multiple of 8) with key_bytes in {8, 16}:
    key words uniform over 64 bits each, then (if rec_bytes > key_bytes) a
    word holding the record's index, then uniform words."""
    assert rec_bytes % 8 == 0 and key_bytes in (8, 16) and key_bytes <= rec_bytes
    words = rec_bytes // 8
    kw = key_bytes // 8
    out = np.empty((n, words), dtype="<u8")
    chunk = 1 << 23
    for a in range(0, n, chunk):
        c = min(chunk, n - a)
        for q in range(words):
            if q == kw:
                out[a:a + c, q] = np.arange(a, a + c, dtype=np.uint64)
            else:
                out[a:a + c, q] = splitmix64(stream_seed(seed, 100 * rec_bytes + q), a, c)
    return out.view(np.uint8).reshape(n, rec_bytes)


def keys16(n: int = 1 << 28, seed: int = 7) -> np.ndarray:
    return sweep_records(n, 16, 16, seed=seed)


WORKLOADS = {
    "uniform8": dict(fn=uniform8, n=1 << 20, rec_bytes=8, key_bytes=8, seed=1),
    "uniform16": dict(fn=uniform16, n=1 << 28, rec_bytes=16, key_bytes=8, seed=2),
    "zipf16": dict(fn=zipf16, n=1 << 28, rec_bytes=16, key_bytes=8, seed=3),
    "deep32": dict(fn=deep32, n=1 << 27, rec_bytes=32, key_bytes=16, seed=4),
    "keys16": dict(fn=keys16, n=1 << 28, rec_bytes=16, key_bytes=16, seed=7),
}


def make(name: str, n: int | None = None) -> tuple[np.ndarray, int]:
    """Records of workload `name` (optionally with a smaller n) and key bytes."""
    w = WORKLOADS[name]
    nn = w["n"] if n is None else n
    return w["fn"](nn, seed=w["seed"]), w["key_bytes"]


def random_records(rng: np.random.Generator, n: int, rec_bytes: int, key_bytes: int,
                   distinct_keys: int | None = None) -> np.ndarray:
    """General-purpose test records: random bytes, optionally with only
    `distinct_keys` different keys (heavy duplicates)."""
    rec = rng.integers(0, 256, size=(n, rec_bytes), dtype=np.uint8)
    if distinct_keys is not None and n > 0:
        pool = rng.integers(0, 256, size=(distinct_keys, key_bytes), dtype=np.uint8)
        rec[:, :key_bytes] = pool[rng.integers(0, distinct_keys, size=n)]
    return rec


# --------------------------------------------------------------------------
# The same streams drawn directly in device memory (torch int64 arithmetic
# wraps modulo 2^64 like uint64; right shifts are made logical by masking).
# Bit-identical to `splitmix64` above; used to build multi-GiB inputs on the
# GPU without a host round trip.

def _s64(x: int) -> int:
    x &= MASK64
    return x - (1 << 64) if x >> 63 else x


def splitmix64_torch(state: int, start: int, count: int, device="cuda"):
    import torch
    i = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = i * _s64(GAMMA) + _s64(state)

    def lsr(x, k):
        return (x >> k) & ((1 << (64 - k)) - 1)

    z = (z ^ lsr(z, 30)) * _s64(0xBF58476D1CE4E5B9)
    z = (z ^ lsr(z, 27)) * _s64(0x94D049BB133111EB)
    return z ^ lsr(z, 31)


def uniform16_torch(n: int, seed: int = 2, device="cuda", chunk: int = 1 << 26):
    """uniform16 built on the device: returns an [n, 16] uint8 tensor."""
    import torch
    out = torch.empty((n, 2), dtype=torch.int64, device=device)
    st = stream_seed(seed, 0)
    for a in range(0, n, chunk):
        c = min(chunk, n - a)
        out[a:a + c, 0] = splitmix64_torch(st, a, c, device)
        out[a:a + c, 1] = torch.arange(a, a + c, dtype=torch.int64, device=device)
    return out.view(torch.uint8).view(n, 16)


def batch_array_torch(j: int, size: int, offset: int, seed: int = 5, device="cuda", out=None):
    """Array j of the batch workload built on the device ([size, 16] uint8)."""
    import torch
    w = torch.empty((size, 2), dtype=torch.int64, device=device) if out is None else out.view(torch.int64).view(size, 2)
    if size:
        w[:, 0] = splitmix64_torch(stream_seed(seed, 1), offset, size, device)
        w[:, 1] = torch.arange(size, dtype=torch.int64, device=device)
    return w.view(torch.uint8).view(size, 16)


def _u64_lt(a, b):
    """a < b for int64 tensors holding uint64 bit patterns."""
    sign = -(1 << 63)
    return (a ^ sign) < (b ^ sign)


def zipf16_torch(n: int, seed: int = 3, values: int = ZIPF_VALUES, s: float = ZIPF_S,
                 override: float = ZIPF_OVERRIDE, device="cuda", chunk: int = 1 << 25):
    """zipf16 built on the device (the dictionary and CDF on the host, the
    draws on the device): returns an [n, 16] uint8 tensor equal to zipf16."""
    import torch
    d, special = zipf_dictionary(seed, values)
    dd = torch.from_numpy(d.view(np.int64)).to(device)
    cdf = torch.from_numpy(zipf_cdf(values, s)).to(device)
    thresh = _s64(min(int(override * 2.0 ** 64), MASK64))
    out = torch.empty((n, 2), dtype=torch.int64, device=device)
    st_u, st_o = stream_seed(seed, 1), stream_seed(seed, 2)
    for a in range(0, n, chunk):
        c = min(chunk, n - a)
        z = splitmix64_torch(st_u, a, c, device)
        u = ((z >> 11) & ((1 << 53) - 1)).to(torch.float64) * (1.0 / (1 << 53))
        rank = torch.searchsorted(cdf, u, right=True).clamp_(max=values - 1)
        key = dd[rank]
        hit = _u64_lt(splitmix64_torch(st_o, a, c, device), torch.tensor(thresh, device=device))
        key[hit] = _s64(special)
        out[a:a + c, 0] = key
        out[a:a + c, 1] = torch.arange(a, a + c, dtype=torch.int64, device=device)
    return out.view(torch.uint8).view(n, 16)


def deep32_torch(n: int, seed: int = 4, hi_values: int = DEEP_HI_VALUES, device="cuda",
                 chunk: int = 1 << 25):
    """deep32 built on the device: returns an [n, 32] uint8 tensor equal to
    deep32 (hi_values must be a power of two)."""
    import torch
    assert hi_values & (hi_values - 1) == 0
    out = torch.empty((n, 4), dtype=torch.int64, device=device)
    for a in range(0, n, chunk):
        c = min(chunk, n - a)
        out[a:a + c, 0] = splitmix64_torch(stream_seed(seed, 1), a, c, device)
        out[a:a + c, 1] = splitmix64_torch(stream_seed(seed, 0), a, c, device) & (hi_values - 1)
        out[a:a + c, 2] = torch.arange(a, a + c, dtype=torch.int64, device=device)
        out[a:a + c, 3] = splitmix64_torch(stream_seed(seed, 2), a, c, device)
    return out.view(torch.uint8).view(n, 32)


def sweep_records_torch(n: int, rec_bytes: int, key_bytes: int, seed: int = SWEEP_SEED,
                        device="cuda", chunk: int = 1 << 25):
    """sweep_records built on the device: returns an [n, rec_bytes] uint8 tensor."""
    import torch
    assert rec_bytes % 8 == 0 and key_bytes in (8, 16) and key_bytes <= rec_bytes
    words = rec_bytes // 8
    kw = key_bytes // 8
    out = torch.empty((n, words), dtype=torch.int64, device=device)
    for a in range(0, n, chunk):
        c = min(chunk, n - a)
        for q in range(words):
            if q == kw:
                out[a:a + c, q] = torch.arange(a, a + c, dtype=torch.int64, device=device)
            else:
                out[a:a + c, q] = splitmix64_torch(stream_seed(seed, 100 * rec_bytes + q), a, c,
                                                   device)
    return out.view(torch.uint8).view(n, rec_bytes)


def uniform8_torch(n: int, seed: int = 1, device="cuda"):
    import torch
    return splitmix64_torch(stream_seed(seed, 0), 0, n, device).view(torch.uint8).view(n, 8)


def keys16_torch(n: int, seed: int = 7, device="cuda"):
    return sweep_records_torch(n, 16, 16, seed=seed, device=device)


def make_torch(name: str, n: int, device="cuda"):
    """Workload `name` with n records built on the device."""
    fns = {"uniform8": uniform8_torch, "uniform16": uniform16_torch, "zipf16": zipf16_torch, "deep32": deep32_torch,
           "keys16": keys16_torch}
    return fns[name](n, device=device)
