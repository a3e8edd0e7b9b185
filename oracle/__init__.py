"""CPU oracle for the RADULS2 record sort (arXiv 1703.00687).

TEST INFRASTRUCTURE ONLY.  The sorting library never imports, loads or calls
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` do.  It shares no code with the HIP path.

The arithmetic lives in ``oracle.cpp`` (plain C++, built with g++ into
``liboracle.so``); this module only marshals numpy arrays through ctypes and
adds pure-Python helpers used by the pins.

Record model: a record is R bytes, its key is bytes [0, K) read as an unsigned
little-endian integer (the paper's 8 B key + 8 B data records, Sec. 4.2; byte
order is a reading of ours, since the paper does not state one).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK = 0
E_INVALID = -1
E_UNSUPPORTED = -4


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with g++ (no GPU code involved)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.c_void_p
    u64 = ctypes.c_uint64
    u32 = ctypes.c_uint32
    lib.oracle_validate.argtypes = [u64, u32, u32]
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_sort.argtypes = [u8p, u8p, u64, u32, u32]
    lib.oracle_sort.restype = ctypes.c_int
    lib.oracle_sort_parallel.argtypes = [u8p, u8p, u64, u32, u32, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]
    lib.oracle_sort_parallel.restype = ctypes.c_int
    lib.oracle_histogram.argtypes = [u8p, u64, u32, u32, u32, u32, u8p]
    lib.oracle_histogram.restype = ctypes.c_int
    lib.oracle_exclusive_scan.argtypes = [u8p, u64, u64, u8p]
    lib.oracle_exclusive_scan.restype = None
    lib.oracle_partition.argtypes = [u8p, u8p, u64, u32, u32, u32, u32]
    lib.oracle_partition.restype = ctypes.c_int
    lib.oracle_enum_sort.argtypes = [u8p, u8p, u64, u32, u32]
    lib.oracle_enum_sort.restype = ctypes.c_int
    lib.oracle_msd_sort.argtypes = [u8p, u8p, u64, u32, u32, u32, u64]
    lib.oracle_msd_sort.restype = ctypes.c_int
    lib.oracle_bins_at_level.argtypes = [u8p, u64, u32, u32, u32, u32, u8p, u8p, u64]
    lib.oracle_bins_at_level.restype = u64
    lib.oracle_first_unsorted.argtypes = [u8p, u64, u32, u32]
    lib.oracle_first_unsorted.restype = u64
    _lib = lib
    return lib


def _as_records(recs: np.ndarray, rec_bytes: int | None = None) -> np.ndarray:
    a = np.ascontiguousarray(recs).view(np.uint8)
    if a.ndim == 1:
        if rec_bytes is None:
            raise ValueError("rec_bytes needed for a flat byte array")
        a = a.reshape(-1, rec_bytes)
    return a


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


class OracleError(RuntimeError):
    pass


def _check(st: int, what: str) -> None:
    if st != OK:
        raise OracleError(f"{what}: status {st}")


def validate(n: int, rec_bytes: int, key_bytes: int) -> int:
    return _load().oracle_validate(n, rec_bytes, key_bytes)


def sort(recs: np.ndarray, key_bytes: int) -> np.ndarray:
    """Stable sort by key: the definition of the result (std::stable_sort)."""
    a = _as_records(recs)
    n, R = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_sort(_ptr(a), _ptr(out), n, R, key_bytes), "oracle_sort")
    return out


def sort_parallel(recs: np.ndarray, key_bytes: int, threads: int = 0) -> tuple[np.ndarray, int]:
    """The same stable sort on several cores (libstdc++ parallel mode over
    OpenMP; `threads` = 0 takes all available).  Used only for the CPU
    baseline; returns (sorted records, threads used)."""
    a = _as_records(recs)
    n, R = a.shape
    out = np.empty_like(a)
    used = ctypes.c_int(0)
    _check(_load().oracle_sort_parallel(_ptr(a), _ptr(out), n, R, key_bytes, threads,
                                        ctypes.byref(used)), "oracle_sort_parallel")
    return out, int(used.value)


def histogram(recs: np.ndarray, key_bytes: int, bits: int, width: int) -> np.ndarray:
    a = _as_records(recs)
    n, R = a.shape
    w = min(width, bits)
    out = np.zeros(1 << w, dtype=np.uint64)
    _check(_load().oracle_histogram(_ptr(a), n, R, key_bytes, bits, width, _ptr(out)),
           "oracle_histogram")
    return out


def exclusive_scan(counts: np.ndarray, base: int = 0) -> np.ndarray:
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    out = np.zeros_like(c)
    _load().oracle_exclusive_scan(_ptr(c), c.size, base, _ptr(out))
    return out


def partition(recs: np.ndarray, key_bytes: int, bits: int, width: int) -> np.ndarray:
    a = _as_records(recs)
    n, R = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_partition(_ptr(a), _ptr(out), n, R, key_bytes, bits, width),
           "oracle_partition")
    return out


def enum_sort(recs: np.ndarray, key_bytes: int) -> np.ndarray:
    a = _as_records(recs)
    n, R = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_enum_sort(_ptr(a), _ptr(out), n, R, key_bytes), "oracle_enum_sort")
    return out


def msd_sort(recs: np.ndarray, key_bytes: int, width: int = 8, tiny_max: int = 32) -> np.ndarray:
    a = _as_records(recs)
    n, R = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_msd_sort(_ptr(a), _ptr(out), n, R, key_bytes, width, tiny_max),
           "oracle_msd_sort")
    return out


def bins_at_level(sorted_recs: np.ndarray, key_bytes: int, width: int, levels: int):
    a = _as_records(sorted_recs)
    n, R = a.shape
    lib = _load()
    need = lib.oracle_bins_at_level(_ptr(a), n, R, key_bytes, width, levels, 0, 0, 0)
    starts = np.zeros(max(int(need), 1), dtype=np.uint64)
    sizes = np.zeros_like(starts)
    got = lib.oracle_bins_at_level(_ptr(a), n, R, key_bytes, width, levels, _ptr(starts),
                                   _ptr(sizes), starts.size)
    return starts[:got], sizes[:got]


def first_unsorted(recs: np.ndarray, key_bytes: int) -> int:
    a = _as_records(recs)
    n, R = a.shape
    return int(_load().oracle_first_unsorted(_ptr(a), n, R, key_bytes))


# ---------------------------------------------------------------------------
# Checkers used by the parity tests (independent of the C++ sort above).

def key_columns(recs: np.ndarray, key_bytes: int) -> np.ndarray:
    """Key as an array of uint64 words, most significant word last.

    The top word is masked to the key bytes it holds.  Word i covers key bytes
    [8i, 8i+8)."""
    a = _as_records(recs)
    n, R = a.shape
    kw = (key_bytes + 7) // 8
    padded = np.zeros((n, kw * 8), dtype=np.uint8)
    padded[:, :key_bytes] = a[:, :key_bytes]
    return padded.view("<u8").reshape(n, kw)


def check_sorted(recs: np.ndarray, key_bytes: int) -> bool:
    """Keys non-decreasing (compared word-wise from the most significant)."""
    kc = key_columns(recs, key_bytes)
    n = kc.shape[0]
    if n < 2:
        return True
    a, b = kc[:-1], kc[1:]
    decided = np.zeros(n - 1, dtype=bool)
    ok = np.ones(n - 1, dtype=bool)
    for w in range(kc.shape[1] - 1, -1, -1):
        lt = (a[:, w] < b[:, w]) & ~decided
        gt = (a[:, w] > b[:, w]) & ~decided
        ok &= ~gt
        decided |= lt | gt
    return bool(ok.all())


def same_multiset(x: np.ndarray, y: np.ndarray) -> bool:
    """Whole records of x and y form the same multiset."""
    xa = _as_records(x)
    ya = _as_records(y)
    if xa.shape != ya.shape:
        return False
    if xa.shape[0] == 0:
        return True
    cols = [xa[:, i] for i in range(xa.shape[1] - 1, -1, -1)]
    ox = np.lexsort(cols)
    cols = [ya[:, i] for i in range(ya.shape[1] - 1, -1, -1)]
    oy = np.lexsort(cols)
    return bool(np.array_equal(xa[ox], ya[oy]))


def parity(gpu_out: np.ndarray, expected: np.ndarray, key_bytes: int) -> bool:
    """Parity rule for results with several correct answers: equal key
    sequences, and each maximal run of equal keys holds the same multiset of
    whole records.  Byte identity implies it."""
    g = _as_records(gpu_out)
    e = _as_records(expected)
    if g.shape != e.shape:
        return False
    if np.array_equal(g, e):
        return True
    kg = key_columns(g, key_bytes)
    ke = key_columns(e, key_bytes)
    if not np.array_equal(kg, ke):
        return False
    n = kg.shape[0]
    change = np.any(kg[1:] != kg[:-1], axis=1)
    bounds = np.concatenate(([0], np.nonzero(change)[0] + 1, [n]))
    for s, t in zip(bounds[:-1], bounds[1:]):
        if t - s > 1 and not same_multiset(g[s:t], e[s:t]):
            return False
    return True
