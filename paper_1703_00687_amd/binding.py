"""ctypes binding of libraduls.so (declared in include/raduls.h).

Argument marshalling only: every step of the sort runs in the HIP kernels of
the native library.  Functions named ``raduls_*`` mirror the C entry points
one to one (device pointers may be given as ints or as torch tensors, whose
``data_ptr()`` is used); ``sort`` and ``sort_batch`` are conveniences that
allocate the scratch buffers through torch and call them.  If the library is
missing the first call raises: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libraduls.so")

OK = 0
E_INVALID = -1
E_ALIGN = -2
E_TMP_SMALL = -3
E_UNSUPPORTED = -4
E_HIP = -5
E_DEVICE = -6
E_SCRATCH = -7
E_BUSY = -8
E_STOPPED = -9
E_TIMEOUT = -10


class RadulsError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status) if _lib is not None else status} ({status})")


class raduls_tuning(ctypes.Structure):
    _fields_ = [
        ("digit_bits", ctypes.c_uint32),
        ("tiny_max", ctypes.c_uint32),
        ("mid_max", ctypes.c_uint32),
        ("grid_blocks", ctypes.c_uint32),
        ("nontemporal", ctypes.c_uint32),
        ("lookback", ctypes.c_uint32),
        ("pair_hist", ctypes.c_uint32),
        ("wave_job_max", ctypes.c_uint32),
        ("es_job_max", ctypes.c_uint32),
        ("tile_items", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 6),
    ]


class raduls_stats(ctypes.Structure):
    _fields_ = [
        ("error", ctypes.c_uint32),
        ("rounds", ctypes.c_uint32),
        ("large_bins", ctypes.c_uint32),
        ("scattered_bins", ctypes.c_uint32),
        ("mid_jobs", ctypes.c_uint32),
        ("copy_jobs", ctypes.c_uint32),
        ("moved_records", ctypes.c_uint64),
        ("large_records", ctypes.c_uint64),
        ("pair_rounds", ctypes.c_uint32),
        ("eq_bins", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_ if name != "reserved"}


class raduls_bin(ctypes.Structure):
    _fields_ = [("start", ctypes.c_uint32), ("size", ctypes.c_uint32), ("bits", ctypes.c_uint32),
                ("side", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class raduls_array(ctypes.Structure):
    _fields_ = [("recs", ctypes.c_void_p), ("tmp", ctypes.c_void_p), ("n", ctypes.c_uint64)]


TUNING_FIELDS = ("digit_bits", "tiny_max", "mid_max", "grid_blocks", "nontemporal", "lookback",
                 "pair_hist", "wave_job_max", "es_job_max", "tile_items")

_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libraduls.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing; build it with `python -m paper_1703_00687_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    sig = {
        "raduls_tmp_bytes": (i32, [u64, u32, u32, u64p]),
        "raduls_sort": (i32, [vp, vp, u64, u32, u32, vp]),
        "raduls_sort_static": (i32, [vp, vp, u64, u32, u32, vp]),
        "raduls_batch_ws_bytes": (i32, [u32, u64, u32, u32, u64p]),
        "raduls_sort_batch": (i32, [vp, u32, u64, u32, u32, vp, u64, vp]),
        "raduls_step_ws_bytes": (i32, [u64, u32, u32, u64p]),
        "raduls_histogram": (i32, [vp, u64, u32, u32, u32, u32, vp, vp, u64, vp]),
        "raduls_partition": (i32, [vp, vp, u64, u32, u32, u32, u32, vp, vp, u64, vp]),
        "raduls_check": (i32, [vp, u64, u32, i32, ctypes.POINTER(raduls_stats), vp]),
        "raduls_set_tuning": (i32, [ctypes.POINTER(raduls_tuning)]),
        "raduls_get_tuning": (i32, [ctypes.POINTER(raduls_tuning)]),
        "raduls_mid_capacity": (u32, [u32, u32]),
        "raduls_inspect_rounds": (i32, [vp, vp, u64, u32, u32, u32, ctypes.POINTER(raduls_bin), u32,
                                        ctypes.POINTER(ctypes.c_uint32), vp]),
        "raduls_set_profile_events": (i32, [ctypes.POINTER(ctypes.c_void_p), u32]),
        "raduls_server_max_records": (i32, [u32, u32, u64p]),
        "raduls_server_create": (i32, [u32, u32, u32, u32, u32, u32, ctypes.POINTER(vp)]),
        "raduls_server_submit": (i32, [vp, vp, u64, u64p]),
        "raduls_server_submit_many": (i32, [vp, ctypes.POINTER(vp), u64p, u32, u64p,
                                            ctypes.POINTER(ctypes.c_uint32)]),
        "raduls_server_poll": (i32, [vp, u64, ctypes.POINTER(ctypes.c_uint32)]),
        "raduls_server_wait": (i32, [vp, u64, u32, ctypes.POINTER(ctypes.c_uint32)]),
        "raduls_server_wait_range": (i32, [vp, u64, u64, u32, ctypes.POINTER(ctypes.c_uint32)]),
        "raduls_server_completed": (i32, [vp, u64p, ctypes.POINTER(ctypes.c_uint32)]),
        "raduls_server_info": (i32, [vp, u64p, ctypes.POINTER(ctypes.c_uint32),
                                     ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
        "raduls_server_destroy": (i32, [vp]),
        "raduls_strerror": (ctypes.c_char_p, [i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return [
        "raduls_tmp_bytes", "raduls_sort", "raduls_batch_ws_bytes", "raduls_sort_batch",
        "raduls_step_ws_bytes", "raduls_histogram", "raduls_partition", "raduls_check",
        "raduls_set_tuning", "raduls_get_tuning", "raduls_mid_capacity", "raduls_strerror",
        "raduls_inspect_rounds", "raduls_sort_static",
        "raduls_set_profile_events",
        "raduls_server_max_records", "raduls_server_create", "raduls_server_submit",
        "raduls_server_submit_many", "raduls_server_poll", "raduls_server_wait_range",
        "raduls_server_completed", "raduls_server_wait", "raduls_server_info", "raduls_server_destroy",
    ]


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, ctypes.c_void_p):
        return x.value
    raise TypeError(f"cannot take a device pointer from {type(x)}")


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status: int, what: str) -> None:
    if status != OK:
        raise RadulsError(status, what)


def strerror(status: int) -> str:
    return load().raduls_strerror(status).decode()


# ---------------------------------------------------------------- C entry points

def raduls_tmp_bytes(n: int, rec_bytes: int, key_bytes: int) -> int:
    out = ctypes.c_uint64()
    _check(load().raduls_tmp_bytes(n, rec_bytes, key_bytes, ctypes.byref(out)), "raduls_tmp_bytes")
    return out.value


def raduls_sort(recs, tmp, n: int, rec_bytes: int, key_bytes: int, stream=None,
                raise_on_error: bool = True) -> int:
    st = load().raduls_sort(_ptr(recs), _ptr(tmp), n, rec_bytes, key_bytes, _stream(stream))
    if raise_on_error:
        _check(st, "raduls_sort")
    return st


def raduls_sort_static(recs, tmp, n: int, rec_bytes: int, key_bytes: int, stream=None,
                       raise_on_error: bool = True) -> int:
    st = load().raduls_sort_static(_ptr(recs), _ptr(tmp), n, rec_bytes, key_bytes, _stream(stream))
    if raise_on_error:
        _check(st, "raduls_sort_static")
    return st


def raduls_batch_ws_bytes(count: int, total_n: int, rec_bytes: int, key_bytes: int) -> int:
    out = ctypes.c_uint64()
    _check(load().raduls_batch_ws_bytes(count, total_n, rec_bytes, key_bytes, ctypes.byref(out)),
           "raduls_batch_ws_bytes")
    return out.value


def raduls_sort_batch(d_arrays, count: int, total_n: int, rec_bytes: int, key_bytes: int, ws,
                      ws_bytes: int, stream=None, raise_on_error: bool = True) -> int:
    st = load().raduls_sort_batch(_ptr(d_arrays), count, total_n, rec_bytes, key_bytes, _ptr(ws),
                                  ws_bytes, _stream(stream))
    if raise_on_error:
        _check(st, "raduls_sort_batch")
    return st


def raduls_step_ws_bytes(n: int, rec_bytes: int, key_bytes: int) -> int:
    out = ctypes.c_uint64()
    _check(load().raduls_step_ws_bytes(n, rec_bytes, key_bytes, ctypes.byref(out)),
           "raduls_step_ws_bytes")
    return out.value


def raduls_histogram(recs, n: int, rec_bytes: int, key_bytes: int, bits: int, width: int,
                     d_counts, ws, ws_bytes: int, stream=None, raise_on_error: bool = True) -> int:
    st = load().raduls_histogram(_ptr(recs), n, rec_bytes, key_bytes, bits, width, _ptr(d_counts),
                                 _ptr(ws), ws_bytes, _stream(stream))
    if raise_on_error:
        _check(st, "raduls_histogram")
    return st


def raduls_partition(src, dst, n: int, rec_bytes: int, key_bytes: int, bits: int, width: int,
                     d_offsets, ws, ws_bytes: int, stream=None, raise_on_error: bool = True) -> int:
    st = load().raduls_partition(_ptr(src), _ptr(dst), n, rec_bytes, key_bytes, bits, width,
                                 _ptr(d_offsets), _ptr(ws), ws_bytes, _stream(stream))
    if raise_on_error:
        _check(st, "raduls_partition")
    return st


def raduls_check(tmp_or_ws, n: int, rec_bytes: int, ws_only: bool, stream=None) -> tuple[int, dict]:
    s = raduls_stats()
    st = load().raduls_check(_ptr(tmp_or_ws), n, rec_bytes, int(ws_only), ctypes.byref(s),
                             _stream(stream))
    if st not in (OK, E_DEVICE):
        _check(st, "raduls_check")
    return st, s.as_dict()


def raduls_get_tuning() -> dict:
    t = raduls_tuning()
    _check(load().raduls_get_tuning(ctypes.byref(t)), "raduls_get_tuning")
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}


def raduls_set_tuning(**fields) -> dict:
    """Set tuning fields (others keep their value); returns the previous tuning."""
    prev = raduls_get_tuning()
    t = raduls_tuning()
    for k in TUNING_FIELDS:
        setattr(t, k, int(fields.get(k, prev[k])))
    unknown = set(fields) - set(TUNING_FIELDS)
    if unknown:
        raise KeyError(f"unknown tuning fields {sorted(unknown)}")
    _check(load().raduls_set_tuning(ctypes.byref(t)), "raduls_set_tuning")
    return prev


def raduls_set_profile_events(events: Sequence[int]) -> None:
    arr = (ctypes.c_void_p * max(len(events), 1))(*events)
    _check(load().raduls_set_profile_events(arr, len(events)), "raduls_set_profile_events")


def raduls_mid_capacity(rec_bytes: int, key_bytes: int) -> int:
    return int(load().raduls_mid_capacity(rec_bytes, key_bytes))


def raduls_inspect_rounds(recs, tmp, n: int, rec_bytes: int, key_bytes: int, rounds: int,
                          cap: int = 1 << 20, stream=None) -> list[tuple[int, int, int, int]]:
    """Run the first `rounds` global rounds only and return the large bins
    they left, as (start, size, bits, side, flags) tuples (synchronizes)."""
    arr = (raduls_bin * max(cap, 1))()
    cnt = ctypes.c_uint32(0)
    _check(load().raduls_inspect_rounds(_ptr(recs), _ptr(tmp), n, rec_bytes, key_bytes, rounds, arr,
                                        cap, ctypes.byref(cnt), _stream(stream)),
           "raduls_inspect_rounds")
    k = min(int(cnt.value), cap)
    return [(arr[i].start, arr[i].size, arr[i].bits, arr[i].side, arr[i].flags) for i in range(k)]


def raduls_server_max_records(rec_bytes: int, key_bytes: int) -> int:
    out = ctypes.c_uint64(0)
    _check(load().raduls_server_max_records(rec_bytes, key_bytes, ctypes.byref(out)),
           "raduls_server_max_records")
    return int(out.value)


class ResidentServer:
    """The resident server of raduls.h: `workgroups` workgroups of the LDS
    sorter stay on the device and sort submitted arrays of at most
    ``max_records`` records in place, with no launch per request.  Use as a
    context manager (or call ``close``); ``submit`` returns a ticket that
    ``poll`` / ``wait`` take."""

    def __init__(self, rec_bytes: int, key_bytes: int, slots: int = 4096, workgroups: int = 0,
                 idle_ms: int = 0, lease_ms: int = 0):
        self.rec_bytes, self.key_bytes = rec_bytes, key_bytes
        h = ctypes.c_void_p()
        _check(load().raduls_server_create(rec_bytes, key_bytes, slots, workgroups, idle_ms,
                                           lease_ms, ctypes.byref(h)), "raduls_server_create")
        self._h = h
        self.max_records, self.workgroups, _, _ = self.info()

    def info(self) -> tuple[int, int, bool, int]:
        """(max_records, workgroups, running, reason: 0, 1 stopped, 2 idle, 3 lease)."""
        m, w, r, why = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(load().raduls_server_info(self._h, ctypes.byref(m), ctypes.byref(w), ctypes.byref(r),
                                         ctypes.byref(why)), "raduls_server_info")
        return int(m.value), int(w.value), bool(r.value), int(why.value)

    def submit_status(self, recs, n: int | None = None) -> tuple[int, int]:
        """(status, ticket): the raw result of raduls_server_submit."""
        if n is None:
            n = int(recs.shape[0])
        t = ctypes.c_uint64(0)
        st = load().raduls_server_submit(self._h, _ptr(recs) if n else None, n, ctypes.byref(t))
        return st, int(t.value)

    def submit(self, recs, n: int | None = None) -> int:
        st, t = self.submit_status(recs, n)
        _check(st, "raduls_server_submit")
        return t

    def submit_many(self, ptrs, ns) -> tuple[int, int]:
        """Submit arrays by device address and record count (sequences or
        numpy arrays); returns (first ticket, how many were accepted: fewer
        than given when the ring's slots ran out)."""
        import numpy as np
        p = np.ascontiguousarray(ptrs, dtype=np.uint64)
        n = np.ascontiguousarray(ns, dtype=np.uint64)
        if p.shape != n.shape:
            raise ValueError("one record count per array")
        first, acc = ctypes.c_uint64(0), ctypes.c_uint32(0)
        _check(load().raduls_server_submit_many(
            self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p)),
            n.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), p.size, ctypes.byref(first),
            ctypes.byref(acc)), "raduls_server_submit_many")
        return int(first.value), int(acc.value)

    def poll(self, ticket: int) -> tuple[int, int]:
        """(1 done / 0 pending / negative status, device error bits)."""
        s = ctypes.c_uint32(0)
        r = load().raduls_server_poll(self._h, ticket, ctypes.byref(s))
        return int(r), int(s.value)

    def wait(self, ticket: int, timeout_ms: int = 10000) -> int:
        """Wait for the request; returns its device error bits (0: sorted)."""
        s = ctypes.c_uint32(0)
        r = load().raduls_server_wait(self._h, ticket, timeout_ms, ctypes.byref(s))
        if r < 0:
            raise RadulsError(r, "raduls_server_wait")
        return int(s.value)

    def completed(self) -> tuple[int, int]:
        """(tickets below this have all completed, OR of the status words of
        those newly found done); raises if requests are pending and the
        kernel was stopped or could not be relaunched."""
        t, s = ctypes.c_uint64(0), ctypes.c_uint32(0)
        _check(load().raduls_server_completed(self._h, ctypes.byref(t), ctypes.byref(s)),
               "raduls_server_completed")
        return int(t.value), int(s.value)

    def wait_range(self, first: int, count: int, timeout_ms: int = 10000) -> int:
        """Wait for tickets [first, first + count); returns the OR of their
        device error bits (0: all sorted)."""
        s = ctypes.c_uint32(0)
        _check(load().raduls_server_wait_range(self._h, first, count, timeout_ms, ctypes.byref(s)),
               "raduls_server_wait_range")
        return int(s.value)

    def close(self) -> None:
        if self._h:
            h, self._h = self._h, None
            _check(load().raduls_server_destroy(h), "raduls_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def raduls_strerror(status: int) -> str:
    return strerror(status)


# ---------------------------------------------------------------- conveniences

def sort(recs, key_bytes: int, tmp=None, stream=None):
    """Sort a [n, R] uint8 CUDA tensor in place by its first key_bytes bytes.

    Allocates the scratch buffer through torch when none is given."""
    import torch
    n, rec_bytes = recs.shape
    if tmp is None:
        tmp = torch.empty(raduls_tmp_bytes(n, rec_bytes, key_bytes), dtype=torch.uint8,
                          device=recs.device)
    raduls_sort(recs, tmp, n, rec_bytes, key_bytes, stream)
    return recs


class Batch:
    """Device-side descriptor table and workspace for raduls_sort_batch.

    Holds torch buffers sized for `count` arrays of at most `total_n` records
    together; ``sort`` writes the descriptors of the given arrays and enqueues
    the batched sort."""

    def __init__(self, count: int, total_n: int, rec_bytes: int, key_bytes: int, device="cuda"):
        import torch
        self.count, self.total_n = count, total_n
        self.rec_bytes, self.key_bytes = rec_bytes, key_bytes
        self.ws_bytes = raduls_batch_ws_bytes(count, total_n, rec_bytes, key_bytes)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)
        self.desc = torch.zeros((max(count, 1), 3), dtype=torch.int64, device=device)
        self.host_desc = torch.zeros((max(count, 1), 3), dtype=torch.int64).pin_memory()

    def set_arrays(self, recs: Sequence, tmps: Sequence, stream=None) -> None:
        import torch
        if len(recs) != self.count or len(tmps) != self.count:
            raise ValueError("one recs and one tmp buffer per array")
        for i, (r, t) in enumerate(zip(recs, tmps)):
            self.host_desc[i, 0] = _ptr(r)
            self.host_desc[i, 1] = _ptr(t)
            self.host_desc[i, 2] = int(r.shape[0]) if hasattr(r, "shape") else 0
        s = torch.cuda.current_stream() if stream is None else stream
        with torch.cuda.stream(s):
            self.desc.copy_(self.host_desc)

    def launch(self, stream=None) -> None:
        raduls_sort_batch(self.desc, self.count, self.total_n, self.rec_bytes, self.key_bytes,
                          self.ws, self.ws_bytes, stream)

    def check(self, stream=None) -> tuple[int, dict]:
        return raduls_check(self.ws, 0, self.rec_bytes, True, stream)


def sort_batch(arrays: Sequence, key_bytes: int, stream=None):
    """Sort every [n_i, R] uint8 CUDA tensor of `arrays` in place, in one
    batched call."""
    import torch
    if not arrays:
        return arrays
    rec_bytes = int(arrays[0].shape[1])
    total = sum(int(a.shape[0]) for a in arrays)
    b = Batch(len(arrays), total, rec_bytes, key_bytes, device=arrays[0].device)
    tmps = [torch.empty_like(a) if a.shape[0] else a for a in arrays]
    b.set_arrays(arrays, tmps, stream)
    b.launch(stream)
    b._keep = tmps
    return arrays
