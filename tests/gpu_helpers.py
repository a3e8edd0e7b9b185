"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
with guard bands around every buffer, and compare with the CPU oracle."""

from __future__ import annotations

import numpy as np
import torch

from paper_1703_00687_amd import binding as b

GUARD = 4096
CANARY_RECS = 0xA5
CANARY_TMP = 0x5A


def dev():
    return torch.device("cuda:0")


def guarded(nbytes: int, fill: int):
    buf = torch.full((nbytes + 2 * GUARD,), fill, dtype=torch.uint8, device=dev())
    return buf, buf[GUARD:GUARD + nbytes]


def guards_intact(buf: torch.Tensor, nbytes: int, fill: int) -> bool:
    head = buf[:GUARD]
    tail = buf[GUARD + nbytes:]
    return bool((head == fill).all().item()) and bool((tail == fill).all().item())


def gpu_sort(recs: np.ndarray, key_bytes: int, check_stats: bool = True):
    """Sort host records on the GPU; returns (sorted host records, stats)."""
    n, r = recs.shape
    need = b.raduls_tmp_bytes(n, r, key_bytes)
    rbuf, rv = guarded(n * r, CANARY_RECS)
    tbuf, tv = guarded(need, CANARY_TMP)
    if n:
        rv.copy_(torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)))
    b.raduls_sort(rv, tv, n, r, key_bytes)
    stats = {}
    if n > 1:
        st, stats = b.raduls_check(tv, n, r, False)
        if check_stats:
            assert st == b.OK, stats
    torch.cuda.synchronize()
    assert guards_intact(rbuf, n * r, CANARY_RECS), "write outside recs"
    assert guards_intact(tbuf, need, CANARY_TMP), "write outside tmp"
    out = rv.cpu().numpy().reshape(n, r) if n else np.zeros((0, r), np.uint8)
    return out, stats


def tuned(**fields):
    """Context manager setting tuning fields for the duration of a block."""

    class _T:
        def __enter__(self):
            self.prev = b.raduls_set_tuning(**fields)
            return self

        def __exit__(self, *exc):
            b.raduls_set_tuning(**self.prev)
            return False

    return _T()
