"""Grid search over the library's tuning knobs on synthetic inputs.

Times the plain sort for each candidate setting (HIP events around the call,
inputs resident, a fresh copy per repetition) and keeps the fastest.  The
result is cached as JSON keyed by (device arch, record bytes, key bytes,
log2 of the record count), and ``apply`` loads the best setting for a call
shape into the process-global tuning.  The sort's output never depends on
the tuning; the candidate setting that wins is verified to sort correctly.
"""

from __future__ import annotations

import itertools
import json
import math
import os
import time

from . import binding as b

DEFAULT_CACHE = os.environ.get(
    "RADULS_TUNE_FILE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json"))

SPACE = {
    "digit_bits": [8, 7, 6],
    "tile_items": [0, 5, 4, 3, 2],      # records per thread of a scatter tile (0: the most)
    "tiny_max": [64, 32, 16, 128],
    "mid_frac": [1.0, 0.75, 0.5],       # mid_max as a fraction of the LDS capacity
    "wave_job_max": [0, 128, 64, 1],    # largest wave-network job (0: the most, 1: none)
    "nontemporal": [1, 2],
    "lookback": [0, 1],
    "pair_hist": [1, 2],
}


def shape_key(arch: str, rec_bytes: int, key_bytes: int, n: int, workload: str | None = None) -> str:
    """Cache key of a call shape; `workload` names the key distribution the
    entry was tuned on (inputs of one shape can want different settings)."""
    k = f"{arch}/R{rec_bytes}/K{key_bytes}/n2^{max(0, int(round(math.log2(max(n, 1)))))}"
    return f"{k}/{workload}" if workload else k


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(cache: dict, arch: str, rec_bytes: int, key_bytes: int, n: int,
           workload: str | None = None):
    """(key, entry) of the cache entry for this shape, or (None, None): the
    same arch, R and K; an entry tuned on `workload` first, then one with no
    workload named; among those the nearest record count.  Entries tuned on
    another distribution are not used."""
    prefix = f"{arch}/R{rec_bytes}/K{key_bytes}/n2^"
    want = math.log2(max(n, 1))
    best = None
    for k, v in cache.items():
        if not k.startswith(prefix):
            continue
        rest = k[len(prefix):].split("/", 1)
        wl_name = rest[1] if len(rest) > 1 else None
        if wl_name is not None and wl_name != workload:
            continue
        score = (wl_name is None, abs(int(rest[0]) - want))
        if best is None or score < best[0]:
            best = (score, k, v)
    return (None, None) if best is None else (best[1], best[2])


def apply(rec_bytes: int, key_bytes: int, n: int, workload: str | None = None,
          path: str = DEFAULT_CACHE):
    """Set the process-global tuning from the cache entry for this shape
    (see lookup); returns (key, entry), or (None, None) with the tuning
    left as it was."""
    key, entry = lookup(load_cache(path), _arch(), rec_bytes, key_bytes, n, workload)
    if entry is not None:
        b.raduls_set_tuning(**entry["tuning"])
    return key, entry


def _time_sort(src, copies, tmp, n, R, K, reps):
    import torch
    times = []
    for i in range(reps):
        c = copies[i % len(copies)]
        c.copy_(src)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        b.raduls_sort(c, tmp, n, R, K)
        e.record()
        e.synchronize()
        times.append(s.elapsed_time(e))
    times.sort()
    return times[len(times) // 2]


def _looks_sorted(out, src, key_bytes: int) -> bool:
    """Keys non-decreasing (keys up to 16 bytes) and the same records in
    total (two wrapping sums of every 64-bit word, one of them weighted by a
    function of the whole record)."""
    import torch
    n, R = int(out.shape[0]), int(out.shape[1])
    if n < 2:
        return True
    w = out.view(torch.int64).view(n, R // 8)
    ws = src.view(torch.int64).view(n, R // 8)

    def digest(x):
        h = x.sum(1) * -7046029254386353131 + x[:, 0]  # per record, wrapping
        return x.sum(0), (h * (h | 1)).sum()

    (a0, a1), (b0, b1) = digest(w), digest(ws)
    if not (bool((a0 == b0).all()) and bool(a1 == b1)):
        return False
    if key_bytes > 16:
        return True
    sign = -(1 << 63)
    kw = (key_bytes + 7) // 8
    cols = []
    for q in range(kw):
        col = w[:, q]
        bytes_here = min(8, key_bytes - 8 * q)
        if bytes_here < 8:
            col = col & ((1 << (8 * bytes_here)) - 1)
        cols.append(col ^ sign)
    le = torch.ones(n - 1, dtype=torch.bool, device=out.device)
    for col in cols:  # least significant word first
        a, c = col[:-1], col[1:]
        le = (c > a) | ((c == a) & le)
    return bool(le.all())


def tune(src, key_bytes: int, reps: int = 5, space: dict | None = None, budget_s: float = 300.0,
         path: str | None = DEFAULT_CACHE, log=print, workload: str | None = None) -> dict:
    """Search the space for the [n, R] uint8 device tensor `src` (left
    unchanged).  Coordinate descent from the defaults: one knob at a time over
    its values, keeping the best, repeated while it improves and time lasts."""
    import torch
    space = dict(SPACE if space is None else space)
    n, R = int(src.shape[0]), int(src.shape[1])
    cap = b.raduls_mid_capacity(R, key_bytes)
    copies = [torch.empty_like(src) for _ in range(2)]
    prev = b.raduls_get_tuning()
    t_start = time.perf_counter()

    def cand_to_tuning(c):
        return {"digit_bits": c["digit_bits"], "tiny_max": c["tiny_max"],
                "mid_max": max(64, int(cap * c["mid_frac"]) // 64 * 64),
                "nontemporal": c["nontemporal"], "lookback": c["lookback"],
                "pair_hist": c.get("pair_hist", 1), "grid_blocks": 0,
                "tile_items": c.get("tile_items", 0), "wave_job_max": c.get("wave_job_max", 0)}

    def measure(c):
        t = cand_to_tuning(c)
        b.raduls_set_tuning(**t)
        tmp = torch.empty(b.raduls_tmp_bytes(n, R, key_bytes), dtype=torch.uint8, device=src.device)
        ms = _time_sort(src, copies, tmp, n, R, key_bytes, reps)
        st, stats = b.raduls_check(tmp, n, R, False)
        if st != b.OK:
            return float("inf")
        return ms

    cur = {k: v[0] for k, v in space.items()}
    best_ms = measure(cur)
    default_ms = best_ms  # the first value of every knob is its default
    log(f"[autotune] start {cur} {best_ms:.3f} ms")
    improved = True
    while improved and time.perf_counter() - t_start < budget_s:
        improved = False
        for knob, values in space.items():
            for v in values:
                if v == cur[knob] or time.perf_counter() - t_start > budget_s:
                    continue
                c = dict(cur, **{knob: v})
                ms = measure(c)
                log(f"[autotune] {knob}={v}: {ms:.3f} ms")
                if ms < best_ms * 0.99:
                    best_ms, cur, improved = ms, c, True
    best = {"tuning": cand_to_tuning(cur), "ms": best_ms, "n": n,
            "records_per_s": n / (best_ms * 1e-3), "default_ms": default_ms,
            "changed": {k: v for k, v in cur.items() if v != space[k][0]},
            "workload": workload}
    # the winner must sort: no device error, keys non-decreasing and the
    # record words' sum and xor unchanged
    b.raduls_set_tuning(**best["tuning"])
    out = copies[0]
    out.copy_(src)
    tmp = torch.empty(b.raduls_tmp_bytes(n, R, key_bytes), dtype=torch.uint8, device=src.device)
    b.raduls_sort(out, tmp, n, R, key_bytes)
    st, stats = b.raduls_check(tmp, n, R, False)
    if st != b.OK or not _looks_sorted(out, src, key_bytes):
        b.raduls_set_tuning(**prev)
        raise RuntimeError(f"autotune: the winning setting {best['tuning']} did not sort ({stats})")
    if path:
        cache = load_cache(path)
        cache[shape_key(_arch(), R, key_bytes, n, workload)] = best
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    b.raduls_set_tuning(**prev)
    return best


if __name__ == "__main__":
    import argparse
    import torch
    from . import workloads as wl
    ap = argparse.ArgumentParser(description="tune the sort for workloads at their full sizes")
    ap.add_argument("--workloads", nargs="+", default=["uniform16", "zipf16", "deep32"])
    ap.add_argument("--log2n", type=int, default=None, help="records = 2^k (default: the workload's)")
    ap.add_argument("--budget-s", type=float, default=240)
    args = ap.parse_args()
    for name in args.workloads:
        spec = wl.WORKLOADS[name]
        n = spec["n"] if args.log2n is None else 1 << args.log2n
        src = wl.make_torch(name, n, device=torch.device("cuda:0"))
        torch.cuda.synchronize()
        best = tune(src, spec["key_bytes"], budget_s=args.budget_s, workload=name,
                    log=lambda m: print(m, flush=True))
        print(json.dumps({name: best}), flush=True)
        del src
        torch.cuda.empty_cache()
