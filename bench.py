#!/usr/bin/env python3
"""Throughput of the MSD radix sort on one MI355X.

Workload (default): 2^28 records of 16 B -- a uint64 key uniform over 64 bits
and a uint64 payload holding the record's input index -- sorted by the 8 key
bytes with 1-byte digits.  `--workload` selects the others (uniform8, zipf16,
deep32, keys16) and `--rec-sweep` adds records of 8-64 B.  Synthetic and
seeded, generated on the device; every step sorts its own resident copy of
the input, so the timed region holds nothing but sorts.  The default run also
compares one batched call over 65,536 uneven arrays with one call per array
and serves the same arrays as a request stream.

Prints one JSON line.  `value` is records sorted per second over the timed
steps.  `roofline` covers the dominant kernel class: of the three passes that
move every record once (top-level scatter, second-round scatter, LDS sort), the
one with the largest time, from HIP events recorded around its launch in every
timed step: algorithmic bytes per launch = 2 * n * R (every record read once
and written once) over its mean duration, against the 8 TB/s HBM peak;
`move_passes` gives the same fraction for each of the three.  `cpu_baseline` is
the CPU oracle's stable sort timed on the host: in libstdc++ parallel mode on
all the cores the process may use (`value`, `cores`) and on one thread.
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "records sorted/s and % of HBM roofline (16B recs, 2^28); batched vs plain"
PROFILE_SLOTS = ["top_hist", "top_scatter", "round2_hist", "round2_scatter", "lds_sort"]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


class HipEvents:
    """Raw HIP events through libamdhip64 (the library records them)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self, count: int) -> list[int]:
        out = []
        for _ in range(count):
            ev = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(ev)) != 0:
                raise RuntimeError("hipEventCreate failed")
            out.append(ev.value)
        return out

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b) != 0:
            return float("nan")
        return float(ms.value)

    def destroy(self, evs: list[int]) -> None:
        for e in evs:
            self.hip.hipEventDestroy(e)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("raduls_kernels.hpp", "raduls_common.hpp"):
        with open(os.path.join(ROOT, "paper_1703_00687_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(phase: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{phase}_{workload}.json")


def load_traffic(workload: str, n: int, rec_bytes: int, phase: str) -> float | None:
    """HBM bytes per launch of the roofline kernel class from committed PMC
    counters, if they were taken on the current kernel source for this
    workload and size."""
    try:
        with open(traffic_file(phase, workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_source_hash") != kernel_source_hash() or t.get("n") != n
            or t.get("rec_bytes") != rec_bytes):
        return None
    return t.get("hbm_bytes_per_launch")


def _u64(x):
    """Order-preserving map of uint64 bit patterns (in int64) onto int64."""
    return x ^ (-(1 << 63))


def lexsort_order(wi, kw):
    """Permutation that stably sorts the rows of wi (int64 [n, words]) by
    their first kw words as one unsigned integer (word kw-1 most
    significant), from torch's own stable sort one word at a time, least
    significant first."""
    import torch
    order = torch.arange(wi.shape[0], device=wi.device)
    for q in range(kw):
        col = wi[:, q].contiguous()
        o = torch.sort(_u64(col[order]), stable=True).indices
        order = order[o]
    return order


def check_sorted_device(out, src, n, R, K):
    """Sort properties on the device.  Keys (K a multiple of 8) must not
    decrease.  With a payload word after the key holding the input index:
    the indices form a permutation, every record equals the input record its
    index names, and equal keys keep input order -- together they pin the
    unique stable result.  Without one (the record is all key): the output
    must equal torch's own stable lexicographic sort of the input."""
    import torch
    words, kw = R // 8, K // 8
    w = out.view(torch.int64).view(n, words)
    ws = src.view(torch.int64).view(n, words)
    le = torch.ones(n - 1, dtype=torch.bool, device=w.device)
    eq = torch.ones_like(le)
    for q in range(kw):  # least significant word first: later words decide
        a, c = _u64(w[:-1, q]), _u64(w[1:, q])
        le = (c > a) | ((c == a) & le)
        eq = eq & (c == a)
    if not bool(le.all()):
        return False
    if R == K:
        order = lexsort_order(ws, kw)
        return all(bool(torch.equal(ws[:, q].contiguous()[order], w[:, q].contiguous()))
                   for q in range(words))
    p = w[:, kw]
    if not bool(((p >= 0) & (p < n)).all()):
        return False
    seen = torch.zeros(n, dtype=torch.bool, device=w.device)
    seen[p] = True
    if not bool(seen.all()):
        return False
    if not bool((ws[p] == w).all()):
        return False
    return bool((p[1:][eq] > p[:-1][eq]).all())


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name: str, log2n: int, par_log2n: int) -> dict:
    """The oracle's stable sort timed on the host: on all the cores this
    process may use (the parallel variant, over 2^par_log2n records) and on
    one thread (over the first 2^log2n records).  `value` is the all-cores
    rate."""
    import oracle
    from paper_1703_00687_amd import workloads as wl
    cores = len(os.sched_getaffinity(0))
    n_par = 1 << par_log2n
    host, k = wl.make(name, n_par)
    oracle.sort(host[:1024], k)  # load/build outside the timing
    t0 = time.perf_counter()
    out_par, used = oracle.sort_parallel(host, k, cores)
    dt_par = time.perf_counter() - t0
    assert oracle.check_sorted(out_par[: 1 << 16], k)
    del out_par
    n1 = 1 << log2n
    t0 = time.perf_counter()
    out1 = oracle.sort(host[:n1], k)
    dt1 = time.perf_counter() - t0
    assert oracle.check_sorted(out1[: 1 << 16], k)
    model = cpu_model()
    return {"value": n_par / dt_par, "unit": "records/s", "cores": used, "kind": "oracle",
            "sample": f"first 2^{par_log2n} records of the same {name} workload: the oracle's stable "
                      f"sort in libstdc++ parallel mode on {used} threads ({dt_par:.1f} s), {model}",
            "cpu_model": model,
            "single_thread": {"value": n1 / dt1, "unit": "records/s", "cores": 1,
                              "sample": f"first 2^{log2n} records, std::stable_sort, one thread "
                                        f"({dt1:.1f} s)"}}


# The passes that move every record once (read + write of n * R bytes).
MOVE_PASSES = ["top_scatter", "round2_scatter", "lds_sort"]


def plain_ms(src, n, R, K, reps):
    """Median of `reps` plain sorts of fresh copies of src (HIP events on the
    current stream around the call only)."""
    import torch
    from paper_1703_00687_amd import binding as b
    c = torch.empty_like(src)
    tmp = torch.empty(b.raduls_tmp_bytes(n, R, K), dtype=torch.uint8, device=src.device)
    times = []
    for i in range(reps + 1):
        c.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.raduls_sort(c, tmp, n, R, K)
        e1.record()
        e1.synchronize()
        if i:
            times.append(e0.elapsed_time(e1))
    st, stats = b.raduls_check(tmp, n, R, False)
    if st != b.OK:
        raise RuntimeError(f"device error: {stats}")
    del c, tmp
    torch.cuda.empty_cache()
    return sorted(times)[len(times) // 2]


def time_sorts(src, n, R, K, steps, warm, verify, roof=None):
    """Sort `steps` resident copies of src (after `warm` untimed sorts), first
    with the library's profile events around every kernel class (the phase
    times), then -- on fresh copies -- the timed steps, with events only
    around the roofline kernel class `roof` (default: the move pass with the
    largest phase time).  The last timed step's output is verified before
    anything else touches it.  Returns (ms per step on the GPU clock, roof,
    mean duration of roof in the timed steps, phase means, device stats,
    verified)."""
    import torch
    from paper_1703_00687_amd import binding as b
    copies = []
    for _ in range(warm + steps):
        c = torch.empty_like(src)
        c.copy_(src)
        copies.append(c)
    tmp = torch.empty(b.raduls_tmp_bytes(n, R, K), dtype=torch.uint8, device=src.device)
    torch.cuda.synchronize()
    log(f"[bench] {warm + steps} resident copies of {n * R / 2**30:.2f} GiB, tmp "
        f"{tmp.numel() / 2**30:.2f} GiB")
    hip = HipEvents()
    nslot = len(PROFILE_SLOTS)
    step_events = [hip.create(2 * nslot) for _ in range(steps)]
    for i in range(warm):
        b.raduls_sort(copies[i], tmp, n, R, K)
    torch.cuda.synchronize()
    st, stats = b.raduls_check(tmp, n, R, False)
    if st != b.OK:
        raise RuntimeError(f"device error in warm-up: {stats}")
    log(f"[bench] warm-up done; stats {stats}")

    # phase times: events around each kernel class (each event recorded
    # between two kernels leaves a gap of several microseconds on the stream,
    # so these steps are not the timed ones)
    for i in range(steps):
        b.raduls_set_profile_events(step_events[i])
        b.raduls_sort(copies[warm + i], tmp, n, R, K)
    torch.cuda.synchronize()
    b.raduls_set_profile_events([])
    st, stats = b.raduls_check(tmp, n, R, False)
    if st != b.OK:
        raise RuntimeError(f"device error in the phase-timed steps: {stats}")
    phases = {}
    for j, name in enumerate(PROFILE_SLOTS):
        vals = [hip.elapsed_ms(ev[2 * j], ev[2 * j + 1]) for ev in step_events]
        phases[name] = sum(vals) / len(vals)
    if roof is None:
        roof = max(MOVE_PASSES, key=lambda k: phases[k])
    log(f"[bench] phase times {phases}; roofline kernel class: {roof}")

    # the timed steps, on fresh copies of the input, with events only around
    # the roofline kernel class
    for i in range(steps):
        copies[warm + i].copy_(src)
    jr = PROFILE_SLOTS.index(roof)
    roof_events = [[ev[k] if k // 2 == jr else None for k in range(2 * nslot)]
                   for ev in step_events]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for i in range(steps):
        b.raduls_set_profile_events(roof_events[i])
        b.raduls_sort(copies[warm + i], tmp, n, R, K)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.raduls_set_profile_events([])
    gpu_ms = start.elapsed_time(stop)
    roof_vals = [hip.elapsed_ms(ev[2 * jr], ev[2 * jr + 1]) for ev in step_events]
    roof_ms = sum(roof_vals) / len(roof_vals)
    log(f"[bench] timed {steps} steps: {gpu_ms:.2f} ms on the GPU clock, {wall * 1e3:.2f} ms wall; "
        f"{roof} {roof_ms:.4f} ms per step")
    st, stats = b.raduls_check(tmp, n, R, False)
    if st != b.OK:
        raise RuntimeError(f"device error in timed steps: {stats}")
    for ev in step_events:
        hip.destroy(ev)
    del tmp
    verified = None
    last = copies[-1]  # the last timed step's output, untouched since
    del copies
    torch.cuda.empty_cache()
    if verify:
        verified = check_sorted_device(last, src, n, R, K)
        if not verified:
            raise RuntimeError("sorted output failed the sort property check")
        log("[bench] the last timed step's output verified on the device")
    del last
    torch.cuda.empty_cache()
    return gpu_ms / steps, roof, roof_ms, phases, stats, verified


SWEEP_SHAPES = [(8, 8), (16, 8), (16, 16), (24, 8), (24, 16), (32, 8), (32, 16), (48, 8),
                (48, 16), (64, 8), (64, 16)]


def rec_sweep(log2n: int, verify: bool) -> list:
    """Records of 8-64 bytes with 8- or 16-byte keys (the paper's sweep over
    record sizes), 2^log2n records each, 1 warm-up and 3 timed sorts."""
    import torch
    from paper_1703_00687_amd import workloads as wl
    n = 1 << log2n
    out = []
    for R, K in SWEEP_SHAPES:
        log(f"[sweep] R={R} K={K} n=2^{log2n}")
        src = wl.sweep_records_torch(n, R, K)
        ms, _, _, ph, stats, ok = time_sorts(src, n, R, K, 3, 1, verify)
        del src
        torch.cuda.empty_cache()
        out.append({"rec_bytes": R, "key_bytes": K, "n": n, "ms": round(ms, 3),
                    "records_per_s": n / (ms * 1e-3),
                    "gbs_per_pass": round(2 * n * R / (ms * 1e-3) / 1e9, 1),
                    "top_scatter_gbs": round(2 * n * R / (ph["top_scatter"] * 1e-3) / 1e9, 1),
                    "rounds": stats["rounds"], "verified": ok})
        log(f"[sweep] {out[-1]}")
    return out


def fill_batch(recs, starts, sizes, seed=5):
    """Write the batch workload into one device buffer holding every array
    back to back (keys continue one stream across arrays; payload = index
    inside the array)."""
    import torch
    from paper_1703_00687_amd import workloads as wl
    total = int(sizes.sum())
    w = recs.view(torch.int64).view(total, 2)
    st = wl.stream_seed(seed, 1)
    dstarts = torch.from_numpy(starts).to(recs.device)
    chunk = 1 << 26
    for a in range(0, total, chunk):
        c = min(chunk, total - a)
        w[a:a + c, 0] = wl.splitmix64_torch(st, a, c, recs.device)
        idx = torch.arange(a, a + c, dtype=torch.int64, device=recs.device)
        arr = torch.searchsorted(dstarts, idx, right=True) - 1
        w[a:a + c, 1] = idx - dstarts[arr]


def bench_batch(args) -> dict:
    """Many uneven arrays: one batched call vs one plain call per array, and
    the same arrays served as a Poisson request stream."""
    import numpy as np
    import torch
    import oracle
    from paper_1703_00687_amd import binding as b
    from paper_1703_00687_amd import serve
    from paper_1703_00687_amd import workloads as wl

    count, R, K = args.batch_count, 16, 8
    sizes = wl.batch_sizes(count, max_log2=args.batch_log2max).astype(np.int64)
    starts = np.zeros(count, dtype=np.int64)
    starts[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    dev = torch.device("cuda:0")
    log(f"[batch] {count} arrays, sizes log-uniform in [1, 2^{args.batch_log2max}], "
        f"{total} records ({total * R / 2**30:.1f} GiB)")
    recs = torch.empty((total, R), dtype=torch.uint8, device=dev)
    tmp = torch.empty((total + 64, R), dtype=torch.uint8, device=dev)
    bt = b.Batch(count, total, R, K, device=dev)
    h = bt.host_desc.numpy()
    h[:, 0] = recs.data_ptr() + starts * R
    h[:, 1] = tmp.data_ptr() + starts * R
    h[:, 2] = sizes
    bt.desc.copy_(bt.host_desc)

    def ev_time(fn):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) * 1e-3

    # batched: one call for every array
    times = []
    for rep in range(1 + args.batch_reps):
        fill_batch(recs, starts, sizes)
        t = ev_time(bt.launch)
        st, stats = bt.check()
        if st != b.OK:
            raise RuntimeError(f"batched sort: device error {stats}")
        if rep:
            times.append(t)
    t_batched = sorted(times)[len(times) // 2]
    # the same call captured once in a HIP graph and replayed (how a serving
    # loop issues it)
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        bt.launch(stream=gs)  # (kernel attributes are set outside the capture)
    gs.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        bt.launch(stream=gs)
    gtimes = []
    for rep in range(1 + args.batch_reps):
        fill_batch(recs, starts, sizes)
        t = ev_time(graph.replay)
        st, stats = bt.check()
        if st != b.OK:
            raise RuntimeError(f"batched sort (graph): device error {stats}")
        if rep:
            gtimes.append(t)
    t_graph = sorted(gtimes)[len(gtimes) // 2]
    del graph
    rng = np.random.default_rng(0)
    for j in rng.choice(count, size=min(48, count), replace=False):
        a, n = int(starts[j]), int(sizes[j])
        got = recs[a:a + n].cpu().numpy()
        if not np.array_equal(got, oracle.sort(wl.batch_array(int(j), n, a), K)):
            raise RuntimeError(f"batched sort: array {j} differs from the oracle")
    log(f"[batch] batched: {t_batched * 1e3:.1f} ms, {total / t_batched / 1e9:.2f} G records/s")

    # plain: one raduls_sort call per array, same stream, same scratch
    fill_batch(recs, starts, sizes)
    nmax = int(sizes.max())
    need = b.raduls_tmp_bytes(nmax, R, K)
    scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    lib = b.load()
    stream = torch.cuda.current_stream().cuda_stream
    base = recs.data_ptr()
    sptr = scratch.data_ptr()

    def plain():
        for j in range(count):
            st = lib.raduls_sort(base + int(starts[j]) * R, sptr, int(sizes[j]), R, K, stream)
            if st:
                raise RuntimeError(f"plain sort of array {j}: {b.strerror(st)}")

    t_plain = ev_time(plain)
    del scratch
    log(f"[batch] plain per-array calls: {t_plain * 1e3:.1f} ms, {total / t_plain / 1e9:.3f} G records/s")

    # served: Poisson arrivals at a fraction of the plain throughput, and a closed run
    out = {
        "workload": f"{count} arrays of 16 B records, sizes log-uniform in [1, 2^{args.batch_log2max}], "
                    "uint64 key uniform, uint64 payload = index",
        "arrays": count, "records": total,
        "batched_ms": round(t_batched * 1e3, 3), "batched_records_per_s": total / t_batched,
        "batched_graph_ms": round(t_graph * 1e3, 3), "batched_graph_records_per_s": total / t_graph,
        "plain_ms": round(t_plain * 1e3, 3), "plain_records_per_s": total / t_plain,
        "batched_vs_plain": t_plain / t_batched,
    }
    if args.serve_requests > 0:
        nreq = min(args.serve_requests, count)
        budget = min(args.serve_budget_gib << 30, total * R)
        be = serve.GpuBackend(R, K, n_streams=args.serve_streams, max_batch=args.serve_max_batch,
                              max_records=budget // R)
        views = [recs[int(starts[j]):int(starts[j]) + int(sizes[j])] for j in range(nreq)]
        import gc

        small_cap = b.raduls_server_max_records(R, K)

        def serve_run(rate, many=True):
            """Serve the first nreq arrays: all at t = 0 (rate None; in one
            submit_many call, or one submit per array if not `many`) or as a
            Poisson stream of `rate` requests per second from an open-loop
            client that submits every request whose arrival time has come,
            one submit each.  Latencies are also reported apart for the
            requests of at most one LDS job (small_cap records) and the
            others."""
            fill_batch(recs, starts, sizes)
            # (so the requests are submitted with ready=False)
            torch.cuda.current_stream().synchronize()
            # Python's cyclic collector would stop both the client and the
            # server thread for up to ~0.15 s at a time while tens of
            # thousands of requests are alive; a latency-sensitive client
            # turns it off while it serves
            gc.collect()
            gc.disable()
            srv = serve.Server(be, R, budget, max_slots=be.n_streams * be.max_batch).start()
            futs = []
            t0 = time.perf_counter()
            if rate is None and many:
                futs = srv.submit_many(views, ready=False)
            elif rate is None:
                for v in views:
                    futs.append(srv.submit(v, ready=False))
            else:
                sched = t0 + np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, size=nreq))
                i = 0
                while i < nreq:
                    now = time.perf_counter()
                    while i < nreq and sched[i] <= now:
                        futs.append(srv.submit(views[i], t_arrival=float(sched[i]), ready=False))
                        i += 1
                    if i < nreq:
                        wait = sched[i] - time.perf_counter()
                        if wait > 0:
                            time.sleep(wait)  # releases the GIL to the scheduler thread
            for f in futs:
                f.result(timeout=600)
            summ = srv.stop()
            gc.enable()
            summ["wall_s"] = time.perf_counter() - t0
            for name, sel in (("small", lambda n: n <= small_cap), ("large", lambda n: n > small_cap)):
                lat = sorted((f.t_done - f.t_arrival) * 1e3 for f in futs if sel(f.n))
                if lat:
                    summ[f"{name}_requests"] = len(lat)
                    summ[f"{name}_p50_ms"] = lat[len(lat) // 2]
                    summ[f"{name}_p99_ms"] = lat[min(len(lat) - 1, int(0.99 * (len(lat) - 1) + 0.5))]
            return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}

        closed = serve_run(None)
        log(f"[serve] closed: {closed}")
        out["served_closed"] = closed
        out["served_config"] = {"streams": be.n_streams, "max_batch": be.max_batch,
                                "budget_gib": budget / 2**30}
        closed1 = serve_run(None, many=False)
        log(f"[serve] closed, one submit per request: {closed1}")
        out["served_closed_per_request"] = closed1
        cap_rate = closed["requests"] / closed["span_s"]  # requests per second the server sustains
        loads = []
        for rho in args.serve_loads:
            s = serve_run(rho * cap_rate)
            s["load_vs_closed"] = rho
            s["arrival_rate_req_s"] = round(rho * cap_rate, 1)
            log(f"[serve] load {rho}: {s}")
            loads.append(s)
        out["served_load"] = loads
        rng = np.random.default_rng(1)
        for j in rng.choice(nreq, size=min(32, nreq), replace=False):
            a, n = int(starts[j]), int(sizes[j])
            if not np.array_equal(recs[a:a + n].cpu().numpy(),
                                  oracle.sort(wl.batch_array(int(j), n, a), K)):
                raise RuntimeError(f"served array {j} differs from the oracle")
    del recs, tmp, bt
    torch.cuda.empty_cache()
    return out


def bench_resident(args) -> dict:
    """Small arrays (1 to the LDS capacity records, log-uniform sizes, uniform
    keys, 16 B records) sorted by the resident server, against the two ways
    of sorting them without it: one plain call per array and one batched
    call over all of them.  Latency: one request at a time (submit, then
    wait on the host; plain: the call, then a synchronize of its stream).
    Throughput: every array submitted at once (submit_many) and waited for,
    against the batched call."""
    import numpy as np
    import torch
    import oracle
    from paper_1703_00687_amd import binding as b
    from paper_1703_00687_amd import workloads as wl

    R, K = 16, 8
    cap = b.raduls_server_max_records(R, K)
    count = args.resident_count
    rng = np.random.default_rng(11)
    sizes = np.exp(rng.uniform(0.0, np.log(cap), size=count)).astype(np.int64).clip(1, cap)
    starts = np.zeros(count, dtype=np.int64)
    starts[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    src = wl.sweep_records_torch(total, R, K, device=dev)
    recs = torch.empty_like(src)
    ptrs = (recs.data_ptr() + starts * R).astype(np.uint64)
    log(f"[resident] {count} arrays of 1..{cap} records (log-uniform), {total} records")

    def refill():
        recs.copy_(src)
        stream.synchronize()  # (a device-wide synchronize would wait for the server)

    sample = np.linspace(0, count - 1, num=min(512, count)).astype(np.int64)
    # one plain call per array, each waited for
    tmp = torch.empty(b.raduls_tmp_bytes(cap, R, K), dtype=torch.uint8, device=dev)
    refill()
    lat_plain = []
    for j in sample:
        a, n = int(starts[j]), int(sizes[j])
        t0 = time.perf_counter()
        b.raduls_sort(recs[a:a + n], tmp, n, R, K)
        stream.synchronize()
        lat_plain.append(time.perf_counter() - t0)
    # one batched call over every array
    bt = b.Batch(count, total, R, K, device=dev)
    btmp = torch.empty_like(src)
    h = bt.host_desc.numpy()
    h[:, 0] = ptrs.astype(np.int64)
    h[:, 1] = btmp.data_ptr() + starts * R
    h[:, 2] = sizes
    bt.desc.copy_(bt.host_desc)
    bms = []
    for rep in range(4):
        refill()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bt.launch()
        e1.record()
        e1.synchronize()
        if rep:
            bms.append(e0.elapsed_time(e1))
    st, stats = bt.check()
    if st != b.OK:
        raise RuntimeError(f"batched small arrays: device error {stats}")
    batched_ms = sorted(bms)[len(bms) // 2]
    del bt, btmp

    def pct(v, p):
        v = sorted(v)
        return v[min(len(v) - 1, int(round(p / 100 * (len(v) - 1))))] * 1e6

    out = {"workload": f"{count} arrays of 16 B records, sizes log-uniform in [1, {cap}], "
                       "uint64 keys uniform",
           "arrays": count, "records": total, "max_records": cap,
           "plain_latency_us": {"p50": round(pct(lat_plain, 50), 1), "p99": round(pct(lat_plain, 99), 1)},
           "batched_ms": round(batched_ms, 4),
           "batched_records_per_s": total / (batched_ms * 1e-3),
           "servers": []}
    for wgs in args.resident_wgs:
        with b.ResidentServer(R, K, slots=max(count, 1024), workgroups=wgs, idle_ms=60000) as srv:
            refill()
            lat = []
            for j in sample:
                t0 = time.perf_counter()
                t = srv.submit(int(ptrs[j]), int(sizes[j]))
                if srv.wait(t) != 0:
                    raise RuntimeError("resident server: device error")
                lat.append(time.perf_counter() - t0)
            runs = []
            for rep in range(3):
                refill()
                t0 = time.perf_counter()
                first, acc = srv.submit_many(ptrs, sizes)
                if acc != count:
                    raise RuntimeError(f"resident server accepted {acc} of {count}")
                if srv.wait_range(first, count) != 0:
                    raise RuntimeError("resident server: device error")
                runs.append(time.perf_counter() - t0)
            wall = sorted(runs)[len(runs) // 2]
            # the last run's output against the oracle, for a sample of arrays
            for j in sample[:: max(1, len(sample) // 24)]:
                a, n = int(starts[j]), int(sizes[j])
                if not np.array_equal(recs[a:a + n].cpu().numpy(),
                                      oracle.sort(src[a:a + n].cpu().numpy(), K)):
                    raise RuntimeError(f"resident server: array {j} differs from the oracle")
            r = {"workgroups": srv.workgroups,
                 "latency_us": {"p50": round(pct(lat, 50), 1), "p99": round(pct(lat, 99), 1)},
                 "closed_ms": round(wall * 1e3, 3),
                 "closed_records_per_s": total / wall, "closed_requests_per_s": count / wall,
                 "verified": True}
            log(f"[resident] {r}")
            out["servers"].append(r)
    log(f"[resident] plain latency {out['plain_latency_us']}, batched {batched_ms:.3f} ms")
    del recs, src, tmp
    return out


TINY_SIZES = [2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 1024, 4096]
# The small-array sorters compared per record layout (the GPU counterpart of
# the paper's comparison of tiny-bin sorters by record layout, Sec. 4.1):
# the wave-level bitonic network, one enumeration sort over the whole array
# in LDS, and the LDS sorter's counting pass followed by enumeration sort of
# its buckets.
TINY_METHODS = {"network": {},
                "es": {"wave_job_max": 1, "es_job_max": 256, "tiny_max": 256},
                "hybrid": {"wave_job_max": 1}}
TINY_LAYOUTS = [(8, 8), (16, 8), (32, 16), (16, 16)]


def tiny_sweep(total_log2: int, verify: bool, methods=None, layouts=None, sizes=None) -> list:
    """Many arrays of n records each (key words uniform, then the array's
    record index where there is room, then random words), 2^total_log2
    records in all, sorted by one batched call: every array is one sort job,
    so this times the small-array sorters per record, for each method and
    record layout."""
    import numpy as np
    import torch
    import oracle
    from paper_1703_00687_amd import binding as b
    from paper_1703_00687_amd import workloads as wl
    dev = torch.device("cuda:0")
    out = []
    for R, K in (layouts or TINY_LAYOUTS):
        for method, knobs in (methods or TINY_METHODS).items():
            for n in (sizes or TINY_SIZES):
                if method != "network" and n > 256:
                    continue
                count = (1 << total_log2) // n
                total = count * n
                src = wl.sweep_records_torch(total, R, K, device=dev)
                recs = torch.empty_like(src)
                tmp = torch.empty_like(src)
                prev = b.raduls_set_tuning(**knobs)
                try:
                    bt = b.Batch(count, total, R, K, device=dev)
                    h = bt.host_desc.numpy()
                    starts = np.arange(count, dtype=np.int64) * n
                    h[:, 0] = recs.data_ptr() + starts * R
                    h[:, 1] = tmp.data_ptr() + starts * R
                    h[:, 2] = n
                    bt.desc.copy_(bt.host_desc)
                    times = []
                    for rep in range(4):
                        recs.copy_(src)
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record()
                        bt.launch()
                        e1.record()
                        torch.cuda.synchronize()
                        if rep:
                            times.append(e0.elapsed_time(e1))
                    st, stats = bt.check()
                finally:
                    b.raduls_set_tuning(**prev)
                if st != b.OK:
                    raise RuntimeError(f"tiny sweep {method} R={R} n={n}: device error {stats}")
                ms = sorted(times)[len(times) // 2]
                ok = None
                if verify:
                    rng = np.random.default_rng(n)
                    ok = True
                    for j in rng.choice(count, size=min(16, count), replace=False):
                        a = int(j) * n
                        if not np.array_equal(recs[a:a + n].cpu().numpy(),
                                              oracle.sort(src[a:a + n].cpu().numpy(), K)):
                            ok = False
                    if not ok:
                        raise RuntimeError(f"tiny sweep {method} R={R} n={n}: an array differs from the oracle")
                out.append({"rec_bytes": R, "key_bytes": K, "method": method, "n": n, "arrays": count,
                            "ms": round(ms, 3), "ns_per_record": round(ms * 1e6 / total, 4),
                            "verified": ok})
                log(f"[tiny] {out[-1]}")
                del src, recs, tmp, bt
                torch.cuda.empty_cache()
    return out


WORKLOAD_DESC = {
    "uniform16": "2^{l} records of 16 B (uint64 key uniform, uint64 payload = index), key 8 B, "
                 "1-byte digits",
    "uniform8": "2^{l} records of 8 B (uint64 key uniform, no payload), key 8 B, 1-byte digits; "
                "8 MiB fits the on-package cache, so the roofline is no HBM claim",
    "zipf16": "2^{l} records of 16 B, keys Zipf(s=1.1) over 2^24 distinct uint64 values with 5% "
              "of records sharing one extra key, payload = index; key 8 B, 1-byte digits",
    "deep32": "2^{l} records of 32 B, 16 B key (low word uniform, high word uniform over "
              "0..2^20-1), payload = index + random word; key 16 B, 1-byte digits",
    "keys16": "2^{l} records of 16 B that are all key (uniform over 128 bits); key 16 B, "
              "1-byte digits",
}
DEFAULT_LOG2 = {"uniform16": 28, "uniform8": 20, "zipf16": 28, "deep32": 27, "keys16": 28}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uniform16", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--log2n", type=int, default=None,
                    help="records = 2^log2n (default: the workload's size)")
    ap.add_argument("--cpu-sample-log2", type=int, default=None,
                    help="one-thread oracle sample, 2^k records (default 25, or the whole input if smaller)")
    ap.add_argument("--cpu-par-log2", type=int, default=None,
                    help="all-cores oracle sample, 2^k records (default: the whole input up to 2^28)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", choices=["cache", "defaults"], default="cache",
                    help="cache: the autotuner's entry for this workload and shape, if any "
                         "(the library defaults are timed beside it); defaults: none")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--batch-count", type=int, default=65536)
    ap.add_argument("--batch-log2max", type=int, default=20)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=65536)
    ap.add_argument("--serve-loads", type=float, nargs="*", default=[0.25, 0.5, 0.75, 0.9],
                    help="Poisson arrival rates as fractions of the rate the server sustains "
                         "with every request present at once")
    ap.add_argument("--serve-budget-gib", type=int, default=32)
    ap.add_argument("--serve-max-batch", type=int, default=2048,
                    help="most requests the server puts in one batched launch")
    ap.add_argument("--serve-streams", type=int, default=3,
                    help="streams the server launches batches on")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched / served comparison (run only with uniform16)")
    ap.add_argument("--no-resident", action="store_true",
                    help="skip the resident-server comparison (run only with uniform16)")
    ap.add_argument("--resident-count", type=int, default=16384)
    ap.add_argument("--resident-wgs", type=int, nargs="+", default=[32, 64, 128],
                    help="workgroups of the resident server, one run each")
    ap.add_argument("--rec-sweep", action="store_true",
                    help="also sort records of 8-64 B with 8/16 B keys (2^--sweep-log2 each)")
    ap.add_argument("--sweep-log2", type=int, default=28)
    ap.add_argument("--tiny-sweep", action="store_true",
                    help="also sort many arrays of 2..4096 records (2^--tiny-log2 records per size), "
                         "by every small-array method and record layout")
    ap.add_argument("--tiny-log2", type=int, default=22)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU path is a design only, not built)", file=sys.stderr)
        return 2

    import torch
    from paper_1703_00687_amd import workloads as wl

    name = args.workload
    log2n = DEFAULT_LOG2[name] if args.log2n is None else args.log2n
    spec = wl.WORKLOADS[name]
    n, R, K = 1 << log2n, spec["rec_bytes"], spec["key_bytes"]
    steps, warm = args.steps, args.warmup
    log(f"[bench] generating {name} n=2^{log2n} on the device")
    dev = torch.device("cuda:0")
    src = wl.make_torch(name, n, device=dev)
    torch.cuda.synchronize()
    pass_bytes = 2 * n * R
    from paper_1703_00687_amd import autotune
    from paper_1703_00687_amd import binding as b
    defaults = b.raduls_get_tuning()
    tune_key, tune_entry = (None, None)
    if args.tuning == "cache":
        tune_key, tune_entry = autotune.apply(R, K, n, name)
    log(f"[bench] tuning: {tune_key or 'library defaults'}"
        + (f" {tune_entry['tuning']}" if tune_entry else ""))
    ms_per_step, roof, roof_ms, phases, stats, verified = time_sorts(
        src, n, R, K, steps, warm, not args.no_verify)
    tuning = {"source": tune_key or "library defaults"}
    if tune_entry is not None:
        # the same plain timing with the tuned setting and with the defaults
        tuned_ms = plain_ms(src, n, R, K, max(steps, 3))
        b.raduls_set_tuning(**defaults)
        default_ms = plain_ms(src, n, R, K, max(steps, 3))
        tuning.update({"knobs": tune_entry["tuning"], "changed": tune_entry.get("changed"),
                       "tuned_ms": round(tuned_ms, 4), "default_ms": round(default_ms, 4),
                       "tuned_beats_defaults": tuned_ms < default_ms})
        log(f"[bench] tuned {tuned_ms:.3f} ms, library defaults {default_ms:.3f} ms")
    b.raduls_set_tuning(**defaults)  # the other legs run the library defaults
    achieved = pass_bytes / (roof_ms * 1e-3) / 1e9
    traffic = load_traffic(name, n, R, roof)
    rw, kw = R // 8, (K + 7) // 8
    roof_kernel = {"top_scatter": f"k_scatter_carry<{rw},{kw},1>",
                   "round2_scatter": f"k_scatter_carry<{rw},{kw},0>",
                   "lds_sort": f"k_tiny<{rw},{kw}> + k_mid<{rw},{kw}>"}[roof]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": f"{roof_kernel} ({roof}, the move pass with the largest time)",
                "bytes_per_launch": pass_bytes, "mean_launch_ms": round(roof_ms, 4)}
    # every pass that moves each record once, with its fraction of the peak
    # (from the phase-timed steps)
    passes = {k: {"ms": round(phases[k], 4),
                  "gbs": round(pass_bytes / (phases[k] * 1e-3) / 1e9, 1),
                  "frac": round(pass_bytes / (phases[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
              for k in MOVE_PASSES if phases[k] > 0.05}
    phase_gbs = {
        "top_hist": n * R / (phases["top_hist"] * 1e-3) / 1e9,
        "top_scatter": pass_bytes / (phases["top_scatter"] * 1e-3) / 1e9,
        "round2_hist": n * R / (phases["round2_hist"] * 1e-3) / 1e9,
        "round2_scatter": pass_bytes / (phases["round2_scatter"] * 1e-3) / 1e9,
        "lds_sort": pass_bytes / (phases["lds_sort"] * 1e-3) / 1e9,
    }

    # for scale: the runtime's own device copy of the same n*R bytes
    dst = torch.empty_like(src)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    ce0.record()
    for _ in range(3):
        dst.copy_(src)
    ce1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * n * R / (ce0.elapsed_time(ce1) / 3 * 1e-3) / 1e9
    del dst, src
    torch.cuda.empty_cache()

    batched = None
    if not args.no_batch and name == "uniform16":
        batched = bench_batch(args)
    resident = None
    if not args.no_resident and name == "uniform16":
        resident = bench_resident(args)
    sweep = None
    if args.rec_sweep:
        sweep = rec_sweep(args.sweep_log2, not args.no_verify)
    tiny = None
    if args.tiny_sweep:
        tiny = tiny_sweep(args.tiny_log2, not args.no_verify)

    cpu = None
    if not args.no_cpu_baseline:
        clog2 = min(log2n, 25) if args.cpu_sample_log2 is None else args.cpu_sample_log2
        plog2 = min(log2n, 28) if args.cpu_par_log2 is None else args.cpu_par_log2
        log(f"[bench] CPU oracle on 2^{plog2} records of {name} (all cores), 2^{clog2} (one thread)")
        cpu = cpu_baseline(name, clog2, plog2)
        log(f"[bench] CPU oracle: {cpu}")

    line = {
        "metric": METRIC,
        "value": n / (ms_per_step * 1e-3),
        "unit": "records/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{name}: " + WORKLOAD_DESC[name].format(l=log2n),
                   "n": n, "rec_bytes": R, "key_bytes": K},
        "roofline": roofline,
        "move_passes": passes,
        "cpu_baseline": cpu,
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "phases_gbs": {k: round(v, 1) for k, v in phase_gbs.items()},
        "whole_sort_gbs_per_pass": round(pass_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "device_copy_gbs": round(copy_gbs, 1),
        "stats": stats,
        "verified": verified,
        "tuning": tuning,
        "batched": batched,
        "resident": resident,
    }
    if sweep is not None:
        line["rec_sweep"] = sweep
    if tiny is not None:
        line["tiny_sweep"] = tiny
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
