"""Summaries of rocprofv3 CSV output for the profiles/ directory.

``trace``: turns ``*_kernel_stats.csv`` (from ``--kernel-trace --stats
--output-format csv``) into a short table of per-kernel calls and durations.

``sq``: turns a ``*_counter_collection.csv`` of SQ counters into per-kernel
instruction counts and per-CU times.

``traffic``: turns two ``*_counter_collection.csv`` files (``--pmc
FETCH_SIZE`` and ``--pmc WRITE_SIZE`` runs of the same command) into HBM
bytes per launch of one kernel.  Each counter is scaled by what it reads for
the runtime's copy kernel of known size in the same run (the benchmark copies
its n*R-byte input with it), so the result is in true bytes.  Writes a JSON
record carrying the kernel source hash, which bench.py uses only while the
kernel source is unchanged.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("raduls_kernels.hpp", "raduls_common.hpp"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    s = (name.replace("raduls::", "").replace("(raduls::Params, unsigned int)", "")
         .replace("(raduls::Params)", "").replace("void ", ""))
    return s if len(s) <= 72 else s[:69] + "..."


def trace(stats_csv: str, command: str, out: str) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "Every kernel of the library and the runtime's copy kernel; torch's own kernels "
             "(input generation, restores, the output check) are left out.", "",
             "| kernel | calls | mean us | min us | max us | total us | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        if "raduls::" not in r["Name"] and COPY_KERNEL not in r["Name"]:
            continue
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_kernel(path: str, counter: str) -> dict:
    vals: dict = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, n: int, rec_bytes: int,
            command: str, out_json: str, out_md: str) -> dict:
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")
    big_copy_f = [v for v in f.get(COPY_KERNEL, []) if v * 1024 > copy_bytes / 8]
    big_copy_w = [v for v in w.get(COPY_KERNEL, []) if v * 1024 > copy_bytes / 8]
    f_scale = copy_bytes / (statistics.mean(big_copy_f) * 1024)
    w_scale = copy_bytes / (statistics.mean(big_copy_w) * 1024)
    kf = statistics.mean(f[kernel]) * 1024 * f_scale
    kw = statistics.mean(w[kernel]) * 1024 * w_scale
    rec = {"kernel": kernel, "n": n, "rec_bytes": rec_bytes, "kernel_source_hash": kernel_source_hash(),
           "fetch_bytes_per_launch": kf, "write_bytes_per_launch": kw,
           "hbm_bytes_per_launch": kf + kw, "fetch_scale": f_scale, "write_scale": w_scale,
           "calibration": f"{COPY_KERNEL} of {copy_bytes} bytes", "command": command}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = [f"# HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
             f"Command (once with `--pmc FETCH_SIZE`, once with `--pmc WRITE_SIZE`): `{command}`", "",
             f"Calibration: {COPY_KERNEL} copying {copy_bytes} bytes reads FETCH_SIZE x{f_scale:.3f}, "
             f"WRITE_SIZE x{w_scale:.3f} of its true bytes; the same factors are applied below.", "",
             "| kernel | launches | fetch GB/launch | write GB/launch |", "|---|---|---|---|"]
    for k in sorted(set(f) | set(w)):
        fv = [v for v in f.get(k, [])]
        wv = [v for v in w.get(k, [])]
        if not fv or not wv:
            continue
        fm = max(fv) * 1024 * f_scale / 1e9
        wm = max(wv) * 1024 * w_scale / 1e9
        if fm < 1e-3 and wm < 1e-3:
            continue
        lines.append(f"| {short(k)} | {len(fv)} | {fm:.3f} (max) | {wm:.3f} (max) |")
    lines += ["", f"Dominant kernel `{short(kernel)}`: {kf / 1e9:.3f} GB read + {kw / 1e9:.3f} GB written "
              f"per launch = {(kf + kw) / 1e9:.3f} GB (algorithmic 2nR = {2 * n * rec_bytes / 1e9:.3f} GB)."]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return rec


def sq(counter_csv: str, command: str, out: str, clock_ghz: float = 2.4, cus: int = 256) -> None:
    """SQ counters per kernel: the largest launch of each kernel (the ones
    that do the work), summed over the chip, and the per-CU time the vector
    ALUs alone need (one wave-level VALU instruction per cycle per CU)."""
    per: dict = {}
    for r in csv.DictReader(open(counter_csv)):
        d = per.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = ["# SQ counters per kernel", "", f"Command: `{command}`", "",
             "Values are the largest launch of each kernel, summed over the chip. Per CU: "
             "wave-level VALU and SALU instructions and LDS bank-conflict cycles divided by "
             f"{cus} CUs, as time at {clock_ghz} GHz (a CU issues at most one wave-level VALU "
             "and one SALU instruction per cycle).", "",
             "| kernel | VALU instr | SALU instr | LDS instr | LDS bank-conflict cycles | "
             "VALU per CU (ms) | SALU per CU (ms) | bank conflicts per CU (ms) |",
             "|---|---|---|---|---|---|---|---|"]
    for k, ds in sorted(per.items()):
        best = max(ds.values(), key=lambda v: v.get("SQ_INSTS_VALU", 0.0))
        va, sa = best.get("SQ_INSTS_VALU", 0.0), best.get("SQ_INSTS_SALU", 0.0)
        la, bc = best.get("SQ_INSTS_LDS", 0.0), best.get("SQ_LDS_BANK_CONFLICT", 0.0)
        if va < 1e6:
            continue
        ms = lambda x: x / cus / (clock_ghz * 1e6)
        lines.append(f"| {short(k)} | {va:.3g} | {sa:.3g} | {la:.3g} | {bc:.3g} | {ms(va):.2f} | "
                     f"{ms(sa):.2f} | {ms(bc):.2f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    p = sub.add_parser("traffic")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("--kernel", required=True)
    p.add_argument("--copy-bytes", type=int, required=True)
    p.add_argument("--n", type=int, required=True)
    p.add_argument("--rec-bytes", type=int, required=True)
    p.add_argument("--command", required=True)
    p.add_argument("--out-json", required=True)
    p.add_argument("--out-md", required=True)
    q = sub.add_parser("sq")
    q.add_argument("counter_csv")
    q.add_argument("--command", required=True)
    q.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.mode == "trace":
        trace(a.stats_csv, a.command, a.out)
    elif a.mode == "sq":
        sq(a.counter_csv, a.command, a.out)
    else:
        print(json.dumps(traffic(a.fetch_csv, a.write_csv, a.kernel, a.copy_bytes, a.n, a.rec_bytes,
                                 a.command, a.out_json, a.out_md)))
