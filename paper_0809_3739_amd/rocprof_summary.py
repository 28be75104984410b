"""Short text summaries of rocprofv3 output (kernel statistics, HBM traffic).

    python -m paper_0809_3739_amd.rocprof_summary stats <kernel_stats.csv> <out.md> "<command>" "<title>"
    python -m paper_0809_3739_amd.rocprof_summary traffic <fetch counter_collection.csv> \
        <write counter_collection.csv> <out.txt> "<fetch command>" "<write command>" \
        <kernel substring> <copy kernel substring> <copy bytes per dispatch (each way)>
    python -m paper_0809_3739_amd.rocprof_summary mfma <counter_collection.csv> <kernel_trace.csv> <out.md> \
        "<command>" "<title>"

MFMA: per kernel, the mean over dispatches of SQ_INSTS_VALU_MFMA_MOPS_F32 / _F64
(flops / 512, so flops = 512 x count); the achieved MFMA rate = flops over the
dispatch's duration from the kernel trace of the same run, and its fraction of
the dense peak of the operand type.  SQ_VALU_MFMA_BUSY_CYCLES is not used: on
MI355X it reads as round multiples of 2^18 (2^30, 2^31 for millisecond kernels),
not a cycle count.

Traffic: rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE report KiB per dispatch
(summed over the L2 channels).  Both are scaled by the factor that makes the
same counter read the known size of a plain copy kernel (one read and one
write of ``copy bytes``) launched in the same run; the summary records the
factor, the scaled bytes per launch of the kernel and a hash of the
propagation kernels' sources, so that a later change of those sources voids
the figure.
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
PROP_SOURCES = ["csrc/prop.hip", "csrc/prop.hpp", "csrc/fft.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in PROP_SOURCES:
        with open(os.path.join(_HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stats(src: str, out: str, command: str, title: str) -> None:
    rows = list(csv.DictReader(open(src)))
    lines = [f"# rocprofv3 kernel statistics: {title}", "", "Command (from the repository root, one MI355X):", "",
             "```", command, "```", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | total (ms) | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("void ", "").split("(")[0].strip() or r["Name"][:50]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(path: str, counter: str, substring: str) -> list:
    vals = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter or substring not in r.get("Kernel_Name", ""):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def traffic(fetch_csv: str, write_csv: str, out: str, cmd_fetch: str, cmd_write: str, kernel: str, copy: str,
            copy_bytes: float) -> dict:
    res = {}
    for label, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        cal = _per_dispatch(path, counter, copy)
        ker = _per_dispatch(path, counter, kernel)
        if not cal or not ker:
            raise SystemExit(f"{counter}: no dispatches of '{copy}' or '{kernel}' in {path}")
        cal_kib = sum(cal) / len(cal)
        factor = copy_bytes / (cal_kib * 1024.0)
        res[label] = {"dispatches": len(ker), "raw_kib": sum(ker) / len(ker), "copy_raw_kib": cal_kib,
                      "factor": factor, "bytes_per_launch": sum(ker) / len(ker) * 1024.0 * factor}
    total = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    lines = [f"# HBM traffic of {kernel} (rocprofv3 --pmc, scaled by a plain copy kernel)", "",
             "FETCH_SIZE command:", "", "    " + cmd_fetch, "", "WRITE_SIZE command:", "", "    " + cmd_write, "",
             f"calibration kernel: {copy} (reads and writes {copy_bytes:.0f} bytes per dispatch)", ""]
    for label in ("fetch", "write"):
        r = res[label]
        lines.append(f"{label}: {r['dispatches']} dispatches, raw {r['raw_kib']:.1f} KiB/dispatch, copy kernel raw "
                     f"{r['copy_raw_kib']:.1f} KiB -> factor {r['factor']:.4f}, "
                     f"{r['bytes_per_launch'] / 1e6:.3f} MB per launch")
    lines += ["", f"bytes_per_launch: {total:.0f}", f"source_hash: {kernel_source_hash()}", ""]
    with open(out, "w") as f:
        f.write("\n".join(lines))
    return res


def read_traffic(path: str) -> float | None:
    """Scaled bytes per launch from a traffic summary, or None when the
    propagation sources changed since it was taken (or it is missing)."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash() or "bytes_per_launch" not in vals:
        return None
    return float(vals["bytes_per_launch"])


def mfma(counters_csv: str, trace_csv: str, out: str, command: str, title: str) -> None:
    per = {}
    for r in csv.DictReader(open(counters_csv)):
        k = r.get("Kernel_Name", "")
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per.setdefault(k, {}).setdefault(d, {})
        c = r.get("Counter_Name")
        per[k][d][c] = per[k][d].get(c, 0.0) + float(r["Counter_Value"])
    dur = {}
    for r in csv.DictReader(open(trace_csv)):
        k = r.get("Kernel_Name", "")
        ns = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        dur.setdefault(k, []).append(ns)
    lines = [f"# rocprofv3 MFMA counters: {title}", "", "Command (from the repository root, one MI355X):", "",
             "```", command, "```", "",
             "| kernel | dispatches | avg us | MFMA F32 GFLOP | MFMA F64 GFLOP | achieved TFLOP/s | % of peak |",
             "|---|---|---|---|---|---|---|"]
    rows = []
    for k, ds in per.items():
        vals = list(ds.values())
        mean = lambda c: sum(v.get(c, 0.0) for v in vals) / len(vals)   # noqa: E731
        f32 = mean("SQ_INSTS_VALU_MFMA_MOPS_F32") * 512
        f64 = mean("SQ_INSTS_VALU_MFMA_MOPS_F64") * 512
        if f32 + f64 <= 0:
            continue
        t = dur.get(k, [])
        avg_us = sum(t) / len(t) / 1e3 if t else float("nan")
        rate = (f32 + f64) / (avg_us * 1e-6) / 1e12 if t else float("nan")
        util = 100.0 * rate / (157.3 * f32 / (f32 + f64) + 78.6 * f64 / (f32 + f64))
        name = k.replace("void ", "").split("(")[0].strip()
        rows.append((f32 + f64, f"| `{name}` | {len(vals)} | {avg_us:.1f} | {f32 / 1e9:.2f} | {f64 / 1e9:.2f} | "
                                f"{rate:.1f} | {util:.1f} |"))
    lines += [r for _, r in sorted(rows, reverse=True)]
    lines += ["", "Peaks (dense, MI355X spec): float32 MFMA 157.3 TFLOP/s, float64 MFMA 78.6 TFLOP/s."]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "stats" and len(a) == 5:
        stats(*a[1:])
    elif a and a[0] == "traffic" and len(a) == 9:
        traffic(a[1], a[2], a[3], a[4], a[5], a[6], a[7], float(a[8]))
    elif a and a[0] == "mfma" and len(a) == 6:
        mfma(*a[1:])
    else:
        print(__doc__)
        sys.exit(2)
