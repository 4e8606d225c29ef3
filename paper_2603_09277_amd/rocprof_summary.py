#!/usr/bin/env python3
"""Summaries of rocprofv3 CSV output for the profiles/ folder.

  stats    kernel_stats.csv (from --kernel-trace --stats --output-format csv)
           -> a Markdown table of per-kernel calls and durations.
  counters counter_collection.csv files of SQ counter runs plus the
           kernel_stats.csv of a --kernel-trace --stats run of the same
           program -> per-dispatch averages of every counter for the chosen
           kernels and the derived VALU / LDS figures (lane utilisation,
           executed lane-operations per second against the VALU peak, LDS
           bank conflicts per access).
  traffic  counter_collection.csv of a FETCH_SIZE run and of a WRITE_SIZE run
           of the same program, plus the same two counters read on a plain
           copy of known size -> per-launch HBM bytes of one kernel, scaled by
           the copy's calibration factors, as Markdown and as the JSON record
           that bench.py reads (it ignores the record once the kernel's source
           file no longer has the recorded hash).

Counters are in KiB per dispatch.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def short_name(name: str) -> str:
    name = name.replace("gsr::(anonymous namespace)::", "").replace("void ", "")
    name = re.sub(r"\(.*\)$", "", name)
    return name.strip()


def stats_rows(path: str):
    """Per-kernel (name, calls, total, avg, min, max ns, share %) from kernel_stats.csv or a rocpd database."""
    if path.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(path)
        q = ("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
             "from kernels group by name")
        raw = con.execute(q).fetchall()
        tot = sum(r[2] for r in raw) or 1
        rows = [(n, c, t, a, lo, hi, 100.0 * t / tot) for n, c, t, a, lo, hi in raw]
    else:
        rows = [(r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]), float(r["MinNs"]),
                 float(r["MaxNs"]), float(r["Percentage"])) for r in csv.DictReader(open(path))]
    rows.sort(key=lambda r: -r[2])
    return rows


def stats_table(path: str, top: int = 40, per: int = 0):
    extra = f" | ms per step ({per} steps) " if per else " "
    out = [f"| kernel | calls | avg us | min us | max us | share %{extra}|",
           "|---|---:|---:|---:|---:|---:|" + ("---:|" if per else "")]
    for n, c, t, a, lo, hi, sh in stats_rows(path)[:top]:
        col = f" {t / per / 1e6:.4f} |" if per else ""
        out.append(f"| `{short_name(n)}` | {c} | {a / 1e3:.2f} | {lo / 1e3:.2f} | {hi / 1e3:.2f} | {sh:.2f} |{col}")
    return out


def counter_by_kernel(path: str, counter: str):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            d[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return d


def pick(d, pattern):
    keys = [k for k in d if re.search(pattern, k)]
    if len(keys) != 1:
        raise SystemExit(f"pattern {pattern!r} matches {keys}")
    return keys[0], d[keys[0]]


# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one FP32 lane-operation per lane per clock
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9


def all_counters(paths):
    """{kernel: {counter: [per-dispatch values]}} over several counter_collection.csv files."""
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        for r in csv.DictReader(open(path)):
            d[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return d


def counters_table(paths, stats_path, patterns):
    cnt = all_counters(paths)
    dur = {short_name(n): a for n, c, t, a, lo, hi, sh in stats_rows(stats_path)}
    out = []
    for pat in patterns:
        k, c = pick(cnt, pat)
        avg = {n: sum(v) / len(v) for n, v in c.items()}
        out += [f"## `{k}`", "", "| counter | per dispatch |", "|---|---:|"]
        out += [f"| {n} | {v:,.0f} |" for n, v in sorted(avg.items())]
        waves = avg.get("SQ_WAVES")
        d_ns = next((v for n, v in dur.items() if n == k), None)
        out += ["", "| derived | value |", "|---|---:|"]
        if d_ns:
            out.append(f"| average duration (kernel trace) | {d_ns / 1e3:.2f} us |")
        if waves:
            for n in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD"):
                if n in avg:
                    out.append(f"| {n} per wave | {avg[n] / waves:,.1f} |")
        if "SQ_THREAD_CYCLES_VALU" in avg and avg.get("SQ_ACTIVE_INST_VALU"):
            out.append(f"| VALU lane utilisation (active lanes / 64) | "
                       f"{avg['SQ_THREAD_CYCLES_VALU'] / (avg['SQ_ACTIVE_INST_VALU'] * 64):.3f} |")
        if "SQ_INSTS_VALU" in avg and d_ns:
            rate = avg["SQ_INSTS_VALU"] * 64 / (d_ns * 1e-9)
            out.append(f"| issued VALU lane-slots / s | {rate / 1e12:.2f} T ({rate / VALU_LANE_OPS_PEAK:.3f} of "
                       f"{VALU_LANE_OPS_PEAK / 1e12:.2f} T) |")
        if "SQ_LDS_BANK_CONFLICT" in avg and "SQ_LDS_IDX_ACTIVE" in avg:
            acc = avg["SQ_LDS_IDX_ACTIVE"] - avg["SQ_LDS_BANK_CONFLICT"]
            if acc > 0:
                out.append(f"| LDS bank conflicts per access (cycles) | {avg['SQ_LDS_BANK_CONFLICT'] / acc:.4f} |")
        out.append("")
    return out


def source_hash(name):
    with open(os.path.join(CSRC, name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv", help="kernel_stats.csv, or the rocpd *_results.db of a --kernel-trace run")
    s.add_argument("--per", type=int, default=0, help="also give total ms divided by this many steps")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--csv", nargs="+", required=True, help="counter_collection.csv files")
    c.add_argument("--stats", required=True, help="kernel_stats.csv (or rocpd .db) of the same program")
    c.add_argument("--kernel", nargs="+", required=True, help="regexes of the kernel names")
    c.add_argument("--title", required=True)
    c.add_argument("--commands", required=True, help="the rocprofv3 commands, separated by ' ;; '")
    c.add_argument("--note", default="")
    c.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--calib-fetch", required=True)
    t.add_argument("--calib-write", required=True)
    t.add_argument("--calib-kernel", default="copyBuffer")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--kernel", required=True, help="regex of the kernel name")
    t.add_argument("--source", required=True, help="source file under csrc/ that holds the kernel")
    t.add_argument("--algorithmic-bytes", type=float, default=None)
    t.add_argument("--title", required=True)
    t.add_argument("--commands", required=True, help="the rocprofv3 commands, separated by ' ;; '")
    t.add_argument("--out-md", required=True)
    t.add_argument("--out-json", required=True)
    a = ap.parse_args()

    if a.cmd == "stats":
        lines = [f"# {a.title}", "", "Command:", "",
                 "```", a.command, "```", ""]
        if a.note:
            lines += [a.note, ""]
        lines += stats_table(a.csv, per=a.per)
        open(a.out, "w").write("\n".join(lines) + "\n")
        return

    if a.cmd == "counters":
        lines = [f"# {a.title}", "", "Commands (run from /tmp):", "", "```"] + a.commands.split(" ;; ") + ["```", ""]
        if a.note:
            lines += [a.note, ""]
        lines += counters_table(a.csv, a.stats, a.kernel)
        open(a.out, "w").write("\n".join(lines) + "\n")
        return

    kib = 1024.0
    fk, fetch = pick(counter_by_kernel(a.fetch, "FETCH_SIZE"), a.kernel)
    wk, write = pick(counter_by_kernel(a.write, "WRITE_SIZE"), a.kernel)
    _, cf = pick(counter_by_kernel(a.calib_fetch, "FETCH_SIZE"), a.calib_kernel)
    _, cw = pick(counter_by_kernel(a.calib_write, "WRITE_SIZE"), a.calib_kernel)
    f_fac = a.copy_bytes / (max(cf) * kib)
    w_fac = a.copy_bytes / (max(cw) * kib)
    fetch_b = sum(fetch) / len(fetch) * kib * f_fac
    write_b = sum(write) / len(write) * kib * w_fac
    rec = {"kernel": fk, "source": a.source, "source_sha256_16": source_hash(a.source),
           "fetch_bytes": round(fetch_b), "write_bytes": round(write_b), "bytes_per_launch": round(fetch_b + write_b),
           "dispatches": [len(fetch), len(write)], "fetch_factor": round(f_fac, 4), "write_factor": round(w_fac, 4)}
    json.dump(rec, open(a.out_json, "w"), indent=1)
    lines = [f"# {a.title}", "", "Commands (run from /tmp):", "", "```"] + a.commands.split(" ;; ") + ["```", "",
             f"Kernel: `{fk}` ({len(fetch)} / {len(write)} dispatches averaged).", "",
             f"Calibration: a plain {a.copy_bytes / 2**20:.0f} MiB device copy reads FETCH_SIZE "
             f"{max(cf):.0f} KiB and WRITE_SIZE {max(cw):.0f} KiB, so FETCH_SIZE is scaled by {f_fac:.4f} "
             f"and WRITE_SIZE by {w_fac:.4f}.", "",
             "| quantity | per launch |", "|---|---:|",
             f"| FETCH_SIZE raw | {sum(fetch) / len(fetch) / 1024:.2f} MiB |",
             f"| WRITE_SIZE raw | {sum(write) / len(write) / 1024:.2f} MiB |",
             f"| HBM read (scaled) | {fetch_b / 2**20:.2f} MiB |",
             f"| HBM write (scaled) | {write_b / 2**20:.2f} MiB |",
             f"| total traffic | {(fetch_b + write_b) / 2**20:.2f} MiB |"]
    if a.algorithmic_bytes:
        lines.append(f"| algorithmic bytes | {a.algorithmic_bytes / 2**20:.2f} MiB |")
        lines.append(f"| traffic / algorithmic | {(fetch_b + write_b) / a.algorithmic_bytes:.2f} |")
    lines += ["", f"Source hash of `{a.source}` when counted: {rec['source_sha256_16']}."]
    open(a.out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
