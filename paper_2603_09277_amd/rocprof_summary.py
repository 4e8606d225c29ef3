#!/usr/bin/env python3
"""Summaries of rocprofv3 CSV output for the profiles/ folder.

  stats    kernel_stats.csv (from --kernel-trace --stats --output-format csv)
           -> a Markdown table of per-kernel calls and durations.
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
        lines = [f"# {a.title}", "", "Command (from the repository root's parent working directory /tmp):", "",
                 "```", a.command, "```", ""]
        if a.note:
            lines += [a.note, ""]
        lines += stats_table(a.csv, per=a.per)
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
