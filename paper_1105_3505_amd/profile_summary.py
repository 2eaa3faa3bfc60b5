"""Summarises rocprofv3 output as markdown tables.

Usage:
  python paper_1105_3505_amd/profile_summary.py trace <results.db | kernel_trace.csv> [title] [command]
  python paper_1105_3505_amd/profile_summary.py counters <counter_collection.csv> [title] [command]

``trace`` gives calls, average and total duration per kernel; ``counters`` gives the average
value per dispatch of every collected counter, per kernel.
"""
from __future__ import annotations

import csv
import re
import sqlite3
import sys
from collections import defaultdict


def _short(name: str) -> str:
    m = re.search(r"(k_\w+(?:<[^>]*>)?)", name)
    if m:
        return m.group(1)
    return name.split("(")[0][:80]


def kernel_table(path: str):
    """(kernel, calls, avg us, total ms, share %) sorted by total time."""
    acc = defaultdict(lambda: [0, 0.0])
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        for name, start, end in con.execute("select name, start, end from kernels"):
            acc[_short(name)][0] += 1
            acc[_short(name)][1] += end - start
    else:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                name = _short(row["Kernel_Name"])
                acc[name][0] += 1
                acc[name][1] += int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
    tot = sum(v[1] for v in acc.values()) or 1.0
    rows = [(k, c, t / c / 1e3, t / 1e6, 100.0 * t / tot) for k, (c, t) in acc.items()]
    return sorted(rows, key=lambda r: -r[3])


def counter_table(path: str):
    """{kernel: {counter: (dispatches, average value per dispatch)}}."""
    acc = defaultdict(lambda: defaultdict(lambda: [0, 0.0]))
    seen = defaultdict(set)
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            name = _short(row["Kernel_Name"])
            key = (row.get("Dispatch_Id"), row["Counter_Name"])
            if key in seen[name]:
                # several rows of one dispatch (per-dimension values): sum them
                acc[name][row["Counter_Name"]][1] += float(row["Counter_Value"])
                continue
            seen[name].add(key)
            a = acc[name][row["Counter_Name"]]
            a[0] += 1
            a[1] += float(row["Counter_Value"])
    return {k: {c: (n, s / n) for c, (n, s) in v.items()} for k, v in acc.items()}


def _header(title: str, command: str):
    lines = []
    if title:
        lines += ["# " + title, ""]
    if command:
        lines += ["Command (GPU box, repo root):", "", "```", command, "```", ""]
    return lines


def markdown_trace(path: str, title: str = "", command: str = "") -> str:
    lines = _header(title, command)
    lines += ["| kernel | calls | avg us | total ms | share |", "|---|---|---|---|---|"]
    for short, cnt, avg, total, share in kernel_table(path):
        lines.append(f"| `{short}` | {cnt} | {avg:.1f} | {total:.3f} | {share:.1f}% |")
    return "\n".join(lines) + "\n"


def markdown_counters(path: str, title: str = "", command: str = "") -> str:
    lines = _header(title, command)
    table = counter_table(path)
    counters = sorted({c for v in table.values() for c in v})
    lines += ["| kernel | dispatches | " + " | ".join(counters) + " |",
              "|---|---|" + "---|" * len(counters)]
    for k in sorted(table):
        v = table[k]
        n = max(x[0] for x in v.values())
        cells = ["%.1f" % v[c][1] if c in v else "" for c in counters]
        lines.append(f"| `{k}` | {n} | " + " | ".join(cells) + " |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    rest = sys.argv[3:5]
    print(markdown_trace(path, *rest) if mode == "trace" else markdown_counters(path, *rest))
