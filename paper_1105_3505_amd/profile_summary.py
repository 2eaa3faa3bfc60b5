"""Summarises a rocprofv3 kernel-trace database (``*_results.db``) as a markdown table.

Usage: python paper_1105_3505_amd/profile_summary.py <results.db> [title] [command]
"""
from __future__ import annotations

import re
import sqlite3
import sys


def kernel_table(db_path: str):
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, count(*), avg(end-start), sum(end-start) from kernels "
                       "group by name order by sum(end-start) desc").fetchall()
    tot = sum(r[3] for r in rows) or 1
    out = []
    for name, cnt, avg, total in rows:
        m = re.search(r"(k_\w+(?:<[^>]*>)?)", name)
        short = m.group(1) if m else name.split("(")[0]
        out.append((short, cnt, avg / 1e3, total / 1e6, 100.0 * total / tot))
    return out


def markdown(db_path: str, title: str = "", command: str = "") -> str:
    lines = []
    if title:
        lines += ["# " + title, ""]
    if command:
        lines += ["Command (GPU box, repo root):", "", "```", command, "```", ""]
    lines += ["| kernel | calls | avg us | total ms | share |", "|---|---|---|---|---|"]
    for short, cnt, avg, total, share in kernel_table(db_path):
        lines.append(f"| `{short}` | {cnt} | {avg:.1f} | {total:.3f} | {share:.1f}% |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    print(markdown(sys.argv[1], *(sys.argv[2:4])))
