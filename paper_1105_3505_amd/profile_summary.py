"""Summarises rocprofv3 output as markdown tables.

Usage:
  python paper_1105_3505_amd/profile_summary.py trace <results.db> [title] [command]
  python paper_1105_3505_amd/profile_summary.py counters <results.db> [title] [command]
  python paper_1105_3505_amd/profile_summary.py traffic <fetch results.db> <write results.db> <out.json>

``trace`` gives calls, average and total duration per kernel; ``counters`` gives the average
value per dispatch of every collected counter, per kernel.  ``traffic`` turns a FETCH_SIZE
run and a WRITE_SIZE run into HBM bytes per dispatch for every kernel, each counter scaled by
what it reads for a plain device copy of known size in the same run (the copy's source and
destination are 1 GiB: the run must start with ``bench.py --copy-probe-mib 1024``), and
records the hash of the kernel sources the numbers belong to.
"""
from __future__ import annotations

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
    con = sqlite3.connect(path)
    for name, start, end in con.execute("select name, start, end from kernels"):
        acc[_short(name)][0] += 1
        acc[_short(name)][1] += end - start
    tot = sum(v[1] for v in acc.values()) or 1.0
    rows = [(k, c, t / c / 1e3, t / 1e6, 100.0 * t / tot) for k, (c, t) in acc.items()]
    return sorted(rows, key=lambda r: -r[3])


def _counter_rows(path: str):
    """(kernel name, dispatch id, counter, value) of a rocprofv3 database."""
    con = sqlite3.connect(path)
    return con.execute("select kernel_name, dispatch_id, counter_name, value from counters_collection").fetchall()


def counter_table(path: str):
    """{kernel: {counter: (dispatches, average value per dispatch)}}."""
    per = defaultdict(float)
    for name, disp, cname, value in _counter_rows(path):
        per[(_short(name), disp, cname)] += float(value)   # rows of one dispatch add up
    acc = defaultdict(lambda: defaultdict(lambda: [0, 0.0]))
    for (name, _, cname), v in per.items():
        a = acc[name][cname]
        a[0] += 1
        a[1] += v
    return {k: {c: (n, s / n) for c, (n, s) in v.items()} for k, v in acc.items()}


COPY_BYTES = 1 << 30


def _copy_reference(path: str, counter: str) -> float:
    """Counter value (KiB) of the largest device copy in the run (the 1-GiB probe)."""
    best = 0.0
    for name, _, cname, value in _counter_rows(path):
        if cname == counter and "copyBuffer" in name:
            best = max(best, float(value))
    if best <= 0:
        raise SystemExit("no copy probe found in %s" % path)
    return best


KERNEL_SOURCES = ("kernels.h", "forest_kernels.hip", "fmm_kernels.hip")


def kernel_sources_hash() -> str:
    """Hash of the device code (kernels and the layouts they read), not of host orchestration."""
    import hashlib
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic(fetch_db: str, write_db: str) -> dict:
    """HBM bytes per dispatch for every kernel of the two runs."""
    f_scale = COPY_BYTES / 1024.0 / _copy_reference(fetch_db, "FETCH_SIZE")
    w_scale = COPY_BYTES / 1024.0 / _copy_reference(write_db, "WRITE_SIZE")
    fetch, write = counter_table(fetch_db), counter_table(write_db)
    out = {}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("k_"):
            continue
        fk = fetch.get(k, {}).get("FETCH_SIZE", (0, 0.0))[1]
        wk = write.get(k, {}).get("WRITE_SIZE", (0, 0.0))[1]
        out[k] = {"fetch_bytes": fk * 1024.0 * f_scale, "write_bytes": wk * 1024.0 * w_scale,
                  "bytes": (fk * f_scale + wk * w_scale) * 1024.0}
    return {"fetch_scale": f_scale, "write_scale": w_scale, "sources_sha256": kernel_sources_hash(),
            "per_dispatch": out}


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
    mode = sys.argv[1]
    if mode == "traffic":
        import json
        with open(sys.argv[4], "w") as fh:
            json.dump(traffic(sys.argv[2], sys.argv[3]), fh, indent=1, sort_keys=True)
            fh.write("\n")
    elif mode == "trace":
        print(markdown_trace(sys.argv[2], *sys.argv[3:5]))
    else:
        print(markdown_counters(sys.argv[2], *sys.argv[3:5]))
