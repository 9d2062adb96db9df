"""Summarise a rocprofv3 kernel trace (CSV) per kernel and launch size.

rocprofv3's --stats table aggregates by kernel name only; one kernel name here
serves several lattice levels, so this groups the dispatches of
``<prefix>_kernel_trace.csv`` by (kernel, grid size) and prints, as Markdown, the
call count, total and average duration of each group (largest total first).

With --counters the input is a rocprofv3 ``<prefix>_counter_collection.csv``
(--pmc runs): per (kernel, grid, counter) the call count and mean counter value.

With --after-gap S only the dispatches after the last idle gap longer than S
seconds are kept (a program that pauses between its setup and a timed region
gives the timed region alone); the summary then also reports the wall span of
those dispatches and the time the device had at least one of them running.

Usage: python profsum.py TRACE.csv [--top N] [--match SUBSTR] [--counters]
       [--after-gap S]
"""

from __future__ import annotations

import argparse
import csv
import re
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    name = re.sub(r"smg::\(anonymous namespace\)::", "", name)
    name = re.sub(r"smg::cpx<(double|float)>", r"z\1", name)
    return name.split("(")[0] if "(" in name else name


def after_gap(rows, gap_s: float):
    """Rows whose dispatch starts after the last idle gap longer than gap_s seconds."""
    ev = sorted(rows, key=lambda r: float(r["Start_Timestamp"]))
    cut, last_end = None, None
    for r in ev:
        st = float(r["Start_Timestamp"])
        if last_end is not None and st - last_end > gap_s * 1e9:
            cut = st
        en = float(r["End_Timestamp"])
        last_end = en if last_end is None else max(last_end, en)
    return [r for r in ev if cut is None or float(r["Start_Timestamp"]) >= cut]


def busy_ns(rows) -> tuple:
    """(wall span, union of the dispatch intervals) in ns."""
    iv = sorted((float(r["Start_Timestamp"]), float(r["End_Timestamp"])) for r in rows)
    if not iv:
        return 0.0, 0.0
    busy, cs, ce = 0.0, iv[0][0], iv[0][1]
    for s_, e_ in iv[1:]:
        if s_ > ce:
            busy += ce - cs
            cs, ce = s_, e_
        else:
            ce = max(ce, e_)
    busy += ce - cs
    return iv[-1][1] - iv[0][0], busy


def summarise(path: str, top: int = 25, match: str = "", gap: float = 0.0) -> str:
    groups = defaultdict(lambda: [0, 0.0])
    with open(path) as f:
        rows = list(csv.DictReader(f))
    if gap > 0:
        rows = after_gap(rows, gap)
    for row in rows:
        name = row.get("Kernel_Name") or row.get("Name") or ""
        if match and match not in name:
            continue
        grid = "x".join(row.get(k, "?") for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"))
        dur = float(row["End_Timestamp"]) - float(row["Start_Timestamp"])
        g = groups[(short_name(name), grid)]
        g[0] += 1
        g[1] += dur
    total = sum(v[1] for v in groups.values())
    lines = ["| kernel | grid | calls | total ms | avg us | % |", "|---|---|---|---|---|---|"]
    for (name, grid), (n, t) in sorted(groups.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"| `{name}` | {grid} | {n} | {t / 1e6:.2f} | {t / n / 1e3:.2f} | {100 * t / total:.1f} |")
    lines.append(f"\nTotal kernel time {total / 1e6:.1f} ms over {sum(v[0] for v in groups.values())} dispatches.")
    if gap > 0:
        span, busy = busy_ns(rows)
        lines.append(f"Wall span {span / 1e6:.1f} ms; device busy (union of dispatch intervals) {busy / 1e6:.1f} ms.")
    return "\n".join(lines)


def summarise_counters(path: str, top: int = 25, match: str = "") -> str:
    groups = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name", "")
            if match and match not in name:
                continue
            key = (short_name(name), row.get("Grid_Size", "?"), row.get("Counter_Name", "?"))
            groups[key].append(float(row["Counter_Value"]))
    lines = ["| kernel | grid | counter | calls | mean value |", "|---|---|---|---|---|"]
    for (name, grid, ctr), vals in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"| `{name}` | {grid} | {ctr} | {len(vals)} | {sum(vals) / len(vals):.1f} |")
    return "\n".join(lines)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--match", default="")
    ap.add_argument("--counters", action="store_true")
    ap.add_argument("--after-gap", type=float, default=0.0)
    a = ap.parse_args(argv)
    if a.counters:
        print(summarise_counters(a.trace, a.top, a.match))
    else:
        print(summarise(a.trace, a.top, a.match, a.after_gap))
    return 0


if __name__ == "__main__":
    sys.exit(main())
