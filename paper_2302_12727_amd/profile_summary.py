"""Per-kernel duration table from a rocprofv3 kernel trace.

    python -m paper_2302_12727_amd.profile_summary <out>/run_kernel_trace.csv

groups the dispatches by kernel and grid size (so that the launches of
different workloads in one run, e.g. a 2^21-particle lattice and a 2^22-
particle clustered set, are kept apart) and prints a Markdown table of calls,
average, minimum and maximum duration, and share of the total.
"""
from __future__ import annotations

import collections
import csv
import re
import sys


def short_name(name: str) -> str:
    """Kernel name without namespaces and argument lists, templates kept."""
    name = re.sub(r"^void ", "", name)
    name = name.replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        out.append(ch)
        depth += ch == "<"
        depth -= ch == ">"
    s = "".join(out)
    if s.startswith("rocprim::"):
        s = "rocprim " + s.split("::")[-1].split("<")[0]
    return s


def summarize(path: str) -> str:
    groups = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            grid = int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)
            groups[(short_name(r["Kernel_Name"]), grid)].append(d)
    total = sum(sum(v) for v in groups.values())
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    out = ["| kernel | grid (threads) | calls | avg (us) | min (us) | max (us) | share |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for (name, grid), v in rows:
        if sum(v) < 1e-4 * total:
            continue
        out.append(f"| {name} | {grid} | {len(v)} | {sum(v) / len(v) / 1e3:.1f} | "
                   f"{min(v) / 1e3:.1f} | {max(v) / 1e3:.1f} | {100 * sum(v) / total:.2f}% |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1]))
