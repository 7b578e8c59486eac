"""Summarise rocprofv3 CSV output for the profiles/ notes.

    python -m paper_2604_14435_amd.profile_summary stats  <dir>/<name>_kernel_stats.csv
    python -m paper_2604_14435_amd.profile_summary counter <dir>/<name>_counter_collection.csv [filter]
    python -m paper_2604_14435_amd.profile_summary trace <dir>/<name>_kernel_trace.csv [filter]

`stats` prints calls and average / min / max duration per kernel.
`trace` prints the same per kernel name and launch grid, from the
per-dispatch trace (one kernel run on different problem sizes is split).
`counter` prints, per kernel name (optionally only names containing
`filter`) and launch grid size, the number of dispatches and the average
counter value per dispatch (FETCH_SIZE / WRITE_SIZE are reported by the
hardware in KiB). Grouping by grid keeps calls of one kernel on different
problem sizes apart.
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict


def stats(path: str) -> None:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print(f"{'kernel':72s} {'calls':>6s} {'avg_us':>11s} {'min_us':>11s} {'max_us':>11s} {'pct':>7s}")
    for r in rows:
        print(f"{r['Name'][:72]:72s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:11.3f} "
              f"{float(r['MinNs']) / 1e3:11.3f} {float(r['MaxNs']) / 1e3:11.3f} {float(r['Percentage']):7.2f}")


def counter(path: str, flt: str | None = None) -> None:
    rows = list(csv.DictReader(open(path)))
    name_key = "Kernel_Name" if "Kernel_Name" in rows[0] else "Name"
    acc = defaultdict(lambda: defaultdict(list))
    for r in rows:
        name = r[name_key]
        if flt and flt not in name:
            continue
        grid = int(r.get("Grid_Size", 0) or 0)
        acc[(name, grid)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    for (name, grid), ctrs in acc.items():
        for c, vals in ctrs.items():
            print(f"{name[:64]:64s} grid={grid:<10d} {c:11s} dispatches={len(vals):4d} "
                  f"avg_per_dispatch={sum(vals) / len(vals):13.1f}")


def trace(path: str, flt: str | None = None) -> None:
    rows = list(csv.DictReader(open(path)))
    acc = defaultdict(list)
    for r in rows:
        name = r["Kernel_Name"]
        if flt and flt not in name:
            continue
        grid = "x".join(r.get(k, "1") for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"))
        acc[(name, grid)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print(f"{'kernel':64s} {'grid':>18s} {'calls':>6s} {'avg_us':>11s} {'min_us':>11s} {'max_us':>11s}")
    for (name, grid), v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        print(f"{name[:64]:64s} {grid:>18s} {len(v):6d} {sum(v) / len(v):11.3f} {min(v):11.3f} {max(v):11.3f}")


def main() -> None:
    if len(sys.argv) < 3:
        print(__doc__)
        sys.exit(2)
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else None)
    else:
        counter(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else None)


if __name__ == "__main__":
    main()
