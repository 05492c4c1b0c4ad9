"""Summarise a rocprofv3 kernel trace as short text.

rocprofv3 --kernel-trace --output-format csv writes one row per dispatch.
A kernel of this library runs at several levels of the hierarchy with the
same name, so a per-name average mixes levels; this summary groups the
dispatches by (kernel name, grid size) as well, which separates the levels
(the grid of a fused grid kernel is tiles x 256 work-items).

With --counters it summarises a rocprofv3 --pmc run instead (counter_collection.csv):
the mean of every counter per (kernel name, grid size), over the dispatches whose
name contains --match.

Usage: python -m paper_2010_00626_amd.profsum <rocprofv3 output dir> [--top 25] [--match SUBSTR] [--counters]
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import sys
from collections import defaultdict


def _rows(path: str):
    with open(path, newline="") as fh:
        yield from csv.DictReader(fh)


def _short(name: str, width: int = 70) -> str:
    name = name.replace("void ", "").replace("(StageArgs)", "").replace("(SubArgs)", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def summarise(root: str, top: int = 25, match: str | None = None) -> str:
    traces = sorted(glob.glob(os.path.join(root, "**", "*kernel_trace.csv"), recursive=True))
    if not traces:
        raise SystemExit(f"no *kernel_trace.csv under {root}")
    by_name = defaultdict(list)
    by_grid = defaultdict(list)
    for path in traces:
        for r in _rows(path):
            name = r.get("Kernel_Name", "?")
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            grid = int(r.get("Grid_Size_X", r.get("Grid_Size", 0)) or 0) * int(r.get("Grid_Size_Y", 1) or 1) * \
                int(r.get("Grid_Size_Z", 1) or 1)
            by_name[name].append(dur)
            by_grid[(name, grid)].append(dur)
    total = sum(sum(v) for v in by_name.values())
    out = [f"# dispatches: {sum(len(v) for v in by_name.values())}, kernel time {total / 1e6:.3f} ms",
           "", "## by kernel (sorted by total time)",
           f"{'kernel':70s} {'calls':>8s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for name, v in sorted(by_name.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append(f"{_short(name):70s} {len(v):8d} {sum(v) / 1e6:10.3f} {sum(v) / len(v) / 1e3:9.2f} "
                   f"{min(v) / 1e3:8.2f} {max(v) / 1e3:8.2f} {100.0 * sum(v) / total:6.2f}")
    out += ["", "## by kernel and grid size (work-items)",
            f"{'kernel':70s} {'grid':>9s} {'calls':>8s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s}"]
    items = sorted(by_grid.items(), key=lambda kv: -sum(kv[1]))
    if match:
        items = [kv for kv in items if match in kv[0][0]]
    for (name, grid), v in items[: top * 2]:
        out.append(f"{_short(name):70s} {grid:9d} {len(v):8d} {sum(v) / 1e6:10.3f} {sum(v) / len(v) / 1e3:9.2f} "
                   f"{min(v) / 1e3:8.2f} {max(v) / 1e3:8.2f}")
    return "\n".join(out) + "\n"


def summarise_counters(root: str, match: str | None = None) -> str:
    files = sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {root}")
    vals = defaultdict(lambda: defaultdict(list))
    names = []
    for path in files:
        for r in _rows(path):
            kern = r.get("Kernel_Name", "?")
            if match and match not in kern:
                continue
            grid = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)) or 0)
            c = r["Counter_Name"]
            if c not in names:
                names.append(c)
            vals[(kern, grid)][c].append(float(r["Counter_Value"]))
    out = [f"{'kernel':44s} {'grid':>9s} {'dispatches':>10s} " + " ".join(f"{c:>16s}" for c in names)]
    for (kern, grid), d in sorted(vals.items()):
        n = max(len(v) for v in d.values())
        cells = " ".join(f"{sum(d[c]) / len(d[c]):16.1f}" if d.get(c) else f"{'-':>16s}" for c in names)
        out.append(f"{_short(kern, 44):44s} {grid:9d} {n:10d} {cells}")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("root")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--match", default=None)
    ap.add_argument("--counters", action="store_true", help="summarise a --pmc run (mean per kernel and grid)")
    a = ap.parse_args(argv)
    if a.counters:
        sys.stdout.write(summarise_counters(a.root, a.match))
    else:
        sys.stdout.write(summarise(a.root, a.top, a.match))


if __name__ == "__main__":
    main()
