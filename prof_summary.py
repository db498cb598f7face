"""Condense rocprofv3 CSV output into a short text summary.

    python3 prof_summary.py DIR [--match SUBSTR] [--block B --grid G] [--split-us T] [--top N] [--delete]

DIR is a rocprofv3 ``-d`` output directory written with ``--output-format csv``.
Prints the per-kernel statistics (``*kernel_stats.csv``: calls, total, average),
and, for the dispatches of the kernels whose name contains SUBSTR (optionally
only those launched with workgroup size B and B*G lanes), the dispatch count
and the average duration (``*kernel_trace.csv``) or the average value of each
hardware counter (``*counter_collection.csv``).  --split-us T also reports the
dispatches shorter and not shorter than T microseconds apart (a solver's
guarded launches that return at once against those that run).  --delete
removes the bulky per-dispatch CSV files afterwards.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import sys
from collections import defaultdict


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _get(row, *names, default=""):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    return default


def _shape_ok(row, block, grid):
    if block is None:
        return True
    wg = int(float(_get(row, "Workgroup_Size_X", "Workgroup_Size", default="0")))
    gs = int(float(_get(row, "Grid_Size_X", "Grid_Size", default="0")))
    if wg != block:
        return False
    return grid is None or gs == block * grid


def _line(label, ts):
    return (f"{label}: {len(ts)}; average {sum(ts) / len(ts) / 1e3:.2f} us; "
            f"min {min(ts) / 1e3:.2f} us; max {max(ts) / 1e3:.2f} us\n")


def summarize(d, match=None, block=None, grid=None, top=25, split_us=None, out=None):
    out = out or sys.stdout
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        rows = _rows(f)
        rows.sort(key=lambda r: -float(_get(r, "TotalDurationNs", default="0")))
        out.write(f"# {os.path.relpath(f, d)}: {len(rows)} kernels (top {top} by total time)\n")
        out.write("calls | total_ms | avg_us | pct | kernel\n")
        for r in rows[:top]:
            out.write(f"{_get(r, 'Calls')} | {float(_get(r, 'TotalDurationNs', default='0')) / 1e6:.3f} | "
                      f"{float(_get(r, 'AverageNs', default='0')) / 1e3:.2f} | {float(_get(r, 'Percentage', default='0')):.2f} | "
                      f"{_get(r, 'Name', 'KernelName')[:150]}\n")
    if match:
        for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
            per = defaultdict(list)
            for r in _rows(f):
                name = _get(r, "Kernel_Name", "Name")
                if match in name and _shape_ok(r, block, grid):
                    t = float(_get(r, "End_Timestamp")) - float(_get(r, "Start_Timestamp"))
                    per[name].append(t)
            for name, ts in per.items():
                out.write(f"# dispatches of {name[:150]}\n")
                shape = f" with workgroup {block}" + (f" and {grid} blocks" if grid is not None else "") if block else ""
                out.write(_line(f"dispatches{shape}", ts))
                if split_us is not None:
                    for label, part in ((f"shorter than {split_us:g} us", [t for t in ts if t < split_us * 1e3]),
                                        (f"{split_us:g} us or longer", [t for t in ts if t >= split_us * 1e3])):
                        if part:
                            out.write(_line(f"  {label}", part))
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        acc = defaultdict(lambda: defaultdict(float))
        for r in _rows(f):
            name = _get(r, "Kernel_Name", "Name")
            if match and match not in name and "copy" not in name.lower() and "elementwise" not in name.lower():
                continue
            if match and match in name and not _shape_ok(r, block, grid):
                continue
            key = (name, _get(r, "Dispatch_Id"))
            acc[key][_get(r, "Counter_Name")] += float(_get(r, "Counter_Value", default="0"))
        per = defaultdict(lambda: defaultdict(list))
        for (name, _), ctr in acc.items():
            for c, v in ctr.items():
                per[name][c].append(v)
        out.write(f"# {os.path.relpath(f, d)}: counters per dispatch (summed over instances)\n")
        for name, ctrs in per.items():
            for c, vs in ctrs.items():
                out.write(f"{c} | dispatches {len(vs)} | avg {sum(vs) / len(vs):.1f} | min {min(vs):.1f} | "
                          f"max {max(vs):.1f} | {name[:150]}\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--match", default=None)
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--grid", type=int, default=None)
    ap.add_argument("--split-us", type=float, default=None)
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--delete", action="store_true")
    a = ap.parse_args(argv)
    summarize(a.dir, a.match, a.block, a.grid, a.top, a.split_us)
    if a.delete:
        for pat in ("*kernel_trace.csv", "*counter_collection.csv"):
            for f in glob.glob(os.path.join(a.dir, "**", pat), recursive=True):
                os.remove(f)


if __name__ == "__main__":
    main()
