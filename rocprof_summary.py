"""Summarise rocprofv3 CSV output for the library's kernels.

    python rocprof_summary.py stats DIR [--top N] [--per STEPS]
        per-kernel calls and mean / min / max duration from the
        ``*_kernel_stats.csv`` that ``rocprofv3 --kernel-trace --stats
        --output-format csv -d DIR`` writes, and the total kernel time (per
        step, with --per: the run's step count);
    python rocprof_summary.py pmc DIR [--match S]
        per-kernel mean counter value per dispatch from the
        ``*_counter_collection.csv`` of a ``rocprofv3 --pmc ...`` run (counters
        summed over their instances within a dispatch).

Reads text files only; prints a Markdown table.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import sys


def _files(d: str, suffix: str):
    out = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not out:
        raise SystemExit(f"no *{suffix} under {d}")
    return out


def _key(row: dict, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(names)


def stats(d: str, top: int, per: int = 0):
    rows = []
    for f in _files(d, "_kernel_stats.csv"):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(_key(r, "TotalDurationNs")))
    print("| kernel | calls | mean us | min us | max us | share % |")
    print("|---|---|---|---|---|---|")
    for r in rows[:top]:
        print(f"| `{_key(r, 'Name')[:110]}` | {_key(r, 'Calls')} | "
              f"{float(_key(r, 'AverageNs')) / 1e3:.2f} | {float(_key(r, 'MinNs')) / 1e3:.2f} | "
              f"{float(_key(r, 'MaxNs')) / 1e3:.2f} | {float(_key(r, 'Percentage')):.2f} |")
    tot = sum(float(_key(r, "TotalDurationNs")) for r in rows) / 1e3
    calls = sum(int(_key(r, "Calls")) for r in rows)
    print(f"\nall kernels: {calls} launches, {tot:.1f} us in total")
    if per > 0:
        print(f"per step ({per} steps): {calls / per:.1f} launches, {tot / per:.2f} us")


def pmc(d: str, match: str):
    per = collections.defaultdict(float)          # (kernel, dispatch, counter) -> value
    for f in _files(d, "_counter_collection.csv"):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _key(r, "Kernel_Name")
                if match and match not in k:
                    continue
                per[(k, _key(r, "Dispatch_Id"), _key(r, "Counter_Name"))] += \
                    float(_key(r, "Counter_Value"))
    agg = collections.defaultdict(list)
    for (k, _, c), v in per.items():
        agg[(k, c)].append(v)
    print("| kernel | counter | dispatches | mean per dispatch | min | max |")
    print("|---|---|---|---|---|---|")
    for (k, c), vs in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{k[:110]}` | {c} | {len(vs)} | {sum(vs) / len(vs):.1f} | {min(vs):.1f} | "
              f"{max(vs):.1f} |")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--top", type=int, default=12)
    a.add_argument("--per", type=int, default=0)
    b = sub.add_parser("pmc")
    b.add_argument("dir")
    b.add_argument("--match", default="")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        stats(args.dir, args.top, args.per)
    else:
        pmc(args.dir, args.match)


if __name__ == "__main__":
    sys.exit(main())
