"""Summarise rocprofv3 CSV output (kernel statistics and counter collections)
into the short text tables kept under profiles/.

    python -m paper_1804_10541_amd.profsum --stats DIR [--pmc DIR ...] [--match REGEX]

--stats DIR: a ``--kernel-trace --stats -f csv`` output directory (reads
*kernel_stats.csv).  --pmc DIR: a ``--pmc ... -f csv`` output directory (reads
*counter_collection.csv; one value per dispatch and counter, averaged here).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import re


def kernel_stats(d, match):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        for r in csv.DictReader(open(f)):
            if match.search(r.get("Name", "")):
                rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                             float(r.get("MinNs", "nan")), float(r.get("MaxNs", "nan")), float(r["Percentage"])))
    return rows


def counters(d, match):
    acc = collections.defaultdict(list)
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        for r in csv.DictReader(open(f)):
            name = r.get("Kernel_Name", "")
            if match.search(name):
                acc[(name, r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v), min(v), max(v)) for k, v in acc.items()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--stats", action="append", default=[])
    ap.add_argument("--pmc", action="append", default=[])
    ap.add_argument("--match", default="mfr::|neg")
    args = ap.parse_args()
    match = re.compile(args.match)
    for d in args.stats:
        print(f"kernel statistics ({d})\n")
        print("| kernel | calls | total ms | avg us | min us | max us | % |")
        print("|---|---|---|---|---|---|---|")
        for name, calls, tot, avg, mn, mx, pct in kernel_stats(d, match):
            print(f"| `{name[:90]}` | {calls} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | {pct:.2f} |")
        print()
    for d in args.pmc:
        print(f"counters per dispatch ({d})\n")
        print("| kernel | counter | dispatches | mean | min | max |")
        print("|---|---|---|---|---|---|")
        for (name, cnt), (n, mean, mn, mx) in sorted(counters(d, match).items()):
            print(f"| `{name[:90]}` | {cnt} | {n} | {mean:.6g} | {mn:.6g} | {mx:.6g} |")
        print()


if __name__ == "__main__":
    main()
