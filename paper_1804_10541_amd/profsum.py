"""Summarise rocprofv3 CSV output (kernel statistics and counter collections)
into the short text tables kept under profiles/.

    python -m paper_1804_10541_amd.profsum --stats DIR [--pmc DIR ...] [--match REGEX]

--stats DIR: a ``--kernel-trace --stats -f csv`` output directory (reads
*kernel_stats.csv).  --pmc DIR: a ``--pmc ... -f csv`` output directory (reads
*counter_collection.csv; one value per dispatch and counter, averaged here).
--traffic REGEX: HBM bytes per launch of the matching kernel from its
FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the same
counter reads for the copy kernel (torch's neg over 2^28 floats: 1 GiB read,
1 GiB written), with the hash of the voxel-tile kernel sources and the tile
configuration given by --tile BXxBY:TARGET.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import hashlib
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the sources the Hessian-vector voxel-tile kernel is compiled from
HV_SOURCES = ("paper_1804_10541_amd/csrc/ngf_tile.hip", "paper_1804_10541_amd/csrc/tile_common.h",
              "paper_1804_10541_amd/csrc/mfr_internal.h")
COPY_BYTES = 1 << 30   # the copy kernel's read and write, each


def kernel_source_hash():
    h = hashlib.sha256()
    for f in HV_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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
    ap.add_argument("--traffic", default=None)
    ap.add_argument("--tile", default=None)
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
    if args.traffic:
        allc = {}
        for d in args.pmc:
            allc.update(counters(d, re.compile(args.traffic + "|neg")))
        want = re.compile(args.traffic)

        def mean(kind, cnt):
            vals = [v[1] for (n, c), v in allc.items() if c == cnt and (want.search(n) if kind == "k" else "neg" in n)]
            if len(vals) != 1:
                raise SystemExit(f"--traffic: {len(vals)} kernels match for {cnt}")
            return vals[0]

        f_scale = COPY_BYTES / (mean("c", "FETCH_SIZE") * 1024.0)
        w_scale = COPY_BYTES / (mean("c", "WRITE_SIZE") * 1024.0)
        fetch = mean("k", "FETCH_SIZE") * 1024.0 * f_scale
        write = mean("k", "WRITE_SIZE") * 1024.0 * w_scale
        print(f"Copy calibration: FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x {w_scale:.4f}")
        print(f"HBM read per launch: {fetch:,.0f} bytes; written: {write:,.0f} bytes")
        print(f"HBM traffic per launch: {fetch + write:,.0f} bytes")
        print(f"Kernel sources (sha256, 16 hex): `{kernel_source_hash()}`")
        if args.tile:
            bxy, target = args.tile.split(":")
            print(f"Tile configuration: {bxy}, split target {target}")


if __name__ == "__main__":
    main()
