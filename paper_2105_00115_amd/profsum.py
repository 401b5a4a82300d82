"""Summarise a rocprofv3 kernel trace (``*_kernel_trace.csv``).

Groups dispatches by short kernel name and reports calls, average, minimum
and maximum duration.  ``--first N`` keeps only the first N dispatches of
each kernel, which isolates the opening phase of a run (bench.py times the
single 2**27 qdot first, then the FP64 dots, then the solvers); ``--bytes``
converts average durations of the named kernels into GB/s.

    python -m paper_2105_00115_amd.profsum TRACE.csv --first 55 \
        --kernels k_scan,k_cut,k_acc,k_dot64 --bytes k_scan=2147483648,...
"""
from __future__ import annotations

import argparse
import csv
import re
import sys
from collections import OrderedDict


def short_name(full: str) -> str:
    s = re.sub(r"\(.*$", "", full)           # drop the argument list
    s = re.sub(r"^void\s+", "", s)
    tmpl = ""
    m = re.search(r"<(.*)>$", s)
    if m:
        tmpl = "<" + m.group(1) + ">"
        s = s[: m.start()]
    return s.split("::")[-1] + tmpl


def summarise(path, first=None, kernels=None):
    groups = OrderedDict()
    with open(path) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    for r in rows:
        name = short_name(r["Kernel_Name"])
        base = name.split("<")[0]
        if kernels and base not in kernels:
            continue
        g = groups.setdefault(name, [])
        if first is not None and len(g) >= first:
            continue
        g.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                  int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"])))
    return groups


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--first", type=int, default=None)
    ap.add_argument("--kernels", default=None)
    ap.add_argument("--bytes", default="", help="kernel=bytes_per_launch,...")
    a = ap.parse_args(argv)
    kernels = set(a.kernels.split(",")) if a.kernels else None
    nbytes = dict(kv.split("=") for kv in a.bytes.split(",") if kv)
    groups = summarise(a.trace, a.first, kernels)
    print("| kernel | calls | avg us | min us | max us | grid x block | GB/s (avg) |")
    print("|---|---|---|---|---|---|---|")
    for name, g in groups.items():
        d = [x[0] for x in g]
        avg = sum(d) / len(d)
        base = name.split("<")[0]
        gbs = f"{float(nbytes[base]) / avg:.1f}" if base in nbytes else ""
        grids = sorted({f"{x[1] // max(x[2], 1)}x{x[2]}" for x in g})
        print(f"| {name} | {len(d)} | {avg / 1e3:.2f} | {min(d) / 1e3:.2f} | "
              f"{max(d) / 1e3:.2f} | {' '.join(grids)} | {gbs} |")


if __name__ == "__main__":
    sys.exit(main())
