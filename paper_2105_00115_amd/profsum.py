"""Summarise a rocprofv3 kernel trace (``*_kernel_trace.csv``).

Groups dispatches by short kernel name and reports calls, average, minimum
and maximum duration.  ``--first N`` keeps only the first N dispatches of
each kernel, which isolates the opening phase of a run (bench.py times the
single 2**27 qdot first, then the FP64 dots, then the solvers); ``--bytes``
converts average durations of the named kernels into GB/s.

    python -m paper_2105_00115_amd.profsum TRACE.csv --first 55 \
        --kernels k_scan,k_cut,k_acc,k_dot64 --bytes k_scan=2147483648,...

With ``--pmc WRITE.csv`` the first file is a FETCH_SIZE counter collection
and the second a WRITE_SIZE one (``rocprofv3 --pmc``, csv output): each
kernel's counters (KiB per dispatch, averaged over its first N dispatches)
are scaled to bytes by what the same counters read for a copy of known
size (``--calib KERNEL:GRID:BYTES``, bytes read = bytes written) and
compared with ``--algo`` bytes per launch; ``--json`` writes the table.
``--each`` lists every dispatch instead, its bytes also divided by
``--per`` (the iteration count of a persistent solver launch).
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


def counters(path, first=None, kernels=None):
    """{short name: [counter values in dispatch order]} and the grid of each."""
    groups = OrderedDict()
    with open(path) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        name = short_name(r["Kernel_Name"])
        base = name.split("<")[0]
        g = groups.setdefault(base, [])
        g.append((int(r["Grid_Size"]), float(r["Counter_Value"]), name))
    out = OrderedDict()
    for base, g in groups.items():
        if kernels and base not in kernels:
            continue
        out[base] = g[:first] if first else g
    return out, groups


def pmc_main(a):
    kernels = a.kernels.split(",") if a.kernels else None
    fetch, fall = counters(a.trace, a.first, kernels)
    write, wall = counters(a.pmc, a.first, kernels)
    ck, cgrid, cbytes = a.calib.split(":")
    cgrid, cbytes = int(cgrid), float(cbytes)
    cf = [v for g, v, _ in fall.get(ck, []) if g == cgrid]
    cw = [v for g, v, _ in wall.get(ck, []) if g == cgrid]
    if not cf or not cw:
        raise SystemExit(f"calibration kernel {ck} with grid {cgrid} not found")
    ff = cbytes / 1024.0 / cf[0]
    wf = cbytes / 1024.0 / cw[0]
    algo = float(a.algo) if a.algo else None
    table = OrderedDict()
    print(f"fetch factor {ff:.4f}, write factor {wf:.4f} "
          f"({ck} grid {cgrid}: FETCH {cf[0]:.1f} KiB, WRITE {cw[0]:.1f} KiB)")
    if a.each:
        # one row per dispatch, bytes divided by --per (e.g. the iterations
        # of a persistent solver launch)
        print(f"| kernel | dispatch | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | "
              f"HBM bytes (scaled) | bytes / {a.per:g} |")
        print("|---|---|---|---|---|---|")
        for base in (kernels or fetch.keys()):
            for i, ((_, fv, name), (_, wv, _)) in enumerate(zip(fetch.get(base, []),
                                                                write.get(base, []))):
                hb = (fv * ff + wv * wf) * 1024.0
                print(f"| {name} | {i} | {fv:.1f} | {wv:.1f} | {hb:.4e} | {hb / a.per:.4e} |")
        return
    print("| kernel | dispatches | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | "
          "HBM bytes / launch (scaled) | / algorithmic |")
    print("|---|---|---|---|---|---|")
    for base in (kernels or fetch.keys()):
        if base not in fetch or base not in write:
            continue
        fv = [v for _, v, _ in fetch[base]]
        wv = [v for _, v, _ in write[base]]
        f_avg, w_avg = sum(fv) / len(fv), sum(wv) / len(wv)
        hb = (f_avg * ff + w_avg * wf) * 1024.0
        ratio = hb / algo if algo else None
        table[base] = {"fetch_kib_raw": f_avg, "write_kib_raw": w_avg,
                       "hbm_bytes_per_launch": hb, "ratio_to_algorithmic": ratio}
        print(f"| {fetch[base][0][2]} | {len(fv)} | {f_avg:.1f} | {w_avg:.1f} | {hb:.4e} | "
              f"{'' if ratio is None else f'{ratio:.4f}'} |")
    if a.json:
        import json
        with open(a.json, "w") as f:
            json.dump({"fetch_factor": ff, "write_factor": wf, "per_kernel": table}, f,
                      indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--pmc", default=None, help="WRITE_SIZE csv (trace is FETCH_SIZE)")
    ap.add_argument("--calib", default="__amd_rocclr_copyBuffer:131072:268435456")
    ap.add_argument("--algo", default=None, help="algorithmic bytes per launch")
    ap.add_argument("--json", default=None)
    ap.add_argument("--first", type=int, default=None)
    ap.add_argument("--kernels", default=None)
    ap.add_argument("--each", action="store_true", help="with --pmc: one row per dispatch")
    ap.add_argument("--per", type=float, default=1.0, help="with --each: divide bytes by this")
    ap.add_argument("--bytes", default="", help="kernel=bytes_per_launch,...")
    a = ap.parse_args(argv)
    if a.pmc:
        return pmc_main(a)
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
