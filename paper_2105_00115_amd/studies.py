"""The paper's synthetic studies (Sec. 4.1) run on the device.

E1, tightness of the error bound: eps = 1e-16; family A with t = 10, 15,
..., 100 and family B with t = 2, 4, ..., 30, 100 pairs per t, for n = 1e2,
1e3, ..., 1e7.  Per pair, qdot's bound minus relerr, where relerr =
|d - qdot| / |d| with d the FP64 dot of the same pair, and the bound is
bound_rel, the Thm 3.3 sum that the proof of Thm 3.5 holds below eps (the
score uses eps / N_bins, as the study does).

E2, approximation effectiveness, speedup and efficiency: eps = 1e-15,
1e-14, ..., 1e-1; families A and B with t in {5, 9, 13}; 50 pairs per eps;
n = 1e5, 1e6, 1e7, 1e8.  Per cell, relerr mean / min / max and the class
mix.  HIP-event kernel times give the approximation speedup
t(FP64 dot) / t(computation phase) and the approximation efficiency
t(FP64 dot) / (t(parameter selection) + t(FP64 dot)) (definitions of Sec. 2).
The computation phase is k_acc + k_fin; the parameter selection is k_scan +
k_cut.

Inputs are drawn on the device (``workloads.paper_dist_torch``), one seed per
pair.  Every call goes through the C ABI; this module only drives it and
summarises the results.

    python -m paper_2105_00115_amd.studies --study all --out FILE
    python -m paper_2105_00115_amd.studies --study e1 --scale small --out FILE
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

E1_EPS = 1e-16
E1_T = {"A": [5 * i for i in range(2, 21)], "B": [2 * i for i in range(1, 16)]}
E1_SIZES = [10 ** k for k in range(2, 8)]
E1_PAIRS = 100
E2_EPS = [10.0 ** -k for k in range(15, 0, -1)]
E2_T = [5, 9, 13]
E2_SIZES = [10 ** k for k in range(5, 9)]
E2_PAIRS = 50


def _cell(h, q, workloads, n, t, family, eps, pairs, seed0, timed=False):
    """Run `pairs` qdot + FP64-dot calls on fresh pairs; returns the parsed
    results, the FP64 dots and (timed) the summed kernel times."""
    import torch

    rb = q.RESULT_BYTES
    out = torch.zeros(pairs * rb, dtype=torch.uint8, device="cuda:0")
    dots = torch.zeros(pairs, dtype=torch.float64, device="cuda:0")
    if timed:
        h.timing_enable(True)
    base = out.data_ptr()
    for i in range(pairs):
        x, y = workloads.paper_dist_torch(n, t, seed0 + i, family)
        h.qdot_async(x, y, eps, base + i * rb)
        h.fp64_dot_async(x, y, dots[i:i + 1])
        del x, y
    torch.cuda.synchronize()
    tm = None
    if timed:
        tm = h.timing_read()
        h.timing_enable(False)
    return q.parse_results(out), dots.cpu().numpy(), tm


def _relerr(res, dots):
    v = np.array([r["value"] for r in res])
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.abs(dots - v) / np.abs(dots)


def _quartiles(a):
    a = np.asarray(a, dtype=np.float64)
    return {"min": float(a.min()), "q1": float(np.quantile(a, 0.25)),
            "median": float(np.median(a)), "q3": float(np.quantile(a, 0.75)),
            "max": float(a.max())}


def study_e1(h, q, workloads, sizes, pairs, ts=E1_T, log=print):
    out = {"eps": E1_EPS, "pairs_per_t": pairs, "t": ts, "cells": []}
    seed = 1_000_000
    for family in ("A", "B"):
        for n in sizes:
            diff, rel, bound, unatt, bad = [], [], [], 0, 0
            t0 = time.perf_counter()
            for t in ts[family]:
                res, dots, _ = _cell(h, q, workloads, n, t, family, E1_EPS, pairs, seed)
                seed += pairs
                r = _relerr(res, dots)
                b = np.array([x["bound_rel"] for x in res])
                bad += sum(x["status"] != q.OK for x in res)
                unatt += sum(bool(x["flags"] & q.F_UNATTAINABLE) for x in res)
                diff.extend((b - r).tolist())
                rel.extend(r.tolist())
                bound.extend(b.tolist())
            diff = np.array(diff)
            out["cells"].append({
                "family": family, "n": n, "samples": len(diff),
                "bound_minus_relerr": _quartiles(diff),
                "relerr": _quartiles(rel), "bound": _quartiles(bound),
                "relerr_above_bound": int((diff < 0).sum()),
                "relerr_above_eps": int((np.array(rel) > E1_EPS).sum()),
                "unattainable": unatt, "bad_status": bad,
                "seconds": round(time.perf_counter() - t0, 2)})
            log(f"[e1] family {family} n={n}: {len(diff)} pairs, "
                f"median bound-relerr {np.median(diff):.3e}, "
                f"relerr > bound in {(diff < 0).sum()}")
    return out


def study_e2(h, q, workloads, sizes, pairs, ts=E2_T, eps_list=E2_EPS, log=print):
    out = {"eps": eps_list, "t": ts, "pairs_per_eps": pairs, "cells": [], "timing": []}
    seed = 2_000_000
    for family in ("A", "B"):
        for t in ts:
            for n in sizes:
                acc = {"scan_ms": 0.0, "cut_ms": 0.0, "acc_ms": 0.0, "fin_ms": 0.0,
                       "dot64_ms": 0.0, "calls": 0}
                for eps in eps_list:
                    res, dots, tm = _cell(h, q, workloads, n, t, family, eps, pairs, seed,
                                          timed=True)
                    seed += pairs
                    r = _relerr(res, dots)
                    cnt = np.array([x["count"] for x in res], dtype=np.float64) / n
                    out["cells"].append({
                        "family": family, "t": t, "n": n, "eps": eps,
                        "relerr_mean": float(r.mean()), "relerr_min": float(r.min()),
                        "relerr_max": float(r.max()),
                        "relerr_above_eps": int((r > eps).sum()),
                        "class_frac_mean": [round(float(v), 6) for v in cnt.mean(axis=0)],
                        "bound_mean": float(np.mean([x["bound_rel"] for x in res]))})
                    for k in ("scan_ms", "cut_ms", "acc_ms", "fin_ms", "dot64_ms"):
                        acc[k] += tm[k]
                    acc["calls"] += tm["qdot_calls"]
                c = acc["calls"]
                comp = (acc["acc_ms"] + acc["fin_ms"]) / c
                sel = (acc["scan_ms"] + acc["cut_ms"]) / c
                d64 = acc["dot64_ms"] / c
                out["timing"].append({
                    "family": family, "t": t, "n": n, "calls": c,
                    "selection_ms": round(sel, 5), "computation_ms": round(comp, 5),
                    "fp64_dot_ms": round(d64, 5),
                    "approx_speedup": round(d64 / comp, 4),
                    "approx_efficiency": round(d64 / (sel + d64), 4)})
                log(f"[e2] family {family} t={t} n={n}: speedup {d64 / comp:.3f}, "
                    f"efficiency {d64 / (sel + d64):.3f}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--study", choices=["e1", "e2", "all"], default="all")
    ap.add_argument("--scale", choices=["paper", "small"], default="paper")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    import workloads
    import paper_2105_00115_amd as q

    def log(msg):
        print(msg, flush=True)

    h = q.Qdot(0)
    res = {"scale": a.scale}
    small = a.scale == "small"
    if a.study in ("e1", "all"):
        ts = {"A": E1_T["A"][::6], "B": E1_T["B"][::5]} if small else E1_T
        res["e1"] = study_e1(h, q, workloads, [100, 1000] if small else E1_SIZES,
                             4 if small else E1_PAIRS, ts=ts, log=log)
    if a.study in ("e2", "all"):
        res["e2"] = study_e2(h, q, workloads, [1000, 100000] if small else E2_SIZES,
                             3 if small else E2_PAIRS,
                             eps_list=E2_EPS[::7] if small else E2_EPS, log=log)
    h.close()
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    log(f"[done] {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
