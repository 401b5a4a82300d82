"""Autotuner for the qdot launch shapes.

Single qdot, per size bucket (n < 2^16, < 2^20, < 2^24, >= 2^24): it times
the exponent scan and the accumulate pass with the library's own HIP-event
kernel timing over

* persistent-grid sizes (blocks per CU) and groups in flight per lane,
* the two forms of the accumulate pass (every candidate leaf formed in
  place, or the kept components compacted per wave),
* the number of global histogram copies the scan blocks merge into,
* the one-pass scan's grid and groups in flight,

and keeps the fastest.  Every swept shape must reproduce the reference
run's per-component classes and exponent histogram bit for bit (and its
counts, t and flags); the one-pass value, an exact sum, must be the same
bits.  The tile structure makes that hold for every shape; the tuner checks
it for each one rather than assuming it.

Batched launch: blocks per CU and the chunk size on a ragged batch (counts
bit for bit, values within 1e-13 of the reference run's scale), and the CG
gang sizing (rows per gang block, largest gang) on a batch of CG systems.

The result is a text file that ``qdot_load_tune`` reads; ``Qdot()`` loads
``tune/<arch>_<cus>cu.txt`` next to this module when it exists.

    python -m paper_2105_00115_amd.autotune [--out PATH] [--reps 20]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

BUCKET_N = [1 << 15, 1 << 19, 1 << 23, 1 << 27]
BPC = (1, 2, 4, 8, 16)
UNROLL = (1, 2, 4)
ACC_FORM = (0, 1)
HIST_COPIES = (1, 2, 4, 8)
BATCH_BPC = (2, 4, 8)
BATCH_CHUNK = (65536, 131072, 262144)
CG_ROWS = (8192, 16384, 32768)
CG_GANG_MAX = (16, 32, 64)


def default_path(arch: str, cus: int) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune",
                        f"{arch}_{cus}cu.txt")


def _time_config(h, x, y, tol, out, cfg, reps, opt=None):
    h.set_tune(-1, *cfg)
    for _ in range(3):
        h.qdot_async(x, y, tol, out, opt=opt)
    import torch
    torch.cuda.synchronize()
    h.timing_read()
    h.timing_enable(True)
    for _ in range(reps):
        h.qdot_async(x, y, tol, out, opt=opt)
    torch.cuda.synchronize()
    h.timing_enable(False)
    t = h.timing_read()
    c = t["qdot_calls"]
    return (t["scan_ms"] / c, t["cut_ms"] / c, t["acc_ms"] / c, t["fin_ms"] / c)


class ShapeChanged(RuntimeError):
    pass


def _check_same(h, x, y, tol, cfg, ref_cls, ref_hist, ref):
    """The shape cfg gives the reference classes and histogram bit for bit."""
    import torch
    h.set_tune(-1, *cfg)
    cls, hist, r = h.qdot_classes(x, y, tol)
    same = (torch.equal(cls, ref_cls) and torch.equal(hist, ref_hist)
            and (r["count"], r["t"], r["flags"], r["n_bins"])
            == (ref["count"], ref["t"], ref["flags"], ref["n_bins"]))
    if not same:
        raise ShapeChanged(f"config {cfg} changed the classes or the histogram")


def tune(reps: int = 20, seed: int = 7, tol: float = 1e-6, log=print, buckets=None):
    """Sweep the launch shapes of the buckets listed (all by default);
    returns the handle, the chosen shapes with their timings, and the number
    of shapes whose classes and histogram were compared."""
    import torch

    import paper_2105_00115_amd as q
    import workloads

    h = q.Qdot(0, load_tuned=False)
    h.reset_tune()
    dev = "cuda:0"
    out = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device=dev)
    chosen = []
    checked = 0
    for b, n in enumerate(BUCKET_N):
        if buckets is not None and b not in buckets:
            continue
        x, y = workloads.log_uniform_pair_torch(n, seed + b, dev)
        ref_cls, ref_hist, ref = h.qdot_classes(x, y, tol)
        d1 = h.get_tune(b)[4:6]
        # grid and groups in flight of both passes (dense form, 8 copies)
        results = {}
        for bpc in BPC:
            for u in UNROLL:
                cfg = (bpc, u, bpc, u) + d1 + (0, 8)
                results[cfg] = _time_config(h, x, y, tol, out, cfg, reps)
                _check_same(h, x, y, tol, cfg, ref_cls, ref_hist, ref)
                checked += 1
        best_scan = min(results, key=lambda c: results[c][0])[:2]
        best_acc = min(results, key=lambda c: results[c][2])[2:4]
        mixed = best_scan + best_acc + d1 + (0, 8)
        if mixed not in results:
            results[mixed] = _time_config(h, x, y, tol, out, mixed, reps)
            _check_same(h, x, y, tol, mixed, ref_cls, ref_hist, ref)
            checked += 1
        best = min(results, key=lambda c: sum(results[c]))
        # accumulate form and histogram copies at that shape
        for af in ACC_FORM:
            for hc in HIST_COPIES:
                cfg = best[:6] + (af, hc)
                if cfg not in results:
                    results[cfg] = _time_config(h, x, y, tol, out, cfg, reps)
                    _check_same(h, x, y, tol, cfg, ref_cls, ref_hist, ref)
                    checked += 1
        best = min(results, key=lambda c: sum(results[c]))
        t = results[best]
        # one-pass scan (accum_mode 1): its value is an exact sum, so every
        # shape must give the same bits
        one = [0, 0, 0, 1]
        h.set_tune(-1, *best)
        ref1 = h.qdot(x, y, tol, opt=one)
        res1 = {}
        for bpc in BPC:
            for u in UNROLL:
                cfg = best[:4] + (bpc, u) + best[6:]
                res1[cfg] = _time_config(h, x, y, tol, out, cfg, reps, opt=one)
                r = q.parse_results(out)[0]
                if (r["count"], r["value"]) != (ref1["count"], ref1["value"]):
                    raise ShapeChanged(f"one-pass config {cfg} changed the result")
        best = min(res1, key=lambda c: sum(res1[c]))
        _check_same(h, x, y, tol, best, ref_cls, ref_hist, ref)
        checked += 1
        t1 = res1[best]
        log(f"bucket {b} n={n}: best {best} scan {t[0]*1e3:.1f} us cut {t[1]*1e3:.1f} us "
            f"acc {t[2]*1e3:.1f} us fin {t[3]*1e3:.1f} us; one-pass scan {t1[0]*1e3:.1f} us")
        chosen.append((b, n, best, t + (t1[0],)))
        del x, y
    return h, chosen, checked


def _time_batch(h, run, reps):
    import torch
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune_batch(h, reps: int = 5, seed: int = 11, log=print):
    """Batched launch shape: blocks per CU and chunk on 512 ragged instances,
    then the CG gang sizing on 32 CG systems.  Returns the chosen
    (blocks_per_cu, chunk, cg_rows_per_block, cg_gang_max)."""
    import torch

    import paper_2105_00115_amd as q
    import workloads

    dev = "cuda:0"
    offs, xh, yh, tols = workloads.ragged_batch(512, seed)
    x, y = torch.from_numpy(xh).to(dev), torch.from_numpy(yh).to(dev)
    del xh, yh
    off_d = torch.from_numpy(offs).to(dev)
    tol_d = torch.from_numpy(tols).to(dev)
    out = torch.zeros(len(tols) * q.RESULT_BYTES, dtype=torch.uint8, device=dev)
    h.set_batch_tune()
    h.batched_async(x, y, off_d, offs, tol_d, out)
    torch.cuda.synchronize()
    ref = q.parse_results(out)
    res = {}
    for bpc in BATCH_BPC:
        for ch in BATCH_CHUNK:
            h.set_batch_tune(blocks_per_cu=bpc, chunk=ch)
            res[(bpc, ch)] = _time_batch(
                h, lambda: h.batched_async(x, y, off_d, offs, tol_d, out), reps)
            got = q.parse_results(out)
            for j, (a, r) in enumerate(zip(got, ref)):
                if a["count"] != r["count"] or a["t"] != r["t"] or a["flags"] != r["flags"]:
                    raise ShapeChanged(f"batch shape {(bpc, ch)} changed instance {j}")
    bpc, ch = min(res, key=res.get)
    log(f"batch: best blocks/CU {bpc} chunk {ch} ({res[(bpc, ch)]*1e3:.3f} ms)")
    # CG gang sizing on 2D Poisson systems with sides 2^U[6, 9]
    sides = workloads.cg_grid_sides(32, seed + 2, 6.0, 9.0)
    systems, xs = [], []
    for s_, m in enumerate(sides):
        rp, ci, va = workloads.poisson2d_csr(int(m))
        A = q.Csr(rp, ci, va, dev)
        b = torch.from_numpy(workloads.normal_vector(A.n, 100 + s_)).to(dev)
        xx = torch.zeros(A.n, dtype=torch.float64, device=dev)
        xs.append(xx)
        systems.append((A, b, xx, 1e-10, 1e-8, 20000, 1))
    cg_res = {}
    for rows in CG_ROWS:
        for gmax in CG_GANG_MAX:
            h.set_batch_tune(blocks_per_cu=bpc, chunk=ch, cg_rows_per_block=rows,
                             cg_gang_max=gmax)
            for xx in xs:
                xx.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rr = h.cg_batched(systems)
            cg_res[(rows, gmax)] = time.perf_counter() - t0
            if any(r["status"] != q.OK for r in rr):
                raise RuntimeError(f"CG gang shape {(rows, gmax)} failed: {rr}")
    rows, gmax = min(cg_res, key=cg_res.get)
    log(f"batch CG: best rows/block {rows} gang max {gmax} ({cg_res[(rows, gmax)]*1e3:.1f} ms)")
    h.set_batch_tune(blocks_per_cu=bpc, chunk=ch, cg_rows_per_block=rows, cg_gang_max=gmax)
    return (bpc, ch, rows, gmax)


def write(path, chosen, arch, cus, batch=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write(f"# qdot launch shapes for {arch} with {cus} CUs, written by "
                f"python -m paper_2105_00115_amd.autotune on {time.strftime('%Y-%m-%d')}\n")
        f.write("# bucket scan_blocks_per_cu scan_unroll acc_blocks_per_cu acc_unroll"
                " onepass_blocks_per_cu onepass_unroll acc_form hist_copies"
                "   (measured n, scan/cut/acc/fin us, one-pass scan us)\n")
        for b, n, cfg, t in chosen:
            f.write(f"{b} {' '.join(str(c) for c in cfg)}   # n={n} "
                    f"{t[0]*1e3:.1f}/{t[1]*1e3:.1f}/{t[2]*1e3:.1f}/{t[3]*1e3:.1f}, "
                    f"{t[4]*1e3:.1f}\n")
        if batch is not None:
            f.write("# batch blocks_per_cu chunk cg_rows_per_block cg_gang_max\n")
            f.write("batch " + " ".join(str(v) for v in batch) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--buckets", default=None,
                    help="comma-separated bucket indices to tune (default: all)")
    ap.add_argument("--no-batch", action="store_true", help="leave the batched shape out")
    a = ap.parse_args(argv)
    import torch

    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    cus = props.multi_processor_count
    buckets = None if a.buckets is None else [int(b) for b in a.buckets.split(",")]
    log = lambda m: print(m, flush=True)  # noqa: E731
    h, chosen, checked = tune(a.reps, log=log, buckets=buckets)
    log(f"{checked} shapes gave the reference classes and histogram bit for bit")
    batch = None if a.no_batch else tune_batch(h, log=log)
    path = a.out or default_path(arch, cus)
    write(path, chosen, arch, cus, batch)
    h.load_tune(path)  # the file must load back
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
