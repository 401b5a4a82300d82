"""A short run of the hot kernels for profiler counter passes.

Runs, in this order, on cuda:0:

1. a 256 MiB ``torch`` copy (256 MiB read, 256 MiB written), whose
   FETCH_SIZE / WRITE_SIZE give the scale factors of the byte counters;
2. the single qdot on the throughput workload (n = 2^27 FP64 components
   +-10^U[-20,20], tol 1e-6): ``steps`` calls of the two-pass mode, of the
   one-pass mode and of the FP64 dot;
3. CG on the 2D Poisson matrix 1024^2 (qdot tol 1e-8, stop at 1e-10) with
   the two-pass qdot, the FP64 dot and the one-pass qdot, one solve each;
4. the power method on the 3D Laplacian 128^3, ``power_iters`` iterations
   with the two-pass qdot;
5. tile skipping: a banded pair of 2^26 components (three quarters of its
   bands 2^-300 below the rest, tol 1e-6), ``steps`` calls without and
   ``steps`` calls with tile_skip (its k_scan / k_acc instantiations carry
   the template flag ``true``);
6. the batched launch on 4096 ragged instances (n = round(10^U[2,6]), tol
   from {1e-4, 1e-6, 1e-8}): one launch two-pass, then one one-pass.

Each phase prints its name and, for the solvers, the iteration counts, so
that per-dispatch counters can be divided by iterations.

    python3 paper_2105_00115_amd/profile_kernels.py [--steps 3] [--power-iters 50]
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--power-iters", type=int, default=50)
    a = ap.parse_args(argv)
    import torch

    import paper_2105_00115_amd as q
    import workloads

    dev = "cuda:0"
    print("[profile] calibration copy 256 MiB", flush=True)
    src = torch.empty(1 << 25, dtype=torch.float64, device=dev).uniform_()
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    n, tol = 1 << 27, 1e-6
    print(f"[profile] single qdot n={n} tol={tol}", flush=True)
    x, y = workloads.log_uniform_pair_torch(n, 2027, dev)
    h = q.Qdot(0)
    out = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device=dev)
    d_out = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(a.steps):
        h.qdot_async(x, y, tol, out)
    for _ in range(a.steps):
        h.qdot_async(x, y, tol, out, opt=[0, 0, 0, 1])
    for _ in range(a.steps):
        h.fp64_dot_async(x, y, d_out)
    torch.cuda.synchronize()
    del x, y

    m = 1024
    print(f"[profile] CG 2D Poisson {m}^2", flush=True)
    A = q.Csr(*workloads.poisson2d_csr(m), device=dev)
    b = torch.from_numpy(workloads.normal_vector(m * m, 3)).to(dev)
    for name, use, opt in (("qdot", 1, None), ("fp64", 0, None), ("qdot_one_pass", 1, [0, 0, 0, 1])):
        xs = torch.zeros(m * m, dtype=torch.float64, device=dev)
        r = h.cg(A, b, xs, 1e-10, 1e-8, 20000, use, opt=opt)
        print(f"[profile] CG {name}: {r['iters']} iterations, status {r['status']}", flush=True)
    del A, b

    m3 = 128
    print(f"[profile] power method 3D Laplacian {m3}^3, {a.power_iters} iterations", flush=True)
    A = q.Csr(*workloads.laplacian3d_csr(m3), device=dev)
    xs = torch.from_numpy(workloads.unit_vector(m3 ** 3, 4)).to(dev)
    r = h.power(A, xs, a.power_iters, 1e-6, 1, trace=False)
    print(f"[profile] power: lambda {r['lambda']!r}, status {r['status']}", flush=True)
    del A, xs

    print("[profile] tile skipping, banded pair 2^26", flush=True)
    xb, yb = workloads.banded_pair(1 << 26, 81, levels=(0, -300, -300, -300),
                                   mean_band=20000.0)
    xb, yb = torch.from_numpy(xb).to(dev), torch.from_numpy(yb).to(dev)
    for opt in (None, [0, 0, 0, 0, 0, 0, 0, 1]):
        for _ in range(a.steps):
            h.qdot_async(xb, yb, 1e-6, out, opt=opt)
    torch.cuda.synchronize()
    del xb, yb

    import numpy as np

    g = workloads.rng(2025)
    sizes = np.rint(10.0 ** g.uniform(2, 6, 4096)).astype(np.int64)
    offs = np.zeros(4097, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    tols = np.array([1e-4, 1e-6, 1e-8])[g.integers(0, 3, 4096)]
    print(f"[profile] batched 4096 ragged instances, {int(offs[-1])} components", flush=True)
    bx, by = workloads.log_uniform_pair_torch(int(offs[-1]), 2025, dev)
    off_d = torch.from_numpy(offs).to(dev)
    tol_d = torch.from_numpy(tols).to(dev)
    bout = torch.zeros(4096 * q.RESULT_BYTES, dtype=torch.uint8, device=dev)
    for opt in (None, [0, 0, 0, 1]):
        h.batched_async(bx, by, off_d, offs, tol_d, bout, opt=opt)
    torch.cuda.synchronize()
    h.close()
    print("[profile] done", flush=True)


if __name__ == "__main__":
    main()
