"""Write the oracle's results on the full-size solver workloads, for the GPU
parity tests (run on the CPU; calls only the oracle and the seeded input
generators):

* power_laplacian3d_128.json: the power method on the 3D 7-point Laplacian
  128^3 from the unit N(0,1) start (seed 4), 500 iterations, both inner
  products by qdot at tol 1e-6, and the same run with the exact dot: every
  lambda (hex), and the counts of both qdot results of every 50th iteration.
* cg_poisson2d_1024.json: CG on the 2D 5-point Poisson 1024^2 with
  b ~ N(0,1) (seed 3), x0 = 0, rtol 1e-10, qdot tol 1e-8, and with the
  exact dot: iteration count, status and residuals.

    python tests/golden/make_solver_goldens.py [power|cg]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def power():
    m, iters, tol = 128, 500, 1e-6
    rp, col, val = workloads.laplacian3d_csr(m)
    x0 = workloads.unit_vector(m ** 3, 4)
    out = {"workload": "3D 7-point Laplacian 128^3, unit N(0,1) start seed 4",
           "iters": iters, "qtol": tol}
    for use, key in ((1, "qdot"), (0, "exact_dot")):
        t = time.time()
        r = oracle.power(rp, col, val, x0, iters, tol, use, want_results=(use == 1))
        out[key] = {"status": r["status"], "lambda_hex": [float(v).hex() for v in r["trace"]]}
        if use == 1:
            out[key]["counts_every_50"] = {
                str(k): [r["results"][2 * k]["count"], r["results"][2 * k + 1]["count"]]
                for k in range(0, iters, 50)}
        print(f"power {key}: {time.time() - t:.0f} s, lambda {r['lambda']!r}", flush=True)
    with open(os.path.join(HERE, "power_laplacian3d_128.json"), "w") as f:
        json.dump(out, f, indent=1)


def cg():
    m = 1024
    rp, col, val = workloads.poisson2d_csr(m)
    b = workloads.normal_vector(m * m, 3)
    out = {"workload": "2D 5-point Poisson 1024^2, b ~ N(0,1) seed 3, x0 = 0",
           "rtol": 1e-10, "qtol": 1e-8}
    for use, key in ((1, "qdot"), (0, "exact_dot")):
        t = time.time()
        r = oracle.cg(rp, col, val, b, 1e-10, 1e-8, 20000, use)
        out[key] = {"status": r["status"], "iters": r["iters"],
                    "relres_est": r["relres_est"], "relres_true": r["relres_true"]}
        print(f"cg {key}: {time.time() - t:.0f} s, {r['iters']} iterations", flush=True)
    with open(os.path.join(HERE, "cg_poisson2d_1024.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    what = sys.argv[1:] or ["power", "cg"]
    for w in what:
        {"power": power, "cg": cg}[w]()
