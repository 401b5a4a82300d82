"""Full-size parity of the single qdot: n = 2^27 (1 GiB per vector), the
law +-10^U[-20,20], in the launch configuration the benchmark times (the
default handle with the tuned shapes), at every tolerance of the
throughput workload (1e-3, 1e-6, 1e-10) and in both readings of the
accumulation (the default two-pass FP32-tile sums, and the one-pass exact
sums).  Exponent histogram, per-component classes, counts, e_min, e_max,
N_bins, t and flags bit for bit; the value within 1e-13 * sum |x_i y_i|.

The oracle runs of all six cases, the exact dot and the parity scale are
taken once, side by side in threads, when the module starts.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from parity_util import VALUE_TOL, host, parallel

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu

N = 1 << 27
TOLS = (1e-3, 1e-6, 1e-10)
S1 = [0, 0, 0, 1]


@pytest.fixture(scope="module")
def case():
    print(f"[gpu-case] full size n={N}: oracle runs", flush=True)
    x, y = workloads.log_uniform_pair(N, 2027)
    jobs = {"scale": lambda: oracle.abs_dot(x, y), "exact": lambda: oracle.dot_exact(x, y)}
    for tol in TOLS:
        jobs[("two", tol)] = lambda tol=tol: oracle.qdot(x, y, tol, want_classes=True,
                                                          want_hist=True)
        jobs[("one", tol)] = lambda tol=tol: oracle.qdot(x, y, tol, opt=S1)
    ref = parallel(jobs)
    h = q.Qdot(0)
    xd = torch.from_numpy(x).to("cuda:0")
    yd = torch.from_numpy(y).to("cuda:0")
    yield {"x": x, "y": y, "xd": xd, "yd": yd, "ref": ref, "h": h}
    h.close()


def _bounds_hold(r, o, tol, exact, scale):
    # the oracle's rigorous bound covers every rounding of the call; the
    # device value is within the parity tolerance of the oracle's
    assert abs(o["value"] - exact) <= o["bound_rig"]
    assert abs(r["value"] - exact) <= o["bound_rig"] + VALUE_TOL * scale
    # Thm 3.5: where Thm 3.3's hypothesis e_max <= flexp(x.y) holds and
    # every bin found a precision, the relative error is within tol
    b = oracle.bound_thm34(r, exact)
    if b["hyp"] and not r["flags"] & q.F_UNATTAINABLE:
        assert b["bound_thm3_rel"] <= tol
        assert abs(r["value"] - exact) <= tol * abs(exact)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("tol", TOLS)
def test_two_pass(case, tol):
    print(f"[gpu-case] full size two-pass tol={tol}", flush=True)
    h, xd, yd = case["h"], case["xd"], case["yd"]
    o = case["ref"][("two", tol)]
    cls, hist, r = h.qdot_classes(xd, yd, tol)
    for k in ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status"):
        assert r[k] == o[k], (k, r[k], o[k])
    np.testing.assert_array_equal(host(hist), o["hist"])
    np.testing.assert_array_equal(host(cls), o["classes"])
    del cls
    scale = case["ref"]["scale"]
    assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale, (r["value"], o["value"])
    for c in range(3):
        assert abs(r["part"][c] - o["part"][c]) <= VALUE_TOL * scale, c
    assert abs(r["bound_rel"] - o["bound_rel"]) <= 1e-12 * o["bound_rel"]
    # the timed entry point gives the debug entry point's result bit for bit
    r2 = h.qdot(xd, yd, tol)
    assert r2["value"] == r["value"] and r2["count"] == r["count"]
    _bounds_hold(r, o, tol, case["ref"]["exact"], scale)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("tol", TOLS)
def test_one_pass(case, tol):
    print(f"[gpu-case] full size one-pass tol={tol}", flush=True)
    h, xd, yd = case["h"], case["xd"], case["yd"]
    o = case["ref"][("one", tol)]
    r = h.qdot(xd, yd, tol, opt=S1)
    for k in ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status"):
        assert r[k] == o[k], (k, r[k], o[k])
    scale = case["ref"]["scale"]
    assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale, (r["value"], o["value"])
    # classes are those of the two-pass selection
    assert r["count"] == case["ref"][("two", tol)]["count"]
    _bounds_hold(r, o, tol, case["ref"]["exact"], scale)
