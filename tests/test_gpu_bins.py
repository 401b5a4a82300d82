"""GPU parity of the other binning strategies of Sec. 3.2 (bin_mode 1:
ranged bins of a fixed width; bin_mode 2: variable-width bins from a number
of splits) against the oracle: per-component classes, exponent histogram,
counts, N_bins, t and flags bit for bit, the value within 1e-13 *
sum |x_i y_i|, bound_rel within 1e-12 relative.  Width 1, and as many
splits as exponents, reduce to exact binning.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from parity_util import INT_KEYS, VALUE_TOL

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


def compare(h, x, y, tol, opt, f32=False):
    print(f"[gpu-case] bins n={len(x)} tol={tol} opt={opt} f32={f32}", flush=True)
    if f32:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        cls, hist, r = h.qdot_f32_classes(dev(x, np.float32), dev(y, np.float32), tol, opt=opt)
        o = oracle.qdot_f32(x, y, tol, opt=opt, want_classes=True, want_hist=True)
    else:
        cls, hist, r = h.qdot_classes(dev(x), dev(y), tol, opt=opt)
        o = oracle.qdot(x, y, tol, opt=opt, want_classes=True, want_hist=True)
    for k in INT_KEYS:
        assert r[k] == o[k], (k, r[k], o[k])
    np.testing.assert_array_equal(hist.cpu().numpy(), o["hist"])
    np.testing.assert_array_equal(cls.cpu().numpy(), o["classes"])
    if o["status"] == oracle.OK:
        scale = oracle.abs_dot(np.float64(x), np.float64(y))
        assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale, (r["value"], o["value"])
        # a ranged bin reaching far past e_max has an infinite Thm 3.3 term
        # (u_k - e_max beyond the double range): both sides report inf
        if np.isinf(o["bound_rel"]):
            assert r["bound_rel"] == o["bound_rel"]
        else:
            assert abs(r["bound_rel"] - o["bound_rel"]) <= 1e-12 * abs(o["bound_rel"])
    return r, o


RANGED = [1, 2, 3, 7, 64, 4196]
SPLITS = [0, 1, 5, 50, 4196]


@pytest.mark.parametrize("w", RANGED)
@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10])
def test_ranged_bins(h, w, tol):
    x, y = workloads.log_uniform_pair(200003, 61)
    compare(h, x, y, tol, [0, 0, 0, 0, 0, 1, w])


@pytest.mark.parametrize("s", SPLITS)
@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10])
def test_variable_bins(h, s, tol):
    x, y = workloads.log_uniform_pair(200003, 62)
    compare(h, x, y, tol, [0, 0, 0, 0, 0, 2, s])


@pytest.mark.parametrize("opt", [[1, 0, 0, 0, 0, 1, 5], [0, 1, 1, 0, 0, 2, 17],
                                 [0, 0, 1, 0, 0, 1, 9], [1, 1, 0, 0, 0, 2, 3]])
def test_bins_with_other_options(h, opt):
    # key, score and boundary modes combine with both strategies; the
    # paper's Dist. B (one sign, narrow exponent spread) and the law of the
    # throughput workload
    x, y = workloads.paper_dist_b(100000, 9.0, 63)
    compare(h, x, y, 1e-6, opt)
    x, y = workloads.log_uniform_pair(65537, 64)
    compare(h, x, y, 1e-8, opt)


def test_bins_reduce_to_exact(h):
    # width 1, and at least e_max - e_min splits, are exact binning
    x, y = workloads.log_uniform_pair(100000, 65)
    r0, _ = compare(h, x, y, 1e-6, None)
    r1, _ = compare(h, x, y, 1e-6, [0, 0, 0, 0, 0, 1, 1])
    r2, _ = compare(h, x, y, 1e-6, [0, 0, 0, 0, 0, 2, 4196])
    for k in INT_KEYS + ("value",):
        assert r0[k] == r1[k] == r2[k], k


@pytest.mark.parametrize("opt", [[0, 0, 0, 0, 0, 1, 4], [0, 0, 0, 0, 0, 2, 12]])
def test_bins_single_precision_inputs(h, opt):
    x, y = workloads.log_uniform_pair(150001, 66, -15.0, 15.0)
    for tol in (1e-2, 1e-5):
        compare(h, x, y, tol, opt, f32=True)


def test_bins_edge_inputs(h):
    # one component, all zeros, a single exponent, empty input
    compare(h, np.array([3.0]), np.array([-5.0]), 1e-6, [0, 0, 0, 0, 0, 2, 3])
    z = np.zeros(5000)
    compare(h, z, z, 1e-6, [0, 0, 0, 0, 0, 1, 8])
    o = np.ones(70000)
    compare(h, o, o, 1e-6, [0, 0, 0, 0, 0, 2, 10])
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    r = h.qdot(e[:0], e[:0], 1e-6, opt=[0, 0, 0, 0, 0, 1, 2])
    assert r["status"] == q.OK and r["flags"] & q.F_ALL_PERF


def test_bins_refused_where_not_supported(h):
    x = dev(np.ones(1000))
    for opt in ([0, 0, 0, 1, 0, 1, 2],     # one-pass reading
                [0, 0, 0, 0, 1, 2, 2],     # guaranteed mode
                [0, 0, 0, 0, 0, 1, 0],     # width 0
                [0, 0, 0, 0, 0, 3, 1]):    # unknown strategy
        with pytest.raises(q.QdotError):
            h.qdot(x, x, 1e-6, opt=opt)
    rp, col, val = workloads.poisson2d_csr(16)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(256, 1))
    with pytest.raises(q.QdotError):
        h.cg(A, b, torch.zeros(256, dtype=torch.float64, device="cuda:0"), 1e-10, 1e-8, 100, 1,
             opt=[0, 0, 0, 0, 0, 1, 2])
