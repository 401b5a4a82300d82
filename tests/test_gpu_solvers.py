"""GPU CG / power method / SpMV against the oracle and against each other.

SpMV rows are summed in the same order with the same roundings on both
sides, so the product must match bit for bit.  CG with qdot must converge in
the same number of iterations as CG with the FP64 dot (the target of the
CG study) and as the oracle's CG, up to one iteration where rounding of the
two inner products lands near the stopping threshold.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


@pytest.mark.parametrize("m", [7, 64])
def test_spmv_bitwise(h, m):
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    x = workloads.normal_vector(m * m, 3)
    y = torch.empty(m * m, dtype=torch.float64, device="cuda:0")
    h.spmv(A, dev(x), y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y.cpu().numpy(), oracle.spmv(rp, col, val, x))


def test_spmv_bitwise_long_rows(h):
    # rows of 6..23 entries: the unrolled first 8 entries and the tail loop
    rp, col, val = workloads.random_spd_csr(3000, 6, 1)
    A = q.Csr(rp, col, val)
    x = workloads.normal_vector(3000, 4)
    y = torch.empty(3000, dtype=torch.float64, device="cuda:0")
    h.spmv(A, dev(x), y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y.cpu().numpy(), oracle.spmv(rp, col, val, x))


def ragged_csr(n, seed):
    """Random CSR with empty rows and rows longer than the SpMV's staged
    range (2048 products), some straddling row groups of 256."""
    g = workloads.rng(seed)
    lens = g.integers(0, 12, n)
    lens[1000:1300] = 0
    for r, ln in ((5, 2500), (300, 9000), (511, 2049), (512, 2048), (767, 4097), (n - 1, 3000)):
        lens[r] = ln
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(lens, out=rp[1:])
    col = g.integers(0, n, int(rp[-1])).astype(np.int32)
    val = g.standard_normal(int(rp[-1]))
    return rp, col, val


@pytest.fixture
def spmv_blocks(h):
    """Sets the handle's SpMV grid (blocks per CU) for one test."""
    def put(bpc):
        if bpc is not None:
            h.set_solver_tune(spmv_blocks_per_cu=bpc)
    yield put
    h.set_solver_tune()


@pytest.mark.parametrize("bpc", [None, 1])
def test_spmv_bitwise_ragged(h, spmv_blocks, bpc):
    # rows split over several staged ranges keep their order; with one block
    # per CU the 274 row groups are walked grid-stride
    n = 70000
    rp, col, val = ragged_csr(n, 11)
    spmv_blocks(bpc)
    A = q.Csr(rp, col, val)
    x = workloads.normal_vector(n, 12)
    y = torch.empty(n, dtype=torch.float64, device="cuda:0")
    print(f"[gpu-case] spmv ragged n={n} nnz={rp[-1]} bpc={bpc}", flush=True)
    h.spmv(A, dev(x), y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y.cpu().numpy(), oracle.spmv(rp, col, val, x))


def test_cg_long_rows(h):
    rp, col, val = workloads.random_spd_csr(5000, 6, 2)
    A = q.Csr(rp, col, val)
    b = workloads.normal_vector(5000, 7)
    for use in (1, 0):
        x = torch.zeros(5000, dtype=torch.float64, device="cuda:0")
        r = h.cg(A, dev(b), x, 1e-10, 1e-8, 2000, use)
        o = oracle.cg(rp, col, val, b, 1e-10, 1e-8, 2000, use)
        assert r["status"] == q.OK and o["status"] == oracle.OK
        assert abs(r["iters"] - o["iters"]) <= 1, (use, r["iters"], o["iters"])
        assert r["relres_true"] < 1e-9
        np.testing.assert_allclose(x.cpu().numpy(), o["x"], rtol=0,
                                   atol=1e-7 * np.abs(o["x"]).max())


@pytest.mark.parametrize("m", [32, 64, 128])
def test_cg_iteration_parity(h, m):
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    b = workloads.normal_vector(m * m, 5)
    bd = dev(b)
    xq = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    xf = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    rq = h.cg(A, bd, xq, 1e-10, 1e-8, 20000, 1, trace=True)
    rf = h.cg(A, bd, xf, 1e-10, 1e-8, 20000, 0)
    assert rq["status"] == q.OK and rf["status"] == q.OK
    # the target of the method: qdot-CG takes the FP64-dot CG's iteration count
    assert rq["iters"] == rf["iters"], (rq["iters"], rf["iters"])
    assert rq["relres_true"] < 1e-9 and rf["relres_true"] < 1e-9
    oq = oracle.cg(rp, col, val, b, 1e-10, 1e-8, 20000, 1, want_trace=True)
    assert abs(oq["iters"] - rq["iters"]) <= 1, (oq["iters"], rq["iters"])
    # the first qdot (r0 = b exactly) classifies identically
    t0, o0 = rq["trace"][0], oq["trace"][0]
    for k in ("count", "n_bins", "e_max", "e_min", "t", "flags"):
        assert t0[k] == o0[k], k
    assert abs(t0["value"] - o0["value"]) <= 1e-13 * float(np.dot(b, b))
    # the solutions agree to the solver tolerance
    np.testing.assert_allclose(xq.cpu().numpy(), oq["x"], rtol=0,
                               atol=1e-7 * np.abs(oq["x"]).max())


ONE_PASS = [0, 0, 0, 1]


@pytest.mark.parametrize("m", [32, 128])
def test_cg_one_pass_mode(h, m):
    # every inner product by the one-pass qdot: the oracle's CG with the same
    # mode (first product bit for bit; iteration counts within one), and the
    # FP64-dot CG's iteration count
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    b = workloads.normal_vector(m * m, 5)
    print(f"[gpu-case] cg one-pass m={m}", flush=True)
    x = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    r = h.cg(A, dev(b), x, 1e-10, 1e-8, 20000, 1, opt=ONE_PASS, trace=True)
    o = oracle.cg(rp, col, val, b, 1e-10, 1e-8, 20000, 1, opt=ONE_PASS, want_trace=True)
    xf = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    rf = h.cg(A, dev(b), xf, 1e-10, 1e-8, 20000, 0)
    assert r["status"] == q.OK and o["status"] == oracle.OK
    assert abs(r["iters"] - o["iters"]) <= 1 and r["iters"] == rf["iters"]
    assert r["relres_true"] < 1e-9
    t0, o0 = r["trace"][0], o["trace"][0]
    for k in ("count", "n_zero", "n_bins", "e_max", "e_min", "t", "flags", "passes"):
        assert t0[k] == o0[k], k
    assert abs(t0["value"] - o0["value"]) <= 1e-13 * float(np.dot(b, b))
    np.testing.assert_allclose(x.cpu().numpy(), o["x"], rtol=0, atol=1e-7 * np.abs(o["x"]).max())


@pytest.mark.parametrize("opt", [[1, 0, 0, 0], [0, 1, 1, 0], [1, 1, 1, 1]])
def test_cg_options(h, opt):
    # key, score and boundary modes (and the one-pass reading) through the
    # gang: the first inner product bit for bit, the iteration count within
    # one of the oracle's CG with the same options
    m = 32
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    b = workloads.normal_vector(m * m, 16)
    print(f"[gpu-case] cg options {opt}", flush=True)
    x = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    r = h.cg(A, dev(b), x, 1e-10, 1e-8, 20000, 1, opt=opt, trace=True)
    o = oracle.cg(rp, col, val, b, 1e-10, 1e-8, 20000, 1, opt=opt, want_trace=True)
    assert r["status"] == q.OK and o["status"] == oracle.OK
    assert abs(r["iters"] - o["iters"]) <= 1
    t0, o0 = r["trace"][0], o["trace"][0]
    for k in ("count", "n_zero", "n_bins", "e_max", "e_min", "t", "flags", "passes"):
        assert t0[k] == o0[k], k
    assert abs(t0["value"] - o0["value"]) <= 1e-13 * float(np.dot(b, b))


@pytest.mark.parametrize("opt", [[1, 0, 0, 0], [0, 1, 1, 0]])
def test_power_method_options(h, opt):
    m = 12
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, val)
    x0 = workloads.unit_vector(m ** 3, 17)
    r = h.power(A, dev(x0), 80, 1e-6, 1, opt=opt)
    o = oracle.power(rp, col, val, x0, 80, 1e-6, 1, opt=opt)
    assert r["status"] == q.OK
    np.testing.assert_allclose(r["trace"], o["trace"], rtol=1e-9, atol=0)


def test_cg_one_pass_repeatable_and_rejected(h):
    # the gang's one-pass tables are left clean: a second solve on the same
    # handle is bitwise the first; an inadmissible tolerance is refused
    m = 64
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(m * m, 6))
    xs = []
    for _ in range(2):
        x = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
        r = h.cg(A, b, x, 1e-10, 1e-8, 20000, 1, opt=ONE_PASS)
        assert r["status"] == q.OK
        xs.append(x.cpu().numpy())
    np.testing.assert_array_equal(xs[0], xs[1])
    with pytest.raises(q.QdotError):
        h.cg(A, b, torch.zeros(m * m, dtype=torch.float64, device="cuda:0"), 1e-10, 1e-300,
             100, 1, opt=ONE_PASS)


@pytest.mark.timeout(300)
def test_full_size_cg_one_pass(h):
    m = 1024
    print(f"[gpu-case] CG one-pass Poisson {m}^2", flush=True)
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(m * m, 3))
    x = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    r = h.cg(A, b, x, 1e-10, 1e-8, 20000, 1, opt=ONE_PASS)
    xf = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    rf = h.cg(A, b, xf, 1e-10, 1e-8, 20000, 0)
    assert r["status"] == q.OK and r["relres_true"] < 2e-10
    assert r["iters"] == rf["iters"], (r["iters"], rf["iters"])


def test_cg_breakdown_when_all_perforated(h):
    rp, col, val = workloads.poisson2d_csr(16)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(256, 6))
    x = torch.zeros(256, dtype=torch.float64, device="cuda:0")
    r = h.cg(A, b, x, 1e-10, 1e300, 100, 1)
    assert r["status"] == q.E_BREAKDOWN


def test_cg_maxit(h):
    rp, col, val = workloads.poisson2d_csr(64)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(4096, 7))
    x = torch.zeros(4096, dtype=torch.float64, device="cuda:0")
    r = h.cg(A, b, x, 1e-14, 1e-8, 10, 1)
    assert r["status"] == q.E_MAXIT and r["iters"] == 10


@pytest.mark.parametrize("first", ["power", "cg"])
def test_power_and_cg_share_one_handle(first):
    # the power method keeps two scratch vectors, CG three: whichever runs
    # first, the other must grow the scratch and give the same results as on
    # a fresh handle
    m = 12
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, val)
    n = m ** 3
    b = workloads.normal_vector(n, 11)
    x0 = workloads.unit_vector(n, 12)

    def run_power(hh):
        return hh.power(A, dev(x0), 50, 1e-6, 1)["trace"]

    def run_cg(hh):
        x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        r = hh.cg(A, dev(b), x, 1e-10, 1e-8, 500, 1)
        return r["iters"], x.cpu().numpy()

    with q.Qdot(0) as fresh:
        p_ref = run_power(fresh)
    with q.Qdot(0) as fresh:
        it_ref, x_ref = run_cg(fresh)
    with q.Qdot(0) as hh:
        if first == "power":
            p_got = run_power(hh)
            it_got, x_got = run_cg(hh)
        else:
            it_got, x_got = run_cg(hh)
            p_got = run_power(hh)
    np.testing.assert_array_equal(p_got, p_ref)
    assert it_got == it_ref
    np.testing.assert_array_equal(x_got, x_ref)


@pytest.mark.parametrize("m", [6, 16])
def test_power_method(h, m):
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, val)
    x0 = workloads.unit_vector(m ** 3, 8)
    iters = 200
    lam_max = 6.0 + 6.0 * math.cos(math.pi / (m + 1))
    for use_qdot in (1, 0):
        xd = dev(x0)
        r = h.power(A, xd, iters, 1e-6, use_qdot)
        o = oracle.power(rp, col, val, x0, iters, 1e-6, use_qdot)
        assert r["status"] == q.OK
        np.testing.assert_allclose(r["trace"], o["trace"], rtol=1e-9, atol=0)
        assert r["lambda"] <= lam_max * (1 + 1e-12)


def test_power_method_grid_stride(h, spmv_blocks):
    # 110592 rows on one block per CU: the SpMV walks two row groups in some
    # blocks; both inner products share their launches (x.w and w.w)
    m = 48
    rp, col, val = workloads.laplacian3d_csr(m)
    spmv_blocks(1)
    A = q.Csr(rp, col, val)
    x0 = workloads.unit_vector(m ** 3, 9)
    print(f"[gpu-case] power grid-stride m={m}", flush=True)
    for use_qdot in (1, 0):
        xd = dev(x0)
        r = h.power(A, xd, 60, 1e-6, use_qdot)
        o = oracle.power(rp, col, val, x0, 60, 1e-6, use_qdot)
        assert r["status"] == q.OK
        np.testing.assert_allclose(r["trace"], o["trace"], rtol=1e-9, atol=0)
        # the last iterate: each iteration's SpMV gathers w / sqrt(c) itself
        # and writes x, and the final update writes the last one
        np.testing.assert_allclose(xd.cpu().numpy(), o["x"], rtol=0, atol=1e-9)


@pytest.mark.parametrize("m,opt", [(16, None), (40, None), (128, None), (16, [0, 0, 0, 0, 1])])
def test_power_pair_matches_separate_calls(h, m, opt):
    # one iteration: lambda = x0 . A x0 and c = w . w from the paired
    # launches equal two separate qdot calls (same classes, same pass-2
    # blocks), and x = w / sqrt(c)
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, val)
    x0 = workloads.unit_vector(m ** 3, 14)
    print(f"[gpu-case] power pair m={m} opt={opt}", flush=True)
    xd = dev(x0)
    r = h.power(A, xd, 1, 1e-6, 1, opt=opt)
    w = torch.empty_like(xd)
    h.spmv(A, dev(x0), w)
    lam = h.qdot(dev(x0), w, 1e-6, opt=opt)
    c = h.qdot(w, w, 1e-6, opt=opt)
    assert r["status"] == q.OK
    assert r["trace"][0] == lam["value"], (r["trace"][0], lam["value"])
    np.testing.assert_allclose(xd.cpu().numpy(), w.cpu().numpy() / math.sqrt(c["value"]),
                               rtol=4e-16, atol=0)


def test_power_method_zero_iterations(h):
    rp, col, val = workloads.laplacian3d_csr(6)
    x0 = workloads.unit_vector(216, 15)
    xd = dev(x0)
    r = h.power(q.Csr(rp, col, val), xd, 0, 1e-6, 1)
    assert r["status"] == q.OK and r["lambda"] == 0.0
    np.testing.assert_array_equal(xd.cpu().numpy(), x0)


def test_power_method_breakdown(h):
    # A = 0: w = 0, so c = w.w = 0 at the first iteration.  The later
    # iterations (up to the first control read, after 64) run on a broken
    # state; the handle is still sound afterwards.
    m = 8
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, np.zeros_like(val))
    x0 = workloads.unit_vector(m ** 3, 10)
    for use_qdot in (1, 0):
        r = h.power(A, dev(x0), 100, 1e-6, use_qdot)
        o = oracle.power(rp, col, np.zeros_like(val), x0, 100, 1e-6, use_qdot)
        assert r["status"] == q.E_BREAKDOWN and o["status"] == oracle.E_BREAKDOWN
    x, y = workloads.log_uniform_pair(5000, 13, -20.0, 20.0)
    rr = h.qdot(dev(x), dev(y), 1e-6)
    oo = oracle.qdot(x, y, 1e-6)
    assert rr["count"] == oo["count"] and rr["flags"] == oo["flags"]
    rl = h.power(q.Csr(rp, col, val), dev(x0), 20, 1e-6, 1)
    ol = oracle.power(rp, col, val, x0, 20, 1e-6, 1)
    np.testing.assert_allclose(rl["trace"], ol["trace"], rtol=1e-9, atol=0)


@pytest.mark.timeout(300)
def test_full_size_cg_poisson_1024(h):
    """The CG workload at its full size (2D Poisson 1024^2, b ~ N(0,1), qdot
    tol 1e-8, stop at 1e-10): qdot-CG needs the FP64-dot CG's iteration
    count and reaches the true residual."""
    m = 1024
    print(f"[gpu-case] CG Poisson {m}^2", flush=True)
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(m * m, 3))
    res = {}
    for use in (1, 0):
        x = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
        res[use] = h.cg(A, b, x, 1e-10, 1e-8, 20000, use)
        assert res[use]["status"] == q.OK
        assert res[use]["relres_true"] < 2e-10
    assert res[1]["iters"] == res[0]["iters"], (res[1]["iters"], res[0]["iters"])


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.timeout(300)
def test_full_size_power_trace_matches_oracle(h):
    """The power-method workload at its full size (3D Laplacian 128^3, unit
    N(0,1) start seed 4, 500 iterations, both inner products by qdot at tol
    1e-6) against the oracle's run stored by make_solver_goldens.py: every
    lambda within rtol 1e-9 (the FP64 sums of the two sides are taken in
    other orders, so x_k may differ in its last bits), the per-class counts
    of both inner products of iteration 0 bit for bit (same x_0, and w_0 =
    A x_0 is formed by the same rounded operations on both sides), and those
    of every 50th iteration within 1e-5 n in total.  The FP64-dot run
    against the oracle's exact-dot run, lambda within rtol 1e-9."""
    m, iters = 128, 500
    with open(os.path.join(GOLDEN, "power_laplacian3d_128.json")) as f:
        gold = json.load(f)
    assert gold["iters"] == iters and gold["qtol"] == 1e-6
    print(f"[gpu-case] power Laplacian {m}^3 trace vs oracle", flush=True)
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, val)
    x0 = workloads.unit_vector(m ** 3, 4)
    r = h.power(A, dev(x0), iters, 1e-6, 1, results=True)
    assert r["status"] == q.OK
    lam_o = np.array([float.fromhex(v) for v in gold["qdot"]["lambda_hex"]])
    np.testing.assert_allclose(r["trace"], lam_o, rtol=1e-9, atol=0)
    n = m ** 3
    for k, (ca, cb) in gold["qdot"]["counts_every_50"].items():
        k = int(k)
        ga, gb = r["results"][2 * k]["count"], r["results"][2 * k + 1]["count"]
        if k == 0:
            assert ga == ca and gb == cb, (k, ga, ca, gb, cb)
        else:
            diff = sum(abs(a - b) for a, b in zip(ga + gb, ca + cb))
            assert diff <= 1e-5 * n, (k, ga, ca, gb, cb)
    r0 = h.power(A, dev(x0), iters, 1e-6, 0)
    assert r0["status"] == q.OK
    lam_e = np.array([float.fromhex(v) for v in gold["exact_dot"]["lambda_hex"]])
    np.testing.assert_allclose(r0["trace"], lam_e, rtol=1e-9, atol=0)
    print(f"[gpu-case] |lambda_500 qdot - oracle| = {abs(r['lambda'] - lam_o[-1]):.3e}, "
          f"|qdot - FP64| = {abs(r['lambda'] - r0['lambda']):.3e}", flush=True)


@pytest.mark.timeout(300)
def test_full_size_power_laplacian_128(h):
    """The power-method workload at its full size (3D Laplacian 128^3, 500
    iterations, qdot tol 1e-6): the eigenvalue estimate agrees with the
    FP64-dot run and stays below the closed-form largest eigenvalue."""
    m = 128
    print(f"[gpu-case] power Laplacian {m}^3", flush=True)
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, val)
    x0 = workloads.unit_vector(m ** 3, 4)
    lam = {}
    for use in (1, 0):
        r = h.power(A, dev(x0), 500, 1e-6, use, trace=False)
        assert r["status"] == q.OK
        lam[use] = r["lambda"]
    lam_max = 6.0 + 6.0 * math.cos(math.pi / (m + 1))
    assert abs(lam[1] - lam[0]) <= 1e-9 * lam[0]
    assert lam[0] <= lam_max * (1 + 1e-12) and lam[0] > 0.99 * lam_max


@pytest.mark.parametrize("m,opt", [(16, None), (64, None), (40, [1, 1, 1, 0]),
                                   (32, [0, 0, 0, 0, 1])])
def test_power_scan_in_spmv_is_the_same_method(h, m, opt):
    # pass 1 of the paired inner products taken inside the SpMV (after the
    # first iteration) gives every iteration's results bit for bit as the
    # separate pass-1 kernel does: lambda trace, qdot results, final x
    rp, col, val = workloads.laplacian3d_csr(m)
    A = q.Csr(rp, col, val)
    x0 = workloads.unit_vector(m ** 3, 21)
    out = {}
    for fused in (0, 1):
        print(f"[gpu-case] power scan in SpMV={fused} m={m} opt={opt}", flush=True)
        h.set_solver_tune(power_scan_in_spmv=fused)
        xd = dev(x0)
        out[fused] = (h.power(A, xd, 40, 1e-6, 1, opt=opt, results=True), xd.cpu().numpy())
    h.set_solver_tune()
    (r0, x0d), (r1, x1d) = out[0], out[1]
    assert r0["status"] == r1["status"] == q.OK
    np.testing.assert_array_equal(r0["trace"], r1["trace"])
    assert r0["results"] == r1["results"]
    np.testing.assert_array_equal(x0d, x1d)
