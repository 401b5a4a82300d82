"""GPU parity of CG systems solved inside the batched persistent launch.

Each system must behave as Alg. 4 on that system alone: the iteration count
of the qdot-CG equal to its FP64-dot twin's (the target of the method), and
within one of the oracle's CG (whose FP64 sums are taken in another order:
the stopping test compares a rounded inner product with a threshold, so one
iteration of slack covers a rounding that lands on the other side), the
true residual below the solver tolerance, and the solution close to the
oracle's.  CG systems and qdot instances share the launch without changing
either's results, and the launch replays from a captured graph.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from parity_util import check_instances, host

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu
INT_KEYS = ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status")


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def poisson_system(m, seed, use_qdot, rtol=1e-10, qtol=1e-8, maxit=20000):
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    b = workloads.normal_vector(m * m, seed)
    x = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
    return {"m": m, "csr": (rp, col, val), "A": A, "b_host": b, "b": dev(b), "x": x,
            "args": (A, None, x, rtol, qtol, maxit, use_qdot)}


def as_tuple(s):
    A, _, x, rtol, qtol, maxit, use = s["args"]
    return (A, s["b"], x, rtol, qtol, maxit, use)


SIDES = (16, 32, 45, 64, 100, 140)  # 140^2 = 19600 rows: a gang of two blocks


def test_cg_batched_matches_oracle_and_fp64_twin(h):
    sq = [poisson_system(m, 100 + m, 1) for m in SIDES]
    sf = [poisson_system(m, 100 + m, 0) for m in SIDES]
    res = h.cg_batched([as_tuple(s) for s in sq + sf])
    for i, m in enumerate(SIDES):
        rq, rf = res[i], res[len(SIDES) + i]
        assert rq["status"] == q.OK and rf["status"] == q.OK, (m, rq, rf)
        assert rq["iters"] == rf["iters"], (m, rq["iters"], rf["iters"])
        assert rq["relres_true"] < 1e-9 and rf["relres_true"] < 1e-9, m
        rp, col, val = sq[i]["csr"]
        o = oracle.cg(rp, col, val, sq[i]["b_host"], 1e-10, 1e-8, 20000, 1)
        assert abs(o["iters"] - rq["iters"]) <= 1, (m, o["iters"], rq["iters"])
        xq = sq[i]["x"].cpu().numpy()
        np.testing.assert_allclose(xq, o["x"], rtol=0, atol=1e-7 * np.abs(o["x"]).max())


@pytest.mark.parametrize("opt", [[1, 0, 0, 0], [0, 1, 1, 0]])
def test_cg_batched_options(h, opt):
    # key, score and boundary modes reach every gang: iteration counts within
    # one of the oracle's CG with the same options
    sq = [poisson_system(m, 200 + m, 1) for m in (16, 45, 140)]
    res = h.cg_batched([as_tuple(s) for s in sq], opt=opt)
    for s, r in zip(sq, res):
        rp, col, val = s["csr"]
        o = oracle.cg(rp, col, val, s["b_host"], 1e-10, 1e-8, 20000, 1, opt=opt)
        assert r["status"] == q.OK and o["status"] == oracle.OK, (s["m"], r)
        assert abs(o["iters"] - r["iters"]) <= 1, (s["m"], o["iters"], r["iters"])
        assert r["relres_true"] < 1e-9


def test_cg_batched_equals_single_system_solver(h):
    sys = [poisson_system(m, 7 + m, 1) for m in (32, 140)]
    res = h.cg_batched([as_tuple(s) for s in sys])
    for s, r in zip(sys, res):
        x1 = torch.zeros_like(s["x"])
        r1 = h.cg(s["A"], s["b"], x1, 1e-10, 1e-8, 20000, 1)
        assert abs(r1["iters"] - r["iters"]) <= 1, (s["m"], r1["iters"], r["iters"])


def test_cg_batched_long_rows(h):
    # a random SPD matrix with rows of 6..23 entries (the SpMV tail loop),
    # 20000 rows: a gang of two blocks
    rp, col, val = workloads.random_spd_csr(20000, 6, 3)
    A = q.Csr(rp, col, val)
    bh = workloads.normal_vector(20000, 8)
    x = torch.zeros(20000, dtype=torch.float64, device="cuda:0")
    r = h.cg_batched([(A, dev(bh), x, 1e-10, 1e-8, 2000, 1)])[0]
    o = oracle.cg(rp, col, val, bh, 1e-10, 1e-8, 2000, 1)
    assert r["status"] == q.OK and abs(r["iters"] - o["iters"]) <= 1, (r["iters"], o["iters"])
    np.testing.assert_allclose(x.cpu().numpy(), o["x"], rtol=0, atol=1e-7 * np.abs(o["x"]).max())


def test_cg_batched_statuses_are_per_system(h):
    ok = poisson_system(40, 3, 1)
    short = poisson_system(40, 3, 1, maxit=3)
    perf = poisson_system(24, 4, 1, qtol=1e300)  # every component perforated
    res = h.cg_batched([as_tuple(s) for s in (ok, short, perf)])
    assert res[0]["status"] == q.OK
    assert res[1]["status"] == q.E_MAXIT and res[1]["iters"] == 3
    assert res[2]["status"] == q.E_BREAKDOWN


def ragged(seed, count):
    g = workloads.rng(seed)
    sizes = [70000, 140000] + list(np.rint(10 ** g.uniform(1, 5, count)).astype(int))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    x, y = workloads.log_uniform_pair(int(offsets[-1]), seed + 1)
    tols = np.array([1e-4, 1e-6, 1e-8])[g.integers(0, 3, len(sizes))]
    return offsets, x, y, tols


def check_qdot(res, offsets, x, y, tols):
    for j in range(len(tols)):
        a, b = offsets[j], offsets[j + 1]
        o = oracle.qdot(x[a:b], y[a:b], tols[j])
        for k in INT_KEYS:
            assert res[j][k] == o[k], (j, k)
        if o["status"] == oracle.OK:
            assert abs(res[j]["value"] - o["value"]) <= 1e-13 * oracle.abs_dot(x[a:b], y[a:b])


def test_batch_run_mixes_qdot_instances_and_cg_systems(h):
    offsets, x, y, tols = ragged(11, 40)
    sys = [poisson_system(m, 50 + m, u) for m in (20, 64, 150) for u in (1, 0)]
    xd, yd = dev(x), dev(y)
    off_d = torch.from_numpy(offsets).to("cuda:0")
    out = torch.zeros(len(tols) * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    cg_out = torch.zeros(len(sys) * q.CG_RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.batch_run_async(xd, yd, off_d, offsets, dev(tols), out, [as_tuple(s) for s in sys], cg_out)
    torch.cuda.synchronize()
    check_qdot(q.parse_results(out), offsets, x, y, tols)
    # the instances alone (the launch's kernel without CG items): the same
    # result bytes
    alone = torch.zeros_like(out)
    h.batched_async(xd, yd, off_d, offsets, dev(tols), alone)
    torch.cuda.synchronize()
    assert torch.equal(alone, out)
    cg = q.parse_cg_results(cg_out)
    for i in range(0, len(sys), 2):
        assert cg[i]["status"] == q.OK and cg[i + 1]["status"] == q.OK
        # (qdot, FP64-dot) pairs of the same system
        assert cg[i]["iters"] == cg[i + 1]["iters"], (i, cg[i]["iters"], cg[i + 1]["iters"])
        assert cg[i]["relres_true"] < 1e-9


def test_batch_run_mixes_one_pass_instances_and_cg_systems(h):
    # qdot instances in the one-pass reading next to CG systems (which keep
    # the default reading): the launch's own kernel variant for that mix
    offsets, x, y, tols = ragged(13, 40)
    sys = [poisson_system(m, 70 + m, u) for m in (20, 64, 150) for u in (1, 0)]
    tup = [as_tuple(s) for s in sys]
    xd, yd = dev(x), dev(y)
    off_d = torch.from_numpy(offsets).to("cuda:0")
    print(f"[gpu-case] batch_run one-pass instances={len(tols)} systems={len(sys)}", flush=True)
    cgs = []
    for opt in ([0, 0, 0, 1], None):
        for s in sys:
            s["x"].zero_()
        out = torch.zeros(len(tols) * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
        cg_out = torch.zeros(len(sys) * q.CG_RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
        h.batch_run_async(xd, yd, off_d, offsets, dev(tols), out, tup, cg_out, opt=opt)
        torch.cuda.synchronize()
        cgs.append(q.parse_cg_results(cg_out))
        if opt is None:
            continue
        res = q.parse_results(out)
        for j in range(len(tols)):
            a, b = offsets[j], offsets[j + 1]
            o = oracle.qdot(x[a:b], y[a:b], tols[j], opt=opt)
            for k in INT_KEYS:
                assert res[j][k] == o[k], (j, k)
            if o["status"] == oracle.OK:
                assert abs(res[j]["value"] - o["value"]) <= 1e-13 * oracle.abs_dot(x[a:b], y[a:b])
    # the systems' solves do not depend on the instances' reading
    for a, b in zip(cgs[0], cgs[1]):
        assert a["status"] == b["status"] == q.OK
        assert a["iters"] == b["iters"] and a["relres_true"] == b["relres_true"]
    for i in range(0, len(sys), 2):
        assert cgs[0][i]["iters"] == cgs[0][i + 1]["iters"]


def test_batch_run_graph_replay(h):
    offsets, x, y, tols = ragged(12, 20)
    sys = [poisson_system(m, 60 + m, 1) for m in (24, 90)]
    tup = [as_tuple(s) for s in sys]
    xd, yd = dev(x), dev(y)
    off_d = torch.from_numpy(offsets).to("cuda:0")
    tol_d = dev(tols)
    out = torch.zeros(len(tols) * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    cg_out = torch.zeros(len(sys) * q.CG_RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.batch_run_async(xd, yd, off_d, offsets, tol_d, out, tup, cg_out)
    torch.cuda.synchronize()
    eager, eager_cg = out.clone(), cg_out.clone()
    eager_x = [s["x"].clone() for s in sys]
    h.batch_plan(offsets, tup)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            h.batch_run_async(xd, yd, off_d, offsets, tol_d, out, tup, cg_out)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        cg_out.zero_()
        for s in sys:
            s["x"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        assert torch.equal(cg_out, eager_cg), rep
        for s, ex in zip(sys, eager_x):
            assert torch.equal(s["x"], ex), rep
        h.qdot(xd[:5000], yd[:5000], 1e-6)  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.timeout(600)
def test_full_size_c5_launch(h):
    """The whole batched workload in one launch: 4096 ragged qdot instances
    (n = round(10^U[2,6])) and 256 CG systems (2D Poisson, side
    round(2^U[5,9])).  Every system converges with its FP64-dot twin's
    iteration count; every instance matches the oracle."""
    g = workloads.rng(2025)
    sizes = np.rint(10.0 ** g.uniform(2, 6, 4096)).astype(np.int64)
    offsets = np.zeros(4097, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    tols = np.array([1e-4, 1e-6, 1e-8])[g.integers(0, 3, 4096)]
    total = int(offsets[-1])
    print(f"[gpu-case] batched C5 with 256 CG systems, total={total}", flush=True)
    xd, yd = workloads.log_uniform_pair_torch(total, 2025, "cuda:0")
    gs = workloads.rng(2026)
    sides = np.rint(2.0 ** gs.uniform(5, 9, 256)).astype(np.int64)
    mats, sysq, sysf = {}, [], []
    xs = []
    for k, m in enumerate(sides):
        m = int(m)
        if m not in mats:
            mats[m] = q.Csr(*workloads.poisson2d_csr(m))
        b = dev(workloads.normal_vector(m * m, 3000 + k))
        xq = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
        xf = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
        sysq.append((mats[m], b, xq, 1e-10, 1e-8, 20000, 1))
        sysf.append((mats[m], b, xf, 1e-10, 1e-8, 20000, 0))
    off_d = torch.from_numpy(offsets).to("cuda:0")
    out = torch.zeros(4096 * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    cg_out = torch.zeros(256 * q.CG_RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.batch_run_async(xd, yd, off_d, offsets, dev(tols), out, sysq, cg_out)
    torch.cuda.synchronize()
    cq = q.parse_cg_results(cg_out)
    cf = h.cg_batched(sysf)
    for s in range(256):
        assert cq[s]["status"] == q.OK and cf[s]["status"] == q.OK, s
        assert cq[s]["iters"] == cf[s]["iters"], (s, cq[s]["iters"], cf[s]["iters"])
        assert cq[s]["relres_true"] < 2e-10
    res = q.parse_results(out)
    assert all(r["status"] == q.OK for r in res)
    # every instance against the oracle on that instance alone
    xh, yh = host(xd), host(yd)
    assert check_instances(res, offsets, xh, yh, tols) == 4096


@pytest.mark.parametrize("rows,gmax", [(4096, 64), (1024, 8)])
def test_cg_batched_gang_sizing(rows, gmax):
    # other gang sizes: every system still takes its FP64 twin's iteration
    # count and stays within one of the oracle's
    with q.Qdot(0, load_tuned=False) as hh:
        hh.set_solver_tune(cg_rows_per_block=rows, cg_gang_max=gmax)
        sides = (45, 140, 256)
        sq = [poisson_system(m, 300 + m, 1) for m in sides]
        sf = [poisson_system(m, 300 + m, 0) for m in sides]
        res = hh.cg_batched([as_tuple(s) for s in sq + sf])
        for i, m in enumerate(sides):
            rq, rf = res[i], res[len(sides) + i]
            assert rq["status"] == q.OK and rf["status"] == q.OK, (m, rq, rf)
            assert rq["iters"] == rf["iters"], (m, rq["iters"], rf["iters"])
            rp, col, val = sq[i]["csr"]
            o = oracle.cg(rp, col, val, sq[i]["b_host"], 1e-10, 1e-8, 20000, 1)
            assert abs(o["iters"] - rq["iters"]) <= 1, (m, o["iters"], rq["iters"])
