"""GPU parity of the guaranteed-eps mode (guard_mode 1, Thm 3.4) inside the
batched persistent launch.

Small instances are certified (or selected again and swept again) by the
block that runs them; a large instance, split into pass-1 and pass-2
chunks, by the block that finishes its last pass-2 chunk, which sweeps the
instance alone after a reselection.  Every instance must give what the
oracle's guaranteed mode gives for it alone: integer outputs (counts,
flags, e_ref, passes included) bit for bit, value and parts within
1e-13 * sum |x_i y_i|, bound_rel within 1e-12 relative, the lower bound
within the same value tolerance.  CG systems in the launch take the
guaranteed inner products of the single-system solver.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
import parity_util

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu
VALUE_TOL = 1e-13
GUARD = [0, 0, 0, 0, 1]
INT_KEYS = ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status", "e_ref",
            "passes")


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def guard_batch(seed):
    """Cancelling instances (reselections) and log-uniform ones (mostly
    certified), small and large (over the default 131072-component chunk),
    plus an empty, an all-zero, a one-sign and a non-finite instance."""
    g = workloads.rng(seed)
    xs, ys, tols = [], [], []
    specs = [(3000, "c"), (40000, "c"), (200000, "c"), (300001, "c"), (70000, "l"),
             (300007, "l"), (0, "z"), (5000, "z"), (20000, "b"), (9000, "n"), (131072, "c"),
             (131073, "l"), (1, "l"), (777, "c")]
    for k, (n, kind) in enumerate(specs):
        if kind == "c":
            x, y = workloads.cancelling_pair(max(n, 2), seed + k, 10.0 ** g.uniform(-7, -2))
        elif kind == "l":
            x, y = workloads.log_uniform_pair(n, seed + k)
        elif kind == "b":
            x, y = workloads.paper_dist_b(n, 9.0, seed + k)
        elif kind == "n":
            x, y = workloads.log_uniform_pair(n, seed + k)
            x[n // 3] = np.nan
        else:
            x, y = np.zeros(n), np.zeros(n)
        xs.append(x[:n])
        ys.append(y[:n])
        tols.append(float([1e-6, 1e-4, 1e-8, 1e-3][k % 4]))
    offsets = np.zeros(len(xs) + 1, dtype=np.int64)
    np.cumsum([len(v) for v in xs], out=offsets[1:])
    return offsets, np.concatenate(xs), np.concatenate(ys), np.array(tols)


def same(a: list, b: list):
    """Result lists equal field by field (a NaN value equals a NaN)."""
    assert len(a) == len(b)
    for j, (ra, rb) in enumerate(zip(a, b)):
        for k in ra:
            va, vb = ra[k], rb[k]
            if isinstance(va, float) and va != va:
                assert vb != vb, (j, k)
            else:
                assert va == vb, (j, k, va, vb)


def check(res, offsets, x, y, tols):
    def one(j):
        a, b = int(offsets[j]), int(offsets[j + 1])
        return oracle.qdot(x[a:b], y[a:b], float(tols[j]), opt=GUARD)

    outs = parity_util.parallel({j: (lambda j=j: one(j)) for j in range(len(tols))})
    reselected_large = 0
    for j in range(len(tols)):
        a, b = int(offsets[j]), int(offsets[j + 1])
        r, o = res[j], outs[j]
        for k in INT_KEYS:
            assert r[k] == o[k], (j, b - a, k, r[k], o[k])
        if o["status"] != oracle.OK:
            assert r["value"] != r["value"], j  # an error result: NaN, the rest 0
            continue
        scale = oracle.abs_dot(x[a:b], y[a:b])
        assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale, (j, r["value"], o["value"])
        for c in range(3):
            assert abs(r["part"][c] - o["part"][c]) <= VALUE_TOL * scale, (j, c)
        assert abs(r["bound_rel"] - o["bound_rel"]) <= 1e-12 * abs(o["bound_rel"]), j
        assert abs(r["lower"] - o["lower"]) <= VALUE_TOL * scale + 1e-12 * abs(o["lower"]), j
        if r["flags"] & q.F_RESELECTED and b - a > 131072:
            reselected_large += 1
    return reselected_large


def test_batched_guard_matches_oracle(h):
    offsets, x, y, tols = guard_batch(500)
    print(f"[gpu-case] batched guard: {len(tols)} instances, {offsets[-1]} components",
          flush=True)
    res = h.batched(dev(x), dev(y), offsets, tols, opt=GUARD)
    flags = [r["flags"] for r in res]
    assert any(f & q.F_RESELECTED for f in flags) and any(f & q.F_GUARANTEED for f in flags)
    assert check(res, offsets, x, y, tols) >= 1


def test_batched_guard_repeat_and_plain_launch_after(h):
    # the guarded launch leaves the plan's counters and histograms clean:
    # a second guarded launch and a plain launch on the same layout agree
    offsets, x, y, tols = guard_batch(501)
    xd, yd = dev(x), dev(y)
    r1 = h.batched(xd, yd, offsets, tols, opt=GUARD)
    r2 = h.batched(xd, yd, offsets, tols, opt=GUARD)
    same(r1, r2)
    plain = h.batched(xd, yd, offsets, tols)
    parity_util.check_instances(plain, offsets, x, y, tols)


def test_batched_guard_graph_replay(h):
    offsets, x, y, tols = guard_batch(502)
    xd, yd = dev(x), dev(y)
    eager = h.batched(xd, yd, offsets, tols, opt=GUARD)
    off_d = torch.from_numpy(offsets).to("cuda:0")
    tol_d = dev(tols)
    out = torch.zeros(len(tols) * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.batch_plan(offsets, [], opt=GUARD)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            h.batched_async(xd, yd, off_d, offsets, tol_d, out, opt=GUARD)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        same(q.parse_results(out), eager)
        h.qdot(xd[:5000], yd[:5000], 1e-6)  # eager work between replays
        torch.cuda.synchronize()


def test_batched_guard_cg_systems(h):
    # CG systems in a guarded launch: every system converges with its
    # FP64-dot twin's iteration count, and within one of the single-system
    # guaranteed solver's
    systems, twins, singles = [], [], []
    for m in (16, 45, 140):
        rp, col, val = workloads.poisson2d_csr(m)
        A = q.Csr(rp, col, val)
        b = dev(workloads.normal_vector(m * m, 600 + m))
        systems.append((A, b, torch.zeros(m * m, dtype=torch.float64, device="cuda:0"),
                        1e-10, 1e-8, 20000, 1))
        twins.append((A, b, torch.zeros(m * m, dtype=torch.float64, device="cuda:0"),
                      1e-10, 1e-8, 20000, 0))
        x1 = torch.zeros(m * m, dtype=torch.float64, device="cuda:0")
        singles.append(h.cg(A, b, x1, 1e-10, 1e-8, 20000, 1, opt=GUARD))
    res = h.cg_batched(systems + twins, opt=GUARD)
    k = len(systems)
    for i in range(k):
        rq, rf = res[i], res[k + i]
        assert rq["status"] == q.OK and rf["status"] == q.OK, (rq, rf)
        assert rq["iters"] == rf["iters"], (rq["iters"], rf["iters"])
        assert abs(rq["iters"] - singles[i]["iters"]) <= 1
        assert rq["relres_true"] < 1e-9


def test_batch_run_guard_instances_and_systems(h):
    offsets, x, y, tols = guard_batch(503)
    xd, yd = dev(x), dev(y)
    rp, col, val = workloads.poisson2d_csr(64)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(64 * 64, 604))
    xs = torch.zeros(64 * 64, dtype=torch.float64, device="cuda:0")
    off_d = torch.from_numpy(offsets).to("cuda:0")
    tol_d = dev(tols)
    out = torch.zeros(len(tols) * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    cg_out = torch.zeros(q.CG_RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    sys = [(A, b, xs, 1e-10, 1e-8, 20000, 1)]
    h.batch_run_async(xd, yd, off_d, offsets, tol_d, out, sys, cg_out, opt=GUARD)
    torch.cuda.synchronize()
    res = q.parse_results(out)
    same(res, h.batched(xd, yd, offsets, tols, opt=GUARD))
    check(res, offsets, x, y, tols)
