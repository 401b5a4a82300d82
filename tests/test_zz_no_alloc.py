"""GPU test of the allocation-free entry point qdot_noalloc_async.

It runs qdot_async's kernels over a fixed device array instead of a
handle's workspace, so its results must equal qdot_async's: integer
outputs bit for bit, the value within 1e-13 * sum |x_i y_i| (the launch
shapes may differ from a handle's tuned ones).  Two calls in a row, the
second on a smaller input, check that what the first call leaves in the
shared array does not leak into the second; the one-pass and guaranteed
modes use the array's per-bin tables and saved histogram.
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _noalloc(xd, yd, tol, opt=None):
    out = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    q.qdot_noalloc_async(xd, yd, tol, out, opt=opt)
    torch.cuda.synchronize()
    return q.parse_results(out)[0]


def _same(r, ref, scale):
    for k in INT_KEYS:
        assert r[k] == ref[k], (k, r[k], ref[k])
    assert abs(r["value"] - ref["value"]) <= VALUE_TOL * scale, (r["value"], ref["value"])
    for c in range(3):
        assert abs(r["part"][c] - ref["part"][c]) <= VALUE_TOL * scale, c


@pytest.mark.parametrize("opt", [None, [0, 0, 0, 1], [0, 0, 0, 0, 1], [1, 1, 1, 0]],
                         ids=["default", "one-pass", "guaranteed", "sum-key-raw-nonstrict"])
def test_noalloc_matches_qdot_async_twice(opt):
    h = q.Qdot(0)
    try:
        # first a large call, then a smaller one with other data and tolerance
        for n, seed, tol in ((1 << 22) + 777, 11, 1e-6, ), ((1 << 16) + 5, 12, 1e-9):
            print(f"[gpu-case] noalloc n={n} seed={seed} tol={tol} opt={opt}", flush=True)
            x, y = workloads.log_uniform_pair(n, seed)
            xd, yd = _dev(x), _dev(y)
            r = _noalloc(xd, yd, tol, opt)
            ref = h.qdot(xd, yd, tol, opt=opt)
            assert r["status"] == q.OK
            _same(r, ref, oracle.abs_dot(x, y))
    finally:
        h.close()


def test_noalloc_cancelling_guaranteed_then_small():
    # the guaranteed mode reselects on this input (a second sweep through
    # the array's partials); the next call must start from a clean state
    h = q.Qdot(0)
    try:
        xc, yc = workloads.cancelling_pair(50000, 700, 3e-4)
        x2, y2 = workloads.log_uniform_pair(3001, 5)
        for x, y, tol, opt in ((xc, yc, 1e-4, [0, 0, 0, 0, 1]), (x2, y2, 1e-6, None)):
            print(f"[gpu-case] noalloc n={len(x)} tol={tol} opt={opt}", flush=True)
            xd, yd = _dev(x), _dev(y)
            r = _noalloc(xd, yd, tol, opt)
            ref = h.qdot(xd, yd, tol, opt=opt)
            _same(r, ref, oracle.abs_dot(x, y))
            for k in ("e_ref", "passes"):
                assert r[k] == ref[k], (k, r[k], ref[k])
    finally:
        h.close()


def test_noalloc_edge_cases():
    # n = 0, a non-finite input (status in the result), and host-side
    # argument errors, which return before anything is enqueued
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    r = _noalloc(e[:0], e[:0], 1e-6)
    assert r["status"] == q.OK and r["value"] == 0.0 and r["flags"] & q.F_ALL_PERF
    x = torch.ones(1000, dtype=torch.float64, device="cuda:0")
    x[17] = float("inf")
    r = _noalloc(x, x, 1e-6)
    assert r["status"] == q.E_NONFINITE
    out = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(q.QdotError):
        q.qdot_noalloc_async(x, x, -1.0, out)
    with pytest.raises(q.QdotError):
        q.qdot_noalloc_async(x, x, 1e-6, out, opt=[0, 0, 0, 0, 7])
    # the state after the rejected calls and the non-finite one is clean
    y = torch.linspace(1.0, 2.0, 1000, dtype=torch.float64, device="cuda:0")
    r = _noalloc(y, y, 1e-6)
    h = q.Qdot(0)
    try:
        ref = h.qdot(y, y, 1e-6)
    finally:
        h.close()
    yy = y.cpu().numpy()
    _same(r, ref, oracle.abs_dot(yy, yy))


def test_noalloc_graph_replay():
    # recorded under graph capture (no allocation inside the call), replayed
    # with eager calls between the replays; every replay equals the eager call
    n, tol = (1 << 20) + 3, 1e-6
    x, y = workloads.log_uniform_pair(n, 21)
    xd, yd = _dev(x), _dev(y)
    ref = _noalloc(xd, yd, tol)
    out = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        q.qdot_noalloc_async(xd, yd, tol, out, stream=s)  # warm (not captured)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        q.qdot_noalloc_async(xd, yd, tol, out, stream=s)
    x2, y2 = workloads.log_uniform_pair(5000, 22)
    x2d, y2d = _dev(x2), _dev(y2)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        r = q.parse_results(out)[0]
        assert r["value"] == ref["value"] and r["count"] == ref["count"]
        _noalloc(x2d, y2d, 1e-8)  # eager work between replays
