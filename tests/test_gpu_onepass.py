"""GPU parity of the one-pass mode (accum_mode 1) through the C ABI.

The one-pass schedule reads x and y once: while it builds the exponent
histogram it also forms, for the bins near the running maximum key, the
candidate sums of every precision, and picks each kept bin's class after
the cutoff.  Its classes and counts are those of the default mode; its
value is the oracle's one-pass reading (the same leaves summed exactly,
rounded once).  Integer outputs must match bit for bit, the value within
1e-13 * sum |x_i y_i|, and because the candidate sums are exact the value
must not depend on launch shape, run or component order.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu

VALUE_TOL = 1e-13
S1 = [0, 0, 0, 1]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")
INT_KEYS = ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status")


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def compare_s1(h, x, y, tol, opt=S1, xd=None, yd=None):
    xd = dev(x) if xd is None else xd
    yd = dev(y) if yd is None else yd
    r = h.qdot(xd, yd, tol, opt=opt)
    o = oracle.qdot(x, y, tol, opt=opt)
    for k in INT_KEYS:
        assert r[k] == o[k], (k, r[k], o[k])
    if o["status"] != oracle.OK:
        return r, o
    scale = oracle.abs_dot(x, y)
    assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale, (r["value"], o["value"], scale)
    for c in range(3):
        assert abs(r["part"][c] - o["part"][c]) <= VALUE_TOL * scale, c
    assert abs(r["bound_rel"] - o["bound_rel"]) <= 1e-12 * abs(o["bound_rel"])
    return r, o


def _golden_inputs(case):
    if "x" in case:
        x = np.array([float.fromhex(s) for s in case["x"]])
        y = np.array([float.fromhex(s) for s in case["y"]])
        return x, y, float(case["tol"])
    if "ones" in case:
        n = case["ones"]
        return np.ones(n), np.ones(n), float(case["tol"])
    n = 4160
    x = np.zeros(n)
    y = np.ones(n)
    x[0] = 1.0
    x[64:4158] = 2.0 ** -24
    if case["name"] == "tile_tree_rounds":
        x[1] = x[3] = 2.0 ** -24
    else:
        x[2] = x[3] = 2.0 ** -24
    return x, y, 2.0 ** -20


@pytest.mark.parametrize("name", [c["name"] for c in json.load(open(GOLDEN))["cases"]])
def test_golden_examples_one_pass(h, name):
    case = next(c for c in json.load(open(GOLDEN))["cases"] if c["name"] == name)
    x, y, tol = _golden_inputs(case)
    r, _ = compare_s1(h, x, y, tol)
    v = case["expect"]["value_s1"]
    want = eval(v.replace("2**", "Fraction(2)**"), {"Fraction": Fraction}) \
        if isinstance(v, str) else Fraction(v)
    assert Fraction(r["value"]) == want


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10])
@pytest.mark.parametrize("seed", [1, 2])
def test_c1_law_n1e5(h, tol, seed):
    x, y = workloads.log_uniform_pair(100000, seed)
    compare_s1(h, x, y, tol)


@pytest.mark.parametrize("n", [0, 1, 3, 63, 64, 65, 1023, 1025, 4097, 100003, (1 << 20) + 7])
def test_ragged_lengths(h, n):
    x, y = workloads.log_uniform_pair(n, 100 + n % 97)
    compare_s1(h, x, y, 1e-6)


@pytest.mark.parametrize("opt", [[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 1], [1, 1, 1, 1]])
def test_options(h, opt):
    x, y = workloads.log_uniform_pair(60000, 7)
    compare_s1(h, x, y, 1e-6, opt=opt)


@pytest.mark.parametrize("law,t", [("A", 20), ("A", 100), ("B", 6), ("B", 30)])
def test_paper_distributions(h, law, t):
    gen = workloads.paper_dist_a if law == "A" else workloads.paper_dist_b
    x, y = gen(50000, t, 11)
    for tol in (1e-4, 1e-8):
        compare_s1(h, x, y, tol)


def test_window_slides_and_deep_windows(h):
    g = workloads.rng(12)
    n = 300000
    # magnitudes rising along the vector: every block's maximum key keeps
    # moving up, so the bin window slides many times
    u = np.sort(g.uniform(-30, 30, n))
    x = np.where(g.random(n) < 0.5, -1.0, 1.0) * 10.0 ** u
    y = 10.0 ** g.uniform(-2, 2, n)
    compare_s1(h, x, y, 1e-6)
    compare_s1(h, x[::-1].copy(), y[::-1].copy(), 1e-6)
    # a tiny tolerance keeps bins about 160 below e_max, close to the window
    x2, y2 = workloads.log_uniform_pair(100000, 13, lo=-60, hi=60)
    r, _ = compare_s1(h, x2, y2, 1e-40)
    assert r["count"][oracle.PERF] < 100000


def test_edge_cases(h):
    compare_s1(h, np.zeros(1000), np.ones(1000), 1e-6)
    x = np.ones(5000)
    x[::7] = 0.0
    compare_s1(h, x, np.ones(5000), 1e-6)
    g = workloads.rng(14)
    xs = np.ldexp(g.uniform(1, 2, 3000), g.integers(-1074, -1000, 3000))  # subnormal
    ys = np.ldexp(g.uniform(1, 2, 3000), g.integers(900, 1000, 3000))
    compare_s1(h, xs, ys, 1e-9)
    xb = np.ones(100)
    xb[5] = np.nan
    r = h.qdot(dev(xb), dev(np.ones(100)), 1e-6, opt=S1)
    assert r["status"] == q.E_NONFINITE and np.isnan(r["value"])


def test_exact_so_independent_of_order_runs_and_launch_shape(h):
    x, y = workloads.log_uniform_pair(400000, 15)
    xd, yd = dev(x), dev(y)
    r0 = h.qdot(xd, yd, 1e-6, opt=S1)
    assert h.qdot(xd, yd, 1e-6, opt=S1)["value"] == r0["value"]
    pm = workloads.rng(16).permutation(len(x))
    assert h.qdot(dev(x[pm]), dev(y[pm]), 1e-6, opt=S1)["value"] == r0["value"]
    try:
        for ob, ou in ((1, 1), (4, 4), (16, 2), (8, 1)):
            h.set_tune(-1, 2, 1, 2, 2, ob, ou)
            cfg = (ob, ou)
            r = h.qdot(xd, yd, 1e-6, opt=S1)
            assert r["value"] == r0["value"] and r["count"] == r0["count"], cfg
    finally:
        h.reset_tune()


def test_same_classes_as_default_mode(h):
    x, y = workloads.log_uniform_pair(200000, 17)
    xd, yd = dev(x), dev(y)
    a = h.qdot(xd, yd, 1e-6)
    b = h.qdot(xd, yd, 1e-6, opt=S1)
    for k in ("count", "n_bins", "e_max", "e_min", "t", "flags", "bound_rel"):
        assert a[k] == b[k], k


def test_inadmissible_requests_are_rejected(h):
    x, y = workloads.log_uniform_pair(1000, 18)
    xd, yd = dev(x), dev(y)
    with pytest.raises(q.QdotError):
        h.qdot(xd, yd, 1e-80, opt=S1)  # kept bins could lie beyond the window
    with pytest.raises(q.QdotError):
        h.qdot_classes(xd, yd, 1e-6, opt=S1)
    # in a batch, only the instance whose tolerance is refused fails
    offs = np.array([0, 500, 1000], dtype=np.int64)
    res = h.batched(xd, yd, offs, [1e-6, 1e-80], opt=S1)
    assert res[0]["status"] == q.OK and res[1]["status"] == q.E_INVAL
    assert np.isnan(res[1]["value"])


def _ragged(seed, extra, count, hi=3e5):
    g = workloads.rng(seed)
    sizes = list(extra) + list(np.rint(10 ** g.uniform(0, np.log10(hi), count)).astype(int))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    x, y = workloads.log_uniform_pair(int(offsets[-1]), seed + 1)
    tols = np.array([1e-4, 1e-6, 1e-8, 1e-3, 1e-12])[g.integers(0, 5, len(sizes))]
    return offsets, x, y, tols


def _check_batched_s1(res, offsets, x, y, tols, opt=S1):
    for j in range(len(tols)):
        a, b = offsets[j], offsets[j + 1]
        o = oracle.qdot(x[a:b], y[a:b], tols[j], opt=opt)
        for k in INT_KEYS:
            assert res[j][k] == o[k], (j, b - a, k, res[j][k], o[k])
        if o["status"] == oracle.OK:
            scale = oracle.abs_dot(x[a:b], y[a:b])
            assert abs(res[j]["value"] - o["value"]) <= VALUE_TOL * scale, (j, b - a)
            for c in range(3):
                assert abs(res[j]["part"][c] - o["part"][c]) <= VALUE_TOL * scale, (j, c)


def test_batched_one_pass_matches_oracle(h):
    # instances above 131072 components go through one-pass chunks that
    # merge into a per-instance bin table; the rest are done by one block
    edge = (0, 1, 65, 1025, 65536, 131072, 131073, 300001, 700000)
    offsets, x, y, tols = _ragged(21, edge, 80)
    res = h.batched(dev(x), dev(y), offsets, tols, opt=S1)
    _check_batched_s1(res, offsets, x, y, tols)
    # repeat: the bin tables and counters were left clean, the sums are exact
    res2 = h.batched(dev(x), dev(y), offsets, tols, opt=S1)
    assert res2 == res


@pytest.mark.parametrize("opt", [[1, 0, 0, 1], [0, 1, 1, 1]])
def test_batched_one_pass_options(h, opt):
    offsets, x, y, tols = _ragged(22, (200000, 5000), 20)
    res = h.batched(dev(x), dev(y), offsets, tols, opt=opt)
    _check_batched_s1(res, offsets, x, y, tols, opt=opt)


def test_batched_one_pass_nonfinite_and_graph_replay(h):
    offsets, x, y, tols = _ragged(23, (250000, 3000), 15)
    xb = x.copy()
    xb[offsets[0] + 11] = np.inf
    xb[offsets[1] + 7] = np.nan
    res = h.batched(dev(xb), dev(y), offsets, tols, opt=S1)
    assert res[0]["status"] == q.E_NONFINITE and res[1]["status"] == q.E_NONFINITE
    # the state is clean for the next call, which is captured and replayed
    xd, yd = dev(x), dev(y)
    off_d = torch.from_numpy(offsets).to("cuda:0")
    tol_d = dev(tols)
    n_inst = len(tols)
    eager = torch.zeros(n_inst * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.batched_async(xd, yd, off_d, offsets, tol_d, eager, opt=S1)
    torch.cuda.synchronize()
    _check_batched_s1(q.parse_results(eager), offsets, x, y, tols)
    out = torch.zeros_like(eager)
    h.batch_plan(offsets, [], opt=S1)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            h.batched_async(xd, yd, off_d, offsets, tol_d, out, opt=S1)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        h.qdot(xd[:1000], yd[:1000], 1e-6, opt=S1)
        torch.cuda.synchronize()


