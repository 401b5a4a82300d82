"""GPU parity of the batched ragged qdot (one persistent launch).

Every instance must give what the oracle gives for that instance alone:
integer outputs bit for bit, the value within 1e-13 * sum |x_i y_i| of the
instance.  The launch must be repeatable (bitwise), must isolate bad
instances, and must replay correctly from a captured HIP graph.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
import parity_util
from parity_util import host

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu
VALUE_TOL = 1e-13
INT_KEYS = ("count", "n_zero", "e_min", "e_max", "n_bins", "t", "flags", "status")


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def ragged_case(seed, extra_sizes=(), count=120, hi=3e5):
    g = workloads.rng(seed)
    sizes = list(extra_sizes) + list(np.rint(10 ** g.uniform(0, np.log10(hi), count)).astype(int))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    x, y = workloads.log_uniform_pair(int(offsets[-1]), seed + 1)
    tols = np.array([1e-4, 1e-6, 1e-8, 1e-3, 1e2])[g.integers(0, 5, len(sizes))]
    return offsets, x, y, tols


def check_instances(res, offsets, x, y, tols, which=None, opt=None):
    idx = range(len(tols)) if which is None else which
    for j in idx:
        a, b = offsets[j], offsets[j + 1]
        o = oracle.qdot(x[a:b], y[a:b], tols[j], opt=opt)
        r = res[j]
        for k in INT_KEYS:
            assert r[k] == o[k], (j, b - a, k, r[k], o[k])
        if o["status"] != oracle.OK:
            continue
        scale = oracle.abs_dot(x[a:b], y[a:b])
        assert abs(r["value"] - o["value"]) <= VALUE_TOL * scale, (j, r["value"], o["value"])
        assert abs(r["bound_rel"] - o["bound_rel"]) <= 1e-12 * abs(o["bound_rel"]), j


EDGE = (0, 1, 3, 63, 64, 65, 1023, 1024, 1025, 32768, 32769, 65536, 65537, 98309,
        131072, 200003)


def test_batched_matches_oracle(h):
    offsets, x, y, tols = ragged_case(1, EDGE)
    res = h.batched(dev(x), dev(y), offsets, tols)
    check_instances(res, offsets, x, y, tols)


@pytest.mark.parametrize("opt", [[1, 0, 0, 0], [0, 1, 1, 0]])
def test_batched_options(h, opt):
    offsets, x, y, tols = ragged_case(2, (70000, 5000), count=30)
    res = h.batched(dev(x), dev(y), offsets, tols, opt=opt)
    check_instances(res, offsets, x, y, tols, opt=opt)


def test_batched_equals_standalone_and_repeats(h):
    offsets, x, y, tols = ragged_case(3, (150000, 70001, 4096), count=40)
    xd, yd = dev(x), dev(y)
    r1 = h.batched(xd, yd, offsets, tols)
    r2 = h.batched(xd, yd, offsets, tols)
    for a, b in zip(r1, r2):  # second launch runs on the reset state
        assert a == b
    for j in range(0, len(tols), 3):
        a, b = offsets[j], offsets[j + 1]
        s = h.qdot(xd[a:b], yd[a:b], tols[j])
        for k in INT_KEYS:
            assert s[k] == r1[j][k], (j, k)
        scale = oracle.abs_dot(x[a:b], y[a:b])
        assert abs(s["value"] - r1[j]["value"]) <= VALUE_TOL * scale


def test_batched_isolates_bad_instances(h):
    offsets, x, y, tols = ragged_case(4, (80000, 3000, 90000, 500), count=10)
    xb = x.copy()
    xb[offsets[0] + 17] = np.nan       # large instance 0: non-finite
    xb[offsets[1] + 5] = np.inf        # small instance 1: non-finite
    tb = tols.copy()
    tb[2] = 0.0                        # large instance 2: bad tolerance
    tb[3] = np.nan                     # small instance 3: bad tolerance
    res = h.batched(dev(xb), dev(y), offsets, tb)
    assert res[0]["status"] == q.E_NONFINITE and np.isnan(res[0]["value"])
    assert res[1]["status"] == q.E_NONFINITE
    assert res[2]["status"] == q.E_INVAL and res[3]["status"] == q.E_INVAL
    check_instances(res, offsets, xb, y, tb, which=range(4, len(tb)))
    # the state is clean for the next call
    res2 = h.batched(dev(x), dev(y), offsets, tols)
    check_instances(res2, offsets, x, y, tols)


def test_batched_zeros_and_subnormals(h):
    g = workloads.rng(5)
    sizes = [70000, 70000, 1000, 1000]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x, y = workloads.log_uniform_pair(int(offsets[-1]), 6)
    x[: offsets[1]] = 0.0                                    # all-zero instance
    x[offsets[1]: offsets[2]: 3] = 0.0
    x[offsets[2]: offsets[3]] = np.ldexp(g.uniform(1, 2, 1000), g.integers(-1074, -1000, 1000))
    y[offsets[2]: offsets[3]] = np.ldexp(g.uniform(1, 2, 1000), g.integers(900, 1000, 1000))
    tols = np.array([1e-6, 1e-6, 1e-9, 1e300])
    res = h.batched(dev(x), dev(y), offsets, tols)
    check_instances(res, offsets, x, y, tols)
    assert res[0]["flags"] & q.F_ALL_PERF and res[3]["value"] == 0.0


def test_batched_graph_replay(h):
    offsets, x, y, tols = ragged_case(7, (100000, 40000), count=25)
    xd, yd = dev(x), dev(y)
    off_d = torch.from_numpy(offsets).to("cuda:0")
    tol_d = dev(tols)
    B = len(tols)
    eager = torch.zeros(B * q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.batched_async(xd, yd, off_d, offsets, tol_d, eager)
    torch.cuda.synchronize()
    out = torch.zeros_like(eager)
    h.batched_plan(offsets)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            h.batched_async(xd, yd, off_d, offsets, tol_d, out)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        # eager work on the same handle between replays
        h.qdot(xd[:1000], yd[:1000], 1e-6)
        torch.cuda.synchronize()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("accum", [0, 1])
def test_batched_c5_full_size(h, accum):
    """4096 instances, lengths round(10^U[2,6]) (about 4.45e8 components in
    all), tolerances from {1e-4, 1e-6, 1e-8}: the launch the batched
    benchmark times, in both readings of the accumulation.  Every instance
    against the oracle on that instance alone."""
    g = workloads.rng(2025)
    sizes = np.rint(10.0 ** g.uniform(2, 6, 4096)).astype(np.int64)
    offsets = np.zeros(4097, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    tols = np.array([1e-4, 1e-6, 1e-8])[g.integers(0, 3, 4096)]
    total = int(offsets[-1])
    opt = [0, 0, 0, accum]
    print(f"[gpu-case] batched C5 total={total} accum_mode={accum}", flush=True)
    xd, yd = workloads.log_uniform_pair_torch(total, 2025, "cuda:0")
    res = h.batched(xd, yd, offsets, tols, opt=opt)
    xh, yh = host(xd), host(yd)
    del xd, yd
    assert parity_util.check_instances(res, offsets, xh, yh, tols, opt=opt) == 4096
    assert sum(sum(r["count"]) for r in res) == total


@pytest.mark.parametrize("shape", [(2, 65536), (8, 262144), (4, 8192)])
def test_batched_under_other_batch_shapes(shape):
    # blocks per CU and chunk size move work between blocks and items but
    # never a tile or a class: every instance still equals the oracle's
    bpc, chunk = shape
    with q.Qdot(0, load_tuned=False) as hh:
        hh.set_solver_tune(batch_blocks_per_cu=bpc, batch_chunk=chunk)
        assert hh.get_solver_tune()[:2] == (bpc, chunk)
        offsets, x, y, tols = ragged_case(31, EDGE + (300000,), count=40)
        for opt in (None, [0, 0, 0, 1]):
            res = hh.batched(dev(x), dev(y), offsets, tols, opt=opt)
            check_instances(res, offsets, x, y, tols, opt=opt)
        hh.set_solver_tune()
        assert hh.get_solver_tune() == (4, 131072, 16384, 16, 8, 2, 0)
        with pytest.raises(q.QdotError):
            hh.set_solver_tune(batch_chunk=1000)  # not a multiple of 2048
        with pytest.raises(q.QdotError):
            hh.set_solver_tune(cg_gang_max=513)
        with pytest.raises(q.QdotError):
            hh.set_solver_tune(cg_blocks_per_cu=3)
