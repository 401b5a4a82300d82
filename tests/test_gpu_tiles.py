"""GPU tests of tile skipping (tile_skip 1): pass 1 records the largest key
slot of every 64-component tile and pass 2 reads no operand of a tile that
lies wholly below the lowest kept bin.  The results, classes and histogram
must be bit for bit those of the default path (tile_skip 0) on every input,
and the default path's integer outputs and value are checked against the
oracle on the new banded inputs (the Sec. 4.2 pattern of whole index ranges
in the perforated class).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import workloads
from parity_util import INT_KEYS, VALUE_TOL

torch = pytest.importorskip("torch")
import paper_2105_00115_amd as q  # noqa: E402

pytestmark = pytest.mark.gpu

TS = [0, 0, 0, 0, 0, 0, 0, 1]


@pytest.fixture(scope="module")
def h():
    handle = q.Qdot(0)
    yield handle
    handle.close()


def dev(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


def with_ts(opt):
    o = list(opt or [0] * 7)
    o += [0] * (7 - len(o))
    return o[:7] + [1]


def same(a: dict, b: dict):
    for k in a:
        va, vb = a[k], b[k]
        if isinstance(va, float) and math.isnan(va):
            assert math.isnan(vb), k
        else:
            assert va == vb, (k, va, vb)


def check(h, x, y, tol, opt=None, f32=False, oracle_check=True):
    """tile_skip 1 against tile_skip 0 (bit for bit, both the plain and the
    classes entry point), and tile_skip 0 against the oracle."""
    print(f"[gpu-case] tiles n={len(x)} tol={tol} opt={opt} f32={f32}", flush=True)
    dt = np.float32 if f32 else np.float64
    xd, yd = dev(x, dt), dev(y, dt)
    plain = h.qdot_f32 if f32 else h.qdot
    classes = h.qdot_f32_classes if f32 else h.qdot_classes
    r0 = plain(xd, yd, tol, opt=opt)
    r1 = plain(xd, yd, tol, opt=with_ts(opt))
    same(r1, r0)
    c0, h0, s0 = classes(xd, yd, tol, opt=opt)
    c1, h1, s1 = classes(xd, yd, tol, opt=with_ts(opt))
    same(s1, s0)
    assert torch.equal(c1, c0) and torch.equal(h1, h0)
    if oracle_check:
        xs, ys = np.asarray(x, dtype=dt), np.asarray(y, dtype=dt)
        o = (oracle.qdot_f32 if f32 else oracle.qdot)(xs, ys, tol, opt=opt, want_classes=True,
                                                        want_hist=True)
        for k in INT_KEYS:
            assert r0[k] == o[k], (k, r0[k], o[k])
        np.testing.assert_array_equal(c0.cpu().numpy()[:len(x)], o["classes"])
        np.testing.assert_array_equal(h0.cpu().numpy(), o["hist"])
        if o["status"] == oracle.OK:
            scale = oracle.abs_dot(np.float64(xs), np.float64(ys))
            assert abs(r0["value"] - o["value"]) <= VALUE_TOL * scale
    return r0


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10])
@pytest.mark.parametrize("seed", [71, 72])
def test_banded_inputs(h, tol, seed):
    x, y = workloads.banded_pair(200003, seed)
    r = check(h, x, y, tol)
    assert r["count"][q.PERF] > 0


@pytest.mark.parametrize("tol", [1e-3, 1e-6])
def test_log_uniform_inputs(h, tol):
    x, y = workloads.log_uniform_pair(300007, 73)
    check(h, x, y, tol)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1023, 1025, 4097, 65536 + 17])
def test_tile_boundaries(h, n):
    x, y = workloads.banded_pair(n, 74 + n % 7, mean_band=40.0)
    check(h, x, y, 1e-6)


def test_options_and_bins(h):
    x, y = workloads.banded_pair(150001, 75)
    for opt in ([1, 0, 0, 0], [0, 1, 1, 0], [0, 0, 0, 0, 0, 1, 3], [0, 0, 0, 0, 0, 2, 9]):
        check(h, x, y, 1e-6, opt=opt)


def test_single_precision_inputs(h):
    x, y = workloads.banded_pair(150001, 76, levels=(0, -8, -20, -40))
    for tol in (1e-2, 1e-5):
        check(h, x, y, tol, f32=True)


def test_edge_inputs(h):
    z = np.zeros(5000)
    check(h, z, z, 1e-6)
    o = np.ones(70001)
    check(h, o, o, 1e-6)
    # everything perforated but the top bin, and a huge tolerance
    x, y = workloads.banded_pair(100000, 77, levels=(0, -200))
    check(h, x, y, 1e-1)
    check(h, x, y, 1e3)
    # a non-finite product: same status and classes either way
    x, y = workloads.banded_pair(20000, 78)
    x[12345] = np.inf
    check(h, x, y, 1e-6, oracle_check=False)
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    r = h.qdot(e[:0], e[:0], 1e-6, opt=TS)
    assert r["status"] == q.OK and r["flags"] & q.F_ALL_PERF


def test_cg_residuals(h):
    # r = b - A x_k of CG on the 2D Poisson matrix with b = A 1 (a smooth
    # right-hand side), after a few iterations: the residual's products
    # decay away from the boundary, so whole tiles are perforated
    m = 256
    rp, col, val = workloads.poisson2d_csr(m)
    A = q.Csr(rp, col, val)
    ones = torch.ones(m * m, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(ones)
    h.spmv(A, ones, b)
    for k in (5, 40):
        x = torch.zeros_like(b)
        h.cg(A, b, x, 1e-30, 1e-8, k, 0)
        ax = torch.empty_like(b)
        h.spmv(A, x, ax)
        r = (b - ax).cpu().numpy()
        check(h, r, r, 1e-8)


def test_tile_keys_grow_and_shrink(h):
    for n in (1000, 300001, 5000, 300001):
        x, y = workloads.banded_pair(n, 79)
        check(h, x, y, 1e-6, oracle_check=False)


def test_graph_replay(h):
    x, y = workloads.banded_pair(300001, 80)
    xd, yd = dev(x), dev(y)
    eager = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    h.qdot_async(xd, yd, 1e-6, eager, opt=TS)  # grows the tile keys outside capture
    torch.cuda.synchronize()
    out = torch.zeros_like(eager)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            h.qdot_async(xd, yd, 1e-6, out, opt=TS)
    torch.cuda.synchronize()
    for rep in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        h.qdot(xd[:7000], yd[:7000], 1e-3, opt=TS)  # eager work on the same handle
        torch.cuda.synchronize()
    r = q.parse_results(eager)[0]
    same(r, h.qdot(xd, yd, 1e-6))


def test_refused_where_not_supported(h):
    x = dev(np.ones(1000))
    for opt in ([0, 0, 0, 1, 0, 0, 0, 1], [0, 0, 0, 0, 1, 0, 0, 1], [0, 0, 0, 0, 0, 0, 0, 2]):
        with pytest.raises(q.QdotError):
            h.qdot(x, x, 1e-6, opt=opt)
    out = torch.zeros(q.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(q.QdotError):
        q.qdot_noalloc_async(x, x, 1e-6, out, opt=TS)
    rp, col, val = workloads.poisson2d_csr(16)
    A = q.Csr(rp, col, val)
    b = dev(workloads.normal_vector(256, 1))
    with pytest.raises(q.QdotError):
        h.cg(A, b, torch.zeros(256, dtype=torch.float64, device="cuda:0"), 1e-10, 1e-8, 100, 1,
             opt=TS)
    with pytest.raises(q.QdotError):
        h.power(A, dev(workloads.unit_vector(256, 2)), 5, 1e-6, 1, opt=TS)


def test_perforated_tiles_are_not_read(h):
    # three quarters of the bands far below the top ones: pass 2 with the
    # tile keys must take clearly less time than without (it reads about a
    # quarter of the operands)
    n = 1 << 25
    x, y = workloads.banded_pair(n, 81, levels=(0, -300, -300, -300), mean_band=20000.0)
    xd, yd = dev(x), dev(y)
    ms = {}
    for name, opt in (("default", None), ("tiles", TS)):
        h.qdot(xd, yd, 1e-6, opt=opt)
        h.timing_read()
        h.timing_enable(True)
        for _ in range(5):
            h.qdot(xd, yd, 1e-6, opt=opt)
        t = h.timing_read()
        h.timing_enable(False)
        ms[name] = t["acc_ms"] / t["qdot_calls"]
    print(f"[gpu-case] accumulate pass ms: {ms}", flush=True)
    assert ms["tiles"] < 0.75 * ms["default"], ms
